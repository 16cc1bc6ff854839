// Tall-skinny Householder QR (TSQR) in FP64.
//
// The m x n matrix is cut into row blocks that each fit in LDS; every block
// is factored by unblocked Householder reflections (one workgroup, the block
// held column-major in LDS so that column sweeps are unit stride).  The n x n
// R factors of the blocks are stacked and factored again, level by level,
// until one block remains.  The explicit Q is then formed top-down: each
// block applies its reflectors to its n x k slice of the Q of the level
// above, padded with zeros.  Reflectors follow the usual convention
// H = I - tau v v^T, v(0) = 1, beta = -sign(x0) ||x||; a zero column gives
// tau = 0 (H = I), so rank-deficient inputs still produce orthonormal Q.
// Finally the signs of diag(R) are made non-negative (columns of Q and rows
// of R flipped together), which fixes the factorization uniquely for
// full-rank input.
#include "common.h"

namespace hatt {

constexpr int kQrChunk = 8;  // Q columns formed per LDS pass

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

static int64_t qr_block_rows_max(int64_t n) { return kQrLdsDoubles / (n + kQrChunk); }

bool qr_make_plan(int64_t m, int64_t n, QrPlan *p) {
  if (m < 1 || n < 1 || n > kQrMaxCols) return false;
  QrPlan q{};
  q.m = m;
  q.n = n;
  q.k = std::min(m, n);
  const int64_t mb = qr_block_rows_max(n);
  int64_t rows = m;
  int64_t off = 0;
  int L = 0;
  while (true) {
    if (L >= kQrMaxLevels) return false;
    int64_t blocks;
    if (rows <= mb) blocks = 1;
    else blocks = std::max<int64_t>(1, std::min((rows + mb - 1) / mb, rows / n));
    if (blocks > 1 && (rows + blocks - 1) / blocks > mb) return false;
    q.rows[L] = rows;
    q.blocks[L] = blocks;
    if (L > 0) {
      q.off_stack[L] = off;
      off += rows * n;
    } else {
      q.off_stack[L] = -1;
    }
    q.off_v[L] = off;
    off += rows * n;
    q.off_tau[L] = off;
    off += blocks * n;
    ++L;
    if (blocks == 1) break;
    rows = blocks * n;
  }
  q.levels = L;
  q.off_rtop = off;
  off += q.k * n;
  q.ws_doubles = off;
  *p = q;
  return true;
}

struct QrLevelArgs {
  CMat src;        // matrix factored at this level (level 0: the input)
  int64_t rows, blocks, n;
  double *ws;      // workspace base of pair 0
  int64_t wsp;     // workspace stride between pairs
  int64_t off_v, off_tau;
  int64_t off_rout;  // where the stacked R factors (or the final R) go
  int64_t ld_rout;   // row stride of that buffer
};

__global__ __launch_bounds__(256) void tsqr_factor_kernel(QrLevelArgs a) {
  extern __shared__ double A[];  // column-major block: A[c * nr + r]
  __shared__ double red[4];
  __shared__ double s_tau, s_scal;
  __shared__ double bet[kQrMaxCols];
  __shared__ double taus[kQrMaxCols];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t blk = blockIdx.x;
  const int p = blockIdx.y;
  const int64_t r0 = blk * a.rows / a.blocks, r1 = (blk + 1) * a.rows / a.blocks;
  const int nr = (int)(r1 - r0);
  const int n = (int)a.n;
  const double *src = a.src.ptr + p * a.src.bs;
  if (a.src.cs == 1) {
    for (int e = tid; e < nr * n; e += 256) {
      int r = e / n, c = e - r * n;
      A[c * nr + r] = src[(r0 + r) * a.src.rs + c];
    }
  } else {
    for (int e = tid; e < nr * n; e += 256) {
      int c = e / nr, r = e - c * nr;
      A[c * nr + r] = src[(r0 + r) * a.src.rs + c * a.src.cs];
    }
  }
  __syncthreads();
  const int kref = min(nr, n);
  for (int j = 0; j < kref; ++j) {
    double part = 0.0;
    for (int r = j + 1 + tid; r < nr; r += 256) {
      double v = A[j * nr + r];
      part += v * v;
    }
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    if (tid == 0) {
      const double sigma2 = red[0] + red[1] + red[2] + red[3];
      const double x0 = A[j * nr + j];
      double tau = 0.0, scal = 0.0, beta = x0;
      if (sigma2 > 0.0) {
        const double nrm = sqrt(x0 * x0 + sigma2);
        beta = (x0 >= 0.0) ? -nrm : nrm;
        tau = (beta - x0) / beta;
        scal = 1.0 / (x0 - beta);
      }
      s_tau = tau;
      s_scal = scal;
      bet[j] = beta;
      taus[j] = tau;
    }
    __syncthreads();
    const double scal = s_scal, tau = s_tau;
    for (int r = j + 1 + tid; r < nr; r += 256) A[j * nr + r] *= scal;
    __syncthreads();
    if (tau != 0.0) {
      for (int c = j + 1 + wave; c < n; c += 4) {
        double pw = 0.0;
        for (int r = j + 1 + lane; r < nr; r += 64) pw += A[j * nr + r] * A[c * nr + r];
        double w = (wave_sum(pw) + A[c * nr + j]) * tau;
        for (int r = j + 1 + lane; r < nr; r += 64) A[c * nr + r] -= A[j * nr + r] * w;
        if (lane == 0) A[c * nr + j] -= w;
      }
    }
    __syncthreads();
  }
  // reflectors (column-major block, contiguous per block) and taus
  double *ws = a.ws + p * a.wsp;
  double *vout = ws + a.off_v + r0 * n;
  for (int e = tid; e < nr * n; e += 256) vout[e] = A[e];
  for (int j = tid; j < n; j += 256) ws[a.off_tau + blk * n + j] = (j < kref) ? taus[j] : 0.0;
  // R rows of this block (kref x n, upper trapezoidal)
  double *rout = ws + a.off_rout + blk * (int64_t)kref * a.ld_rout;
  for (int e = tid; e < kref * n; e += 256) {
    int jj = e / n, c = e - jj * n;
    double v = 0.0;
    if (c > jj) v = A[c * nr + jj];
    else if (c == jj) v = bet[jj];
    rout[jj * a.ld_rout + c] = v;
  }
}

struct QrFormArgs {
  int64_t rows, blocks, n, k;
  double *ws;
  int64_t wsp;
  int64_t off_v, off_tau;
  int top;            // 1: the seed is diag(sign(diag R)) from the final R
  int64_t off_rtop;   // final R (k x n, row stride n)
  int64_t off_cin;    // level above's explicit Q (rows_{L+1} x k, row stride k)
  Mat dst;            // this level's explicit Q (rows x k)
  Mat rdst;           // final R destination (top level only, may be null)
};

__global__ __launch_bounds__(256) void tsqr_formq_kernel(QrFormArgs a) {
  extern __shared__ double sm[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t blk = blockIdx.x;
  const int p = blockIdx.y;
  const int64_t r0 = blk * a.rows / a.blocks, r1 = (blk + 1) * a.rows / a.blocks;
  const int nr = (int)(r1 - r0);
  const int n = (int)a.n, k = (int)a.k;
  const int kref = min(nr, n);
  double *Vs = sm;                  // nr x n column-major
  double *X = Vs + nr * n;          // nr x kQrChunk column-major
  __shared__ double taus[kQrMaxCols];
  __shared__ double sgn[kQrMaxCols];
  double *ws = a.ws + p * a.wsp;
  const double *vin = ws + a.off_v + r0 * n;
  for (int e = tid; e < nr * n; e += 256) Vs[e] = vin[e];
  for (int j = tid; j < n; j += 256) taus[j] = ws[a.off_tau + blk * n + j];
  if (a.top) {
    const double *rt = ws + a.off_rtop;
    for (int j = tid; j < k; j += 256) sgn[j] = (rt[j * n + j] < 0.0) ? -1.0 : 1.0;
  }
  __syncthreads();
  const double *cin = a.top ? nullptr : ws + a.off_cin + blk * (int64_t)n * k;
  double *dst = a.dst.ptr + p * a.dst.bs;
  for (int c0 = 0; c0 < k; c0 += kQrChunk) {
    const int cw = min(kQrChunk, k - c0);
    for (int e = tid; e < nr * cw; e += 256) {
      int cc = e / nr, r = e - cc * nr;
      double v = 0.0;
      if (r < kref) {
        if (a.top) v = (r == c0 + cc) ? sgn[r] : 0.0;
        else v = cin[r * k + c0 + cc];
      }
      X[cc * nr + r] = v;
    }
    __syncthreads();
    for (int cc = wave; cc < cw; cc += 4) {
      double *x = X + cc * nr;
      for (int j = kref - 1; j >= 0; --j) {
        const double tau = taus[j];
        if (tau == 0.0) continue;
        const double *v = Vs + j * nr;
        double pw = 0.0;
        for (int r = j + 1 + lane; r < nr; r += 64) pw += v[r] * x[r];
        const double w = (wave_sum(pw) + x[j]) * tau;
        for (int r = j + 1 + lane; r < nr; r += 64) x[r] -= v[r] * w;
        if (lane == 0) x[j] -= w;
      }
    }
    __syncthreads();
    for (int e = tid; e < nr * cw; e += 256) {
      int r = e / cw, cc = e - r * cw;
      dst[(r0 + r) * a.dst.rs + (c0 + cc) * a.dst.cs] = X[cc * nr + r];
    }
    __syncthreads();
  }
  if (a.top && a.rdst.ptr != nullptr && blk == 0) {
    const double *rt = ws + a.off_rtop;
    double *rd = a.rdst.ptr + p * a.rdst.bs;
    for (int e = tid; e < k * n; e += 256) {
      int j = e / n, c = e - j * n;
      rd[j * a.rdst.rs + c * a.rdst.cs] = sgn[j] * rt[j * n + c];
    }
  }
}

hipError_t launch_tsqr(const QrPlan &p, CMat a, Mat q, Mat r, double *ws, int64_t wsp, int batch,
                       hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const int64_t n = p.n;
  const int64_t mb = qr_block_rows_max(n);
  // upward pass
  for (int L = 0; L < p.levels; ++L) {
    QrLevelArgs la{};
    if (L == 0) la.src = a;
    else la.src = CMat{ws + p.off_stack[L], n, 1, wsp};
    la.rows = p.rows[L];
    la.blocks = p.blocks[L];
    la.n = n;
    la.ws = ws;
    la.wsp = wsp;
    la.off_v = p.off_v[L];
    la.off_tau = p.off_tau[L];
    la.off_rout = (L + 1 < p.levels) ? p.off_stack[L + 1] : p.off_rtop;
    la.ld_rout = n;
    const int64_t nrmax = (la.rows + la.blocks - 1) / la.blocks;
    const size_t lds = (size_t)nrmax * n * sizeof(double);
    hipFuncSetAttribute((const void *)tsqr_factor_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)(mb * (n + kQrChunk) * sizeof(double)));
    tsqr_factor_kernel<<<dim3((unsigned)la.blocks, (unsigned)batch), 256, lds, s>>>(la);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // downward pass
  for (int L = p.levels - 1; L >= 0; --L) {
    QrFormArgs fa{};
    fa.rows = p.rows[L];
    fa.blocks = p.blocks[L];
    fa.n = n;
    fa.k = p.k;
    fa.ws = ws;
    fa.wsp = wsp;
    fa.off_v = p.off_v[L];
    fa.off_tau = p.off_tau[L];
    fa.top = (L == p.levels - 1);
    fa.off_rtop = p.off_rtop;
    fa.off_cin = fa.top ? 0 : p.off_stack[L + 1];
    if (L == 0) fa.dst = q;
    else fa.dst = Mat{ws + p.off_stack[L], p.k, 1, wsp};
    fa.rdst = fa.top ? r : Mat{nullptr, 0, 0, 0};
    const int64_t nrmax = (fa.rows + fa.blocks - 1) / fa.blocks;
    const size_t lds = (size_t)nrmax * (n + kQrChunk) * sizeof(double);
    hipFuncSetAttribute((const void *)tsqr_formq_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)(mb * (n + kQrChunk) * sizeof(double)));
    tsqr_formq_kernel<<<dim3((unsigned)fa.blocks, (unsigned)batch), 256, lds, s>>>(fa);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace hatt
