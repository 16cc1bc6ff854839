// Tall-skinny Householder QR (TSQR) in FP64.
//
// The m x n matrix is cut into row blocks that each fit in LDS; every block
// is factored by unblocked Householder reflections in one workgroup, the
// block held column-major in LDS (odd leading dimension, so that lanes that
// walk down one column touch distinct banks).  The k x n R factors of the
// blocks are stacked and factored again, level by level, until one block
// remains.  The explicit Q is then formed top-down: each block applies its
// reflectors, last to first, to its slice of the Q of the level above padded
// with zeros.
//
// Inner products never go through cross-lane shuffles: for a reflector step
// the (column, row-group) products are spread over all 256 threads, written
// as partial sums to LDS and summed by one thread per column after a
// barrier.  With v = A(j:, j) / (x0 - beta), the products needed by a step,
// D_c = sum_{r>j} A(r, j) A(r, c), are all available before the reflector is
// known, so one pass gives both ||A(j+1:, j)||^2 (c = j) and the trailing
// projections.  Reflector convention: H = I - tau v v^T, v(j) = 1,
// beta = -sign(x0) ||x||; a zero column gives tau = 0 (H = I), so
// rank-deficient input still yields an orthonormal Q.  Finally the signs of
// diag(R) are made non-negative (columns of Q and rows of R flipped
// together).
#include <mutex>
#include "common.h"
#include "stage.h"

namespace hatt {

// Column chunk width the Q-forming kernel keeps in LDS next to the
// reflectors, for an m x n matrix: the largest that lets a block hold 2n
// rows (the tree then shrinks), else n rows.  A matrix of fewer than 2n rows
// cannot be cut into blocks of n rows, so there one block must hold all m.
static int qr_chunk(int64_t m, int64_t n, int64_t k) {
  const int cand[6] = {(int)std::min<int64_t>(k, 64), 32, 16, 8, 4, 1};
  const int64_t need[2] = {m < 2 * n ? m : 2 * n, m < 2 * n ? m : n};
  for (int t = 0; t < 2; ++t) {
    for (int i = 0; i < 6; ++i) {
      const int ch = std::max(1, std::min<int>(cand[i], (int)k));
      const int64_t mb = kQrLdsDoubles / (n + ch) - 1;
      if (mb >= need[t]) return ch;
    }
  }
  return 1;
}

static int64_t qr_block_rows_max(int64_t m, int64_t n, int64_t k) {
  return kQrLdsDoubles / (n + qr_chunk(m, n, k)) - 1;
}

bool qr_make_plan(int64_t m, int64_t n, QrPlan *p) {
  if (m < 1 || n < 1 || n > kQrMaxCols) return false;
  QrPlan q{};
  q.m = m;
  q.n = n;
  q.k = std::min(m, n);
  const int64_t mb = qr_block_rows_max(m, n, q.k);
  if (mb < std::min(m, n)) return false;
  int64_t rows = m;
  int64_t off = 0;
  int L = 0;
  while (true) {
    if (L >= kQrMaxLevels) return false;
    int64_t blocks;
    if (rows <= mb) blocks = 1;
    else blocks = std::max<int64_t>(1, std::min((rows + mb - 1) / mb, rows / n));
    if ((rows + blocks - 1) / blocks > mb) return false;  // a block must fit in LDS
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
    if (blocks * n >= rows) return false;  // a level that does not shrink: use panels instead
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
  const int *skip;   // optional: pairs with skip[p * skip_stride] == 1 are left untouched
  int64_t skip_stride;
};

__global__ __launch_bounds__(256) void tsqr_factor_kernel(QrLevelArgs a) {
  if (a.skip != nullptr && a.skip[blockIdx.y * a.skip_stride] == 1) return;
  extern __shared__ double A[];  // column-major block: A[c * ld + r]
  __shared__ double part[256];
  __shared__ double Ds[kQrMaxCols];
  __shared__ double Ws[kQrMaxCols];
  __shared__ double bet[kQrMaxCols];
  __shared__ double taus[kQrMaxCols];
  __shared__ double scals[kQrMaxCols];
  const int tid = threadIdx.x;
  const int64_t blk = blockIdx.x;
  const int p = blockIdx.y;
  const int64_t r0 = blk * a.rows / a.blocks, r1 = (blk + 1) * a.rows / a.blocks;
  const int nr = (int)(r1 - r0);
  const int ld = nr | 1;
  const int n = (int)a.n;
  const double *src = a.src.ptr + p * a.src.bs;
  if (a.src.cs == 1) {
    for (int e = tid; e < nr * n; e += 256) {
      int r = e / n, c = e - r * n;
      A[c * ld + r] = src[(r0 + r) * a.src.rs + c];
    }
  } else {
    for (int e = tid; e < nr * n; e += 256) {
      int c = e / nr, r = e - c * nr;
      A[c * ld + r] = src[(r0 + r) * a.src.rs + c * a.src.cs];
    }
  }
  __syncthreads();
  const int kref = min(nr, n);
  for (int j = 0; j < kref; ++j) {
    const int nc = n - j;           // columns j..n-1
    const int nrow = nr - j - 1;    // rows j+1..nr-1
    const int NG = max(1, 256 / nc);
    // pass 1: partial products D_c over row groups; deferred scaling of column j-1
    if (tid < nc * NG) {
      const int rg = tid % NG, c = j + tid / NG;
      const double *aj = A + j * ld, *ac = A + c * ld;
      double s = 0.0;
      for (int r = j + 1 + rg; r < nr; r += NG) s += aj[r] * ac[r];
      part[tid] = s;
    }
    if (j > 0) {
      const double sc = scals[j - 1];
      double *ap = A + (j - 1) * ld;
      for (int r = j + tid; r < nr; r += 256) ap[r] *= sc;
    }
    __syncthreads();
    if (tid < nc) {
      double s = 0.0;
      for (int g = 0; g < NG; ++g) s += part[tid * NG + g];
      Ds[j + tid] = s;
      if (tid == 0) {
        const double sigma2 = s;
        const double x0 = A[j * ld + j];
        double tau = 0.0, scal = 0.0, beta = x0;
        if (sigma2 > 0.0) {
          const double nrm = sqrt(x0 * x0 + sigma2);
          beta = (x0 >= 0.0) ? -nrm : nrm;
          tau = (beta - x0) / beta;
          scal = 1.0 / (x0 - beta);
        }
        bet[j] = beta;
        taus[j] = tau;
        scals[j] = scal;
      }
    }
    __syncthreads();
    const double tau = taus[j], scal = scals[j];
    if (tau != 0.0) {
      if (tid < nc - 1) {
        const int c = j + 1 + tid;
        Ws[c] = tau * (A[c * ld + j] + scal * Ds[c]);
      }
      __syncthreads();
      // pass 2: trailing update of rows j..nr-1 in columns j+1..n-1; a wave
      // walks 64 consecutive rows of one column, the 4 waves take every 4th column
      const double *aj = A + j * ld;
      const int lane = tid & 63, wv = tid >> 6;
      for (int c = j + 1 + wv; c < n; c += 4) {
        const double w = Ws[c];
        const double sw = scal * w;
        double *ac = A + c * ld;
        for (int r = j + 1 + lane; r < nr; r += 64) ac[r] -= aj[r] * sw;
        if (lane == 0) ac[j] -= w;
      }
    }
    __syncthreads();
  }
  if (kref > 0) {
    const double sc = scals[kref - 1];
    double *ap = A + (kref - 1) * ld;
    for (int r = kref + tid; r < nr; r += 256) ap[r] *= sc;
  }
  __syncthreads();
  // reflectors (column-major, leading dimension nr, contiguous per block) and taus
  double *ws = a.ws + p * a.wsp;
  double *vout = ws + a.off_v + r0 * n;
  for (int e = tid; e < nr * n; e += 256) {
    int c = e / nr, r = e - c * nr;
    vout[e] = A[c * ld + r];
  }
  for (int j = tid; j < n; j += 256) ws[a.off_tau + blk * n + j] = (j < kref) ? taus[j] : 0.0;
  // R rows of this block (kref x n, upper trapezoidal)
  double *rout = ws + a.off_rout + blk * (int64_t)kref * a.ld_rout;
  for (int e = tid; e < kref * n; e += 256) {
    int jj = e / n, c = e - jj * n;
    double v = 0.0;
    if (c > jj) v = A[c * ld + jj];
    else if (c == jj) v = bet[jj];
    rout[jj * a.ld_rout + c] = v;
  }
}

struct QrFormArgs {
  int64_t rows, blocks, n, k;
  int chunk;
  double *ws;
  int64_t wsp;
  int64_t off_v, off_tau;
  int top;            // 1: the seed is diag(sign(diag R)) from the final R
  int64_t off_rtop;   // final R (k x n, row stride n)
  int64_t off_cin;    // level above's explicit Q (rows_{L+1} x k, row stride k)
  Mat dst;            // this level's explicit Q (rows x k)
  Mat rdst;           // final R destination (top level only, may be null)
  const int *skip;
  int64_t skip_stride;
};

__global__ __launch_bounds__(256) void tsqr_formq_kernel(QrFormArgs a) {
  if (a.skip != nullptr && a.skip[blockIdx.y * a.skip_stride] == 1) return;
  extern __shared__ double sm[];
  __shared__ double part[256];
  __shared__ double Ws[kQrMaxCols];
  __shared__ double taus[kQrMaxCols];
  __shared__ double sgn[kQrMaxCols];
  const int tid = threadIdx.x;
  const int64_t blk = blockIdx.x;
  const int p = blockIdx.y;
  const int64_t r0 = blk * a.rows / a.blocks, r1 = (blk + 1) * a.rows / a.blocks;
  const int nr = (int)(r1 - r0);
  const int ld = nr | 1;
  const int n = (int)a.n, k = (int)a.k, CH = a.chunk;
  const int kref = min(nr, n);
  double *Vs = sm;              // ld x n column-major
  double *X = Vs + ld * n;      // ld x CH column-major
  double *ws = a.ws + p * a.wsp;
  const double *vin = ws + a.off_v + r0 * n;
  for (int e = tid; e < nr * n; e += 256) {
    int c = e / nr, r = e - c * nr;
    Vs[c * ld + r] = vin[e];
  }
  for (int j = tid; j < n; j += 256) taus[j] = ws[a.off_tau + blk * n + j];
  if (a.top) {
    const double *rt = ws + a.off_rtop;
    for (int j = tid; j < k; j += 256) sgn[j] = (rt[j * n + j] < 0.0) ? -1.0 : 1.0;
  }
  __syncthreads();
  const double *cin = a.top ? nullptr : ws + a.off_cin + blk * (int64_t)n * k;
  double *dst = a.dst.ptr + p * a.dst.bs;
  for (int c0 = 0; c0 < k; c0 += CH) {
    const int cw = min(CH, k - c0);
    for (int e = tid; e < nr * cw; e += 256) {
      int cc = e / nr, r = e - cc * nr;
      double v = 0.0;
      if (r < kref) {
        if (a.top) v = (r == c0 + cc) ? sgn[r] : 0.0;
        else v = cin[r * k + c0 + cc];
      }
      X[cc * ld + r] = v;
    }
    __syncthreads();
    const int NG = max(1, 256 / cw);
    for (int j = kref - 1; j >= 0; --j) {
      const double tau = taus[j];
      if (tau == 0.0) continue;
      const double *vj = Vs + j * ld;
      if (tid < cw * NG) {
        const int rg = tid % NG, cc = tid / NG;
        const double *xc = X + cc * ld;
        double s = 0.0;
        for (int r = j + 1 + rg; r < nr; r += NG) s += vj[r] * xc[r];
        part[tid] = s;
      }
      __syncthreads();
      if (tid < cw) {
        double s = X[tid * ld + j];
        for (int g = 0; g < NG; ++g) s += part[tid * NG + g];
        Ws[tid] = tau * s;
      }
      __syncthreads();
      {
        const int lane = tid & 63, wv = tid >> 6;
        for (int cc = wv; cc < cw; cc += 4) {
          const double w = Ws[cc];
          double *xc = X + cc * ld;
          for (int r = j + 1 + lane; r < nr; r += 64) xc[r] -= vj[r] * w;
          if (lane == 0) xc[j] -= w;
        }
      }
      __syncthreads();
    }
    for (int e = tid; e < nr * cw; e += 256) {
      int r = e / cw, cc = e - r * cw;
      dst[(r0 + r) * a.dst.rs + (c0 + cc) * a.dst.cs] = X[cc * ld + r];
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
                       hipStream_t s, const int *skip_flag, int64_t skip_stride) {
  if (batch <= 0) return hipSuccess;
  const int64_t n = p.n;
  const int ch = qr_chunk(p.m, n, p.k);
  const size_t lds_max = (size_t)kQrLdsDoubles * sizeof(double);
  static std::once_flag attr_done;  // set once: the maximum a launch may ask for
  std::call_once(attr_done, [&] {
    hipFuncSetAttribute((const void *)tsqr_factor_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
    hipFuncSetAttribute((const void *)tsqr_formq_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
  });
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
    la.skip = skip_flag;
    la.skip_stride = skip_stride;
    const int64_t nrmax = (la.rows + la.blocks - 1) / la.blocks;
    const size_t lds = (size_t)(nrmax | 1) * n * sizeof(double);
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
    fa.chunk = ch;
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
    fa.skip = skip_flag;
    fa.skip_stride = skip_stride;
    const int64_t nrmax = (fa.rows + fa.blocks - 1) / fa.blocks;
    const size_t lds = (size_t)(nrmax | 1) * (n + ch) * sizeof(double);
    tsqr_formq_kernel<<<dim3((unsigned)fa.blocks, (unsigned)batch), 256, lds, s>>>(fa);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Cholesky factor R (G = R^T R) and R^{-1} of a small Gram matrix, from one
// symmetric Gaussian elimination of the augmented block [G | I]: after step j
// the upper triangle of the left half holds D L^T (G = L D L^T, L unit lower)
// and the right half holds L^{-1}; then R = D^{1/2} L^T and
// R^{-1} = L^{-T} D^{-1/2}.  Only the upper triangle of the left half is
// updated (the trailing block stays symmetric, so the multiplier of row i at
// step j is read from row j).  G is read as the in-order sum of ks split-K
// partial products (ks = 1: G itself), the same order a split-K reduction
// uses.  One 256-thread block per pair; W has n rows of 2n + 1 doubles.
// Elimination of [G | I] held in W (n rows of 2n + 1; only the upper
// triangle of the left half need be set), then R, R^{-1} and the pair's flag.
// Every thread of the 256-thread block calls it.
template <int KMAX>
__device__ void chol_eliminate(double *W, double *piv, double &dmax_s, int n, double *ro, double *ri, int *f,
                               int first, double thr_rel) {
  // The matrix [G | I] lives in registers during the elimination: thread
  // (ty, tx) holds rows ty + 4k of columns tx and tx + 64.  By symmetry the
  // multipliers of pivot j are its pivot row, so only that row travels, through
  // a double-buffered LDS row published by its owner wave (one barrier per
  // pivot); every entry gets the same update W(i,c) -= W(j,i) (W(j,c) / d_j)
  // as in place.
  __shared__ double prow[2][2 * kCholMaxN];
  const int ld = 2 * n + 1, n2 = 2 * n;
  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
  static_assert(KMAX >= 1 && 4 * KMAX <= kCholMaxN, "rows per thread");  // n <= 4 KMAX
  const int c0 = tx, c1 = tx + 64;
  double w0[KMAX], w1[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int i = ty + 4 * k;
    w0[k] = (i < n && c0 < n2) ? W[i * ld + c0] : 0.0;
    w1[k] = (i < n && c1 < n2) ? W[i * ld + c1] : 0.0;
  }
  if (tid == 0) {
    double m = 0.0;
    for (int j = 0; j < n; ++j) m = fmax(m, W[j * ld + j]);
    dmax_s = m;
  }
  if (ty == 0) {  // pivot row 0
    if (c0 < n2) prow[0][c0] = w0[0];
    if (c1 < n2) prow[0][c1] = w1[0];
  }
  __syncthreads();
  const double dmax = dmax_s;
  const bool dmax_ok = (dmax > 0.0) && (dmax < 1e300);
  const double thr = thr_rel * dmax;
  int bad = dmax_ok ? 0 : 1;
  // rows updated in column c: left half up to the diagonal, right half all
  const int lim0 = (c0 < n) ? c0 : n - 1, lim1 = (c1 < n) ? c1 : n - 1;
  for (int j = 0; j < n; ++j) {
    const double *pr = prow[j & 1];
    double d = pr[j];
    if (!(d > thr)) {  // also catches NaN; every thread takes the same decision
      bad = 1;
      d = (thr > 0.0 && thr < 1e300) ? thr : 1.0;
    }
    if (tid == 0) piv[j] = d;
    const double inv = 1.0 / d;
    // left columns <= j are final; right columns beyond n + j are still zero
    const bool a0 = (c0 < n) ? (c0 > j) : (c0 < n2 && c0 <= n + j);
    const bool a1 = (c1 < n) ? (c1 > j) : (c1 < n2 && c1 <= n + j);
    const double p0 = a0 ? pr[c0] * inv : 0.0;
    const double p1 = a1 ? pr[c1] * inv : 0.0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int i = ty + 4 * k;
      if (i > j && i < n) {
        const double mul = pr[i];
        if (a0 && i <= lim0) w0[k] = w0[k] - mul * p0;
        if (a1 && i <= lim1) w1[k] = w1[k] - mul * p1;
      }
    }
    // the owner of row j + 1 publishes it, updated through pivot j
    if (j + 1 < n && ty == ((j + 1) & 3)) {
      const int kk = (j + 1) >> 2;
      double *nr = prow[(j + 1) & 1];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k == kk) {
          if (c0 < n2) nr[c0] = w0[k];
          if (c1 < n2) nr[c1] = w1[k];
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int i = ty + 4 * k;
    if (i < n) {
      if (c0 < n2) W[i * ld + c0] = w0[k];
      if (c1 < n2) W[i * ld + c1] = w1[k];
    }
  }
  __syncthreads();
  for (int i = ty; i < n; i += 4) {
    const double si = sqrt(piv[i]);
    for (int c = tx; c < n; c += 64) {
      // R(i, c) = U(i, c) / sqrt(d_i) above the diagonal, sqrt(d_i) on it
      ro[i * n + c] = (c > i) ? W[i * ld + c] / si : ((c == i) ? si : 0.0);
      // R^{-1}(i, c) = L^{-1}(c, i) / sqrt(d_c), zero below the diagonal
      ri[i * n + c] = (c >= i) ? W[c * ld + n + i] / sqrt(piv[c]) : 0.0;
    }
  }
  if (tid == 0) {
    const int ok = bad ? 0 : 1;
    *f = first ? ok : (*f & ok);
  }
}


__global__ __launch_bounds__(256) void chol_kernel(const double *g, int64_t gbs, int ks, int64_t kstride,
                                                   double *r, double *rinv, int64_t rbs, int n, int *flag,
                                                   int64_t fstride, int first, double thr_rel) {
  extern __shared__ double W[];
  __shared__ double piv[kCholMaxN];
  __shared__ double dmax_s;
  const int ld = 2 * n + 1;
  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
  const int p = blockIdx.x;
  const double *G = g + p * gbs;
  for (int i = ty; i < n; i += 4) {
    for (int c = tx; c < n; c += 64) {
      // partials fetched 8 at a time, summed in chunk order
      double v = 0.0;
      for (int t0 = 0; t0 < ks; t0 += 8) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = (t0 + u < ks) ? G[(t0 + u) * kstride + i * n + c] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (t0 + u < ks) v += x[u];
      }
      W[i * ld + c] = v;
      W[i * ld + n + c] = (i == c) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  chol_eliminate<kCholMaxN / 4>(W, piv, dmax_s, n, r + p * rbs, rinv + p * rbs, flag + p * fstride, first, thr_rel);
}

// CholeskyQR step fused with its Gram matrix, for batches of many pairs: the
// block of pair p streams A_p (m x n, n <= 64) once; the four waves take
// interleaved groups of 4 rows and accumulate the upper-triangle 16 x 16
// blocks of A^T A on the matrix cores (a lane's fragment of rows 4s..4s+3 is
// both operands: A(l%16, l/16) of block i is A(4s + l/16, 16 i + l%16), the
// same element as B(l/16, l%16) of block j); the waves then add their
// partial blocks into W in wave order (deterministic) and the block runs the
// elimination above.
template <int NB>
__global__ __launch_bounds__(256, 2) void gram_chol_kernel(CMat A, int64_t m, double *r, double *rinv, int64_t rbs,
                                                        int n, int *flag, int64_t fstride, int first,
                                                        double thr_rel) {
  extern __shared__ double W[];
  __shared__ double piv[kCholMaxN];
  __shared__ double dmax_s;
  // row groups of 4 per load batch: two batches of 3 in flight up to 48
  // columns; one batch of 4 beyond (two would exceed 256 VGPRs)
  constexpr int U = NB <= 3 ? 3 : 4;
  const int ld = 2 * n + 1;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r16 = lane & 15, q4 = lane >> 4;
  const int p = blockIdx.x;
  const double *Ab = A.ptr + p * A.bs;
  d4_t acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = d4_t{0, 0, 0, 0};
  const int64_t groups = (m + 3) / 4;
  // the next iteration's rows are loaded while this iteration's MFMAs run
  auto load = [&](int64_t s0, double (&v)[U][NB]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row = 4 * (s0 + u) + q4;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int col = 16 * b + r16;
        v[u][b] = (row < m && col < n) ? Ab[row * A.rs + (int64_t)col * A.cs] : 0.0;
      }
    }
  };
  auto gram = [&](const double (&v)[U][NB]) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = i; j < NB; ++j) acc[i][j] = mfma16(v[u][i], v[u][j], acc[i][j]);
  };
  if constexpr (NB <= 3) {
    double va[U][NB], vb[U][NB];
    int64_t s0 = (int64_t)wave * U;
    if (s0 < groups) load(s0, va);
    for (; s0 < groups; s0 += 8 * U) {
      const int64_t s1 = s0 + 4 * U;
      if (s1 < groups) load(s1, vb);
      gram(va);
      if (s1 >= groups) break;
      if (s1 + 4 * U < groups) load(s1 + 4 * U, va);
      gram(vb);
    }
  } else {
    for (int64_t s0 = (int64_t)wave * U; s0 < groups; s0 += 4 * U) {
      double v[U][NB];
      load(s0, v);
      gram(v);
    }
  }
  for (int e = tid; e < n * ld; e += 256) {
    const int i = e / ld, c = e - i * ld;
    W[e] = (c == n + i) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = i; j < NB; ++j)
#pragma unroll
          for (int vv = 0; vv < 4; ++vv) {
            const int row = 16 * i + mfma_row<double>(q4, vv), col = 16 * j + r16;
            if (row < n && col < n && col >= row) W[row * ld + col] += acc[i][j][vv];
          }
    }
    __syncthreads();
  }
  chol_eliminate<4 * NB>(W, piv, dmax_s, n, r + p * rbs, rinv + p * rbs, flag + p * fstride, first, thr_rel);
}

hipError_t launch_chol(const double *g, int64_t gbs, int ks, int64_t kstride, double *r, double *rinv,
                       int64_t rbs, int n, int *flag, int64_t fstride, int first, double thr_rel, int batch,
                       hipStream_t s) {
  if (n > kCholMaxN || n < 1 || ks < 1) return hipErrorInvalidValue;
  const size_t lds = (size_t)n * (2 * n + 1) * sizeof(double);
  static std::once_flag attr_done;
  std::call_once(attr_done, [&] {
    hipFuncSetAttribute((const void *)chol_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)(kCholMaxN * (2 * kCholMaxN + 1) * sizeof(double)));
  });
  chol_kernel<<<batch, 256, lds, s>>>(g, gbs, ks, kstride, r, rinv, rbs, n, flag, fstride, first, thr_rel);
  return hipGetLastError();
}

hipError_t launch_gram_chol(CMat A, int64_t m, int n, double *r, double *rinv, int64_t rbs, int *flag,
                            int64_t fstride, int first, double thr_rel, int batch, hipStream_t s) {
  if (n > kCholMaxN || n < 1 || m < 1) return hipErrorInvalidValue;
  const size_t lds = (size_t)n * (2 * n + 1) * sizeof(double);
  static std::once_flag attr_done;
  std::call_once(attr_done, [&] {
    const int mx = (int)(kCholMaxN * (2 * kCholMaxN + 1) * sizeof(double));
    hipFuncSetAttribute((const void *)gram_chol_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    hipFuncSetAttribute((const void *)gram_chol_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    hipFuncSetAttribute((const void *)gram_chol_kernel<3>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    hipFuncSetAttribute((const void *)gram_chol_kernel<4>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
  });
  const int nb = (n + 15) / 16;
  if (nb == 1) gram_chol_kernel<1><<<batch, 256, lds, s>>>(A, m, r, rinv, rbs, n, flag, fstride, first, thr_rel);
  else if (nb == 2) gram_chol_kernel<2><<<batch, 256, lds, s>>>(A, m, r, rinv, rbs, n, flag, fstride, first, thr_rel);
  else if (nb == 3) gram_chol_kernel<3><<<batch, 256, lds, s>>>(A, m, r, rinv, rbs, n, flag, fstride, first, thr_rel);
  else gram_chol_kernel<4><<<batch, 256, lds, s>>>(A, m, r, rinv, rbs, n, flag, fstride, first, thr_rel);
  return hipGetLastError();
}

}  // namespace hatt
