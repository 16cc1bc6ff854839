// Dense kernels for the QR of tall frames that may be rank deficient:
//
//  * hh_qr_kernel: economy Householder QR of one short matrix (m <= 384
//    rows for n <= 64 columns, m <= 256 for n <= 128) per workgroup, the matrix resident in registers.
//    This is the QR Alg. 4 asks for (the paper's econ-QR), exact for rank
//    deficient input: whatever the rank, Q has orthonormal columns and
//    Q R = A to rounding.
//  * trinv_kernel: inverse of an upper triangular n x n matrix (n <= 128).
//  * chol1k_kernel: Cholesky factor R and R^{-1} of an n x n Gram matrix
//    (n <= 128), the symmetric elimination of [G | I] with 1024 threads.
//  * sketch_rows_kernel: B = Omega A for a sparse sign matrix Omega with k
//    rows (row r of B sums the rows pi(r), pi(r + k), pi(r + 2k), ... of A
//    with hashed signs, pi a pseudo-random permutation of the rows, so that
//    every row of B mixes unrelated rows of A); B R0^{-1} well conditioned
//    makes A R0^{-1} well conditioned enough for CholeskyQR2 (randomised
//    preconditioning of CholeskyQR).
//
// Register layout of hh_qr_kernel (1024 threads = 16 waves): wave w owns the
// columns w, w + 16, w + 32, ... (CPW of them); lane l holds the rows l,
// l + 64, ... (RPL of them).  Column dot products are wave reductions, so a
// Householder step needs one barrier: the owner of column j publishes its
// reflector through LDS and every wave updates its own columns.
#include <mutex>
#include "common.h"

namespace hatt {

namespace {

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 64 lanes, the same bits in every lane (each butterfly step
// adds the pair in both orders, and x + y == y + x exactly).
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror: quads of an 8-lane half
  v += dpp_d<0x140>(v);  // row_mirror: halves of a 16-lane row
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// Sum over aligned groups of 8 lanes (every lane of the group gets it).
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  return v;
}

__device__ __forceinline__ double lane_bcast(double v, int src) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, src);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Wave sums of 8 values per lane at once (a reduce-scatter): halving
// exchanges across lanes 32, 16 and 8 apart leave lanes 8t .. 8t+7 with
// partial sums of value t, an 8-lane sum completes them, and lane 8t
// broadcasts.  out[t] = sum over the 64 lanes of d[t], the same in every
// lane.
__device__ __forceinline__ void wave_sum8(const double (&d)[8], double (&out)[8]) {
  const int lane = threadIdx.x & 63;
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
  double e[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double keep = b5 ? d[k + 4] : d[k], give = b5 ? d[k] : d[k + 4];
    e[k] = keep + __shfl_xor(give, 32);
  }
  double f[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double keep = b4 ? e[k + 2] : e[k], give = b4 ? e[k] : e[k + 2];
    f[k] = keep + __shfl_xor(give, 16);
  }
  double g = (b3 ? f[1] : f[0]) + __shfl_xor(b3 ? f[0] : f[1], 8);
  g += dpp_d<0xB1>(g);
  g += dpp_d<0x4E>(g);
  g += dpp_d<0x141>(g);
  // lanes 8t..8t+7 hold value t' with t' = (lane>>3 & 1) + 2 (lane>>4 & 1) + 4 (lane>>5 & 1)
#pragma unroll
  for (int t = 0; t < 8; ++t) out[t] = lane_bcast(g, 8 * t);
}

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  // integer finaliser of MurmurHash3 (Appleby)
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}

// Random bit stream for completion vectors: entry r of vector c under a
// key; nested hashes, so that different (key, c) give unrelated vectors.
__device__ __forceinline__ uint32_t rand_sign(uint32_t key, int c, int64_t r) {
  const uint32_t col = hash32(hash32(key) ^ ((uint32_t)c * 0x85EBCA77u + 0x27D4EB2Fu));
  return hash32(col ^ ((uint32_t)r * 0x9E3779B1u)) >> 7;
}

}  // namespace

// ---------------------------------------------------------------------------
// Householder QR.  Reflector j (LAPACK's dlarfg convention): for the column
// x = A(j:m, j), beta = -sign(alpha) ||x||, tau = (beta - alpha) / beta,
// v = [1; x(2:) / (alpha - beta)], H_j = I - tau v v^T, H_j x = beta e_1;
// x(2:) = 0 gives tau = 0.  Q = H_0 H_1 ... H_{n-1} [I_n; 0] is formed by
// backward accumulation.  Finally rows of R and columns of Q are flipped so
// that diag(R) >= 0.
// x(:, c) -= tau v (v^T x(:, c)) for the wave's columns c with c0 <= c < n.
template <int CPW, int RPL>
__device__ __forceinline__ void hh_apply(double (&x)[CPW][RPL], const double (&v)[RPL], double tau, int w, int c0,
                                         int n) {
  static_assert(CPW % 4 == 0 && CPW <= 8, "column slots");
  if (w + 16 * (CPW - 1) < c0) return;  // no live column (wave-uniform)
  double d[8], sum[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    d[t] = 0.0;
    if (t < CPW) {
#pragma unroll
      for (int q = 0; q < RPL; ++q) d[t] += v[q] * x[t < CPW ? t : 0][q];
    }
  }
  wave_sum8(d, sum);
#pragma unroll
  for (int t = 0; t < CPW; ++t) {
    const int c = w + 16 * t;
    if (c >= c0 && c < n) {  // uniform per wave
      const double f = tau * sum[t];
#pragma unroll
      for (int q = 0; q < RPL; ++q) x[t][q] -= f * v[q];
    }
  }
}

template <int CPW, int RPL>
__global__ __launch_bounds__(1024) void hh_qr_kernel(HhArgs a) {
  constexpr int MR = 64 * RPL;
  __shared__ double vbuf[2][MR];
  __shared__ double tau_s[16 * CPW];
  __shared__ double sgn_s[16 * CPW];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int p = blockIdx.x;
  if (a.skip_flag != nullptr && a.skip_flag[p * a.skip_stride] == 1) return;
  const int m = a.m, n = a.n;
  const double *A = a.A.ptr + p * a.A.bs;
  double x[CPW][RPL];
#pragma unroll
  for (int t = 0; t < CPW; ++t) {
    const int c = w + 16 * t;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = lane + 64 * q;
      x[t][q] = (c < n && r < m) ? A[r * a.A.rs + c * a.A.cs] : 0.0;
    }
  }
  // A may alias Q: every load above is done before any store below
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const int ow = j & 15, tj = j >> 4;
    double *vb = vbuf[j & 1];
    if (w == ow) {
      double col[RPL];
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        col[q] = 0.0;
#pragma unroll
        for (int t = 0; t < CPW; ++t)
          if (t == tj) col[q] = x[t][q];
      }
      double s = 0.0, al = 0.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int r = lane + 64 * q;
        if (r > j) s += col[q] * col[q];
        if (r == j) al = col[q];
      }
      const double sigma = wave_sum(s);
      const double alpha = wave_sum(al);  // one lane holds it
      double tau = 0.0, beta = alpha, scale = 0.0;
      if (sigma > 0.0) {
        const double nrm = sqrt(alpha * alpha + sigma);
        beta = (alpha >= 0.0) ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int r = lane + 64 * q;
        const double v = (r > j) ? col[q] * scale : (r == j ? 1.0 : 0.0);
        vb[r] = v;
        // the owner keeps beta on the diagonal and v below it
        const double nv = (r > j) ? v : (r == j ? beta : col[q]);
#pragma unroll
        for (int t = 0; t < CPW; ++t)
          if (t == tj) x[t][q] = nv;
      }
      if (lane == 0) {
        tau_s[j] = tau;
        sgn_s[j] = (beta < 0.0) ? -1.0 : 1.0;
      }
    }
    __syncthreads();
    const double tau = tau_s[j];
    double v[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) v[q] = vb[lane + 64 * q];
    hh_apply<CPW, RPL>(x, v, tau, w, j + 1, n);
  }
  __syncthreads();
  // R: rows i <= c of column c, sign-flipped per row
  if (a.R.ptr != nullptr) {
    double *R = a.R.ptr + p * a.R.bs;
#pragma unroll
    for (int t = 0; t < CPW; ++t) {
      const int c = w + 16 * t;
      if (c < n) {
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
          const int r = lane + 64 * q;
          if (r < n) R[r * a.R.rs + c * a.R.cs] = (r <= c) ? sgn_s[r] * x[t][q] : 0.0;
        }
      }
    }
  }
  if (a.Q.ptr == nullptr) return;
  // reflectors to the Q buffer (below the diagonal; read back by every wave)
  double *Q = a.Q.ptr + p * a.Q.bs;
#pragma unroll
  for (int t = 0; t < CPW; ++t) {
    const int c = w + 16 * t;
    if (c < n) {
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int r = lane + 64 * q;
        if (r > c && r < m) Q[r * a.Q.rs + c * a.Q.cs] = x[t][q];
      }
    }
  }
  __syncthreads();
  // Q = H_0 ... H_{n-1} [I; 0], starting from the identity columns
#pragma unroll
  for (int t = 0; t < CPW; ++t) {
    const int c = w + 16 * t;
#pragma unroll
    for (int q = 0; q < RPL; ++q) x[t][q] = (lane + 64 * q == c) ? 1.0 : 0.0;
  }
  // reflector j is read one step ahead of its use
  double vn[RPL];
  auto vload = [&](int j, double(&v)[RPL]) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = lane + 64 * q;
      v[q] = (j >= 0 && r > j && r < m) ? Q[r * a.Q.rs + j * a.Q.cs] : (r == j ? 1.0 : 0.0);
    }
  };
  vload(n - 1, vn);
  for (int j = n - 1; j >= 0; --j) {
    const double tau = tau_s[j];
    double v[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) v[q] = vn[q];
    vload(j - 1, vn);
    if (tau == 0.0) continue;  // uniform
    hh_apply<CPW, RPL>(x, v, tau, w, j, n);
  }
  __syncthreads();  // every reflector has been read
#pragma unroll
  for (int t = 0; t < CPW; ++t) {
    const int c = w + 16 * t;
    if (c < n) {
      const double sg = sgn_s[c];
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int r = lane + 64 * q;
        if (r < m) Q[r * a.Q.rs + c * a.Q.cs] = sg * x[t][q];
      }
    }
  }
}

bool hh_qr_supported(int64_t m, int64_t n) { return n >= 1 && n <= 128 && m >= n && m <= (n <= 64 ? 384 : 256); }

hipError_t launch_hh_qr(const HhArgs &a, int batch, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  if (!hh_qr_supported(a.m, a.n)) return hipErrorInvalidValue;
  const int m = (int)a.m;
  if (a.n <= 64) {
    if (m <= 128) hh_qr_kernel<4, 2><<<batch, 1024, 0, s>>>(a);
    else if (m <= 256) hh_qr_kernel<4, 4><<<batch, 1024, 0, s>>>(a);
    else hh_qr_kernel<4, 6><<<batch, 1024, 0, s>>>(a);
  } else {
    if (m <= 128) hh_qr_kernel<8, 2><<<batch, 1024, 0, s>>>(a);
    else hh_qr_kernel<8, 4><<<batch, 1024, 0, s>>>(a);
  }
  return hipGetLastError();
}

const char *hh_qr_kernel_name(int64_t m, int64_t n) {
  if (n <= 64) {
    if (m <= 128) return "hh_qr_kernel<4, 2>";
    if (m <= 256) return "hh_qr_kernel<4, 4>";
    return "hh_qr_kernel<4, 6>";
  }
  if (m <= 128) return "hh_qr_kernel<8, 2>";
  return "hh_qr_kernel<8, 4>";
}

// ---------------------------------------------------------------------------
// X = R^{-1} for upper triangular R (n x n, n <= 128): eight lanes per
// column c run the back substitution X(i, c) = -(sum_{i<k<=c} R(i,k) X(k,c))
// / R(i,i), lane t of the group holding X(k, c) for k = t (mod 8).  R sits in
// LDS.  With mask != nullptr, a column whose diagonal entry is at most
// 1e-12 of the column's norm (a column of the factored matrix that depends
// on the ones before it) is replaced by dmax e_j before the inversion and
// marked mask[j] = 1 (else 0); otherwise a zero or non-finite diagonal entry
// clears the pair's flag (may be null).
constexpr double kDepRel = 1e-12;

__global__ __launch_bounds__(1024) void trinv_kernel(const double *r, int64_t rbs, double *xo, int64_t xbs, int n,
                                                     int *flag, int64_t fstride, int first, int *mask,
                                                     int64_t mbs, double dep_abs) {
  extern __shared__ double Rs[];  // n x n, then the reciprocal diagonal
  double *dinv = Rs + n * n;
  __shared__ int ok_s;
  __shared__ double dmax_s;
  const int tid = threadIdx.x;
  const int p = blockIdx.x;
  const double *R = r + p * rbs;
  if (tid == 0) ok_s = 1;
  for (int e = tid; e < n * n; e += 1024) Rs[e] = R[e];
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i < n; ++i) mx = fmax(mx, fabs(Rs[i * n + i]));
    dmax_s = mx;
  }
  __syncthreads();
  const double dmax = dmax_s;
  if (mask != nullptr) {
    // one thread per column: a column whose pivot is at most kDepRel of its
    // own norm (the norm of the factored column), or at most dep_abs when
    // that is set, depends on the ones before it; its entries above the
    // diagonal are cleared
    for (int j = tid; j < n; j += 1024) {
      const double d = Rs[j * n + j];
      double cn = 0.0;
      for (int i = 0; i <= j; ++i) cn += Rs[i * n + j] * Rs[i * n + j];
      const double thr = dep_abs > 0.0 ? dep_abs : kDepRel * sqrt(cn);
      const int dep = !(fabs(d) > thr) || !(fabs(d) > 1e-300) ? 1 : 0;  // also NaN
      mask[p * mbs + j] = dep;
      if (dep) {
        for (int i = 0; i < j; ++i) Rs[i * n + j] = 0.0;
        Rs[j * n + j] = (dmax > 0.0 && isfinite(dmax)) ? dmax : 1.0;
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += 1024) {
    const double d = Rs[i * n + i];
    if (!(d != 0.0) || !isfinite(d)) ok_s = 0;
    dinv[i] = 1.0 / d;
  }
  __syncthreads();
  const int c = tid >> 3, t = tid & 7;
  double xk[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) xk[s] = 0.0;
  // the column's first entry; groups beyond n idle but take part in the
  // group sums with zeros
  const int cc = (c < n) ? c : -1;
  if (cc >= 0 && (cc & 7) == t) {
#pragma unroll
    for (int s = 0; s < 16; ++s)
      if (s == (cc >> 3)) xk[s] = dinv[cc];
  }
  // the wave runs to the largest column it holds (columns 8 w' .. 8 w' + 7)
  const int cmax = ((tid >> 6) << 3) + 7;
  for (int i = cmax - 1; i >= 0; --i) {
    double acc = 0.0;
    if (cc > i) {
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const int k = t + 8 * s;
        if (k > i && k <= cc) acc += Rs[i * n + k] * xk[s];
      }
    }
    const double sum = group8_sum(acc);
    if (cc > i && (i & 7) == t) {
      const double v = -sum * dinv[i];
#pragma unroll
      for (int s = 0; s < 16; ++s)
        if (s == (i >> 3)) xk[s] = v;
    }
  }
  if (cc >= 0) {
    double *X = xo + p * xbs;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int k = t + 8 * s;
      if (k < n) X[k * n + cc] = (k <= cc) ? xk[s] : 0.0;
    }
  }
  if (flag != nullptr && tid == 0) {
    int *f = flag + p * fstride;
    *f = first ? ok_s : (*f & ok_s);
  }
}

hipError_t launch_trinv(const double *r, int64_t rbs, double *x, int64_t xbs, int n, int *flag, int64_t fstride,
                        int first, int *mask, int64_t mbs, double dep_abs, int batch, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  if (n < 1 || n > 128) return hipErrorInvalidValue;
  const size_t lds = (size_t)(n * n + n) * sizeof(double);
  static std::once_flag attr;
  std::call_once(attr, [&] {
    hipFuncSetAttribute((const void *)trinv_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)((128 * 128 + 128) * sizeof(double)));
  });
  trinv_kernel<<<batch, 1024, lds, s>>>(r, rbs, x, xbs, n, flag, fstride, first, mask, mbs, dep_abs);
  return hipGetLastError();
}

// Columns j of A (m x n row-major per pair, pair stride abs) with
// mask[p * mbs + j] set are replaced by a hashed random sign vector of unit
// norm (entries +-1/sqrt(m)).
__global__ void complete_cols_kernel(double *a, int64_t m, int n, int64_t abs_, const int *mask, int64_t mbs,
                                     uint32_t key) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (e >= m * n) return;
  const int c = (int)(e % n);
  if (!mask[p * mbs + c]) return;
  const int64_t r = e / n;
  const double v = 1.0 / sqrt((double)m);
  a[p * abs_ + e] = (rand_sign(key, c, r) & 1u) ? -v : v;
}

hipError_t launch_complete_cols(double *a, int64_t m, int n, int64_t abs_, const int *mask, int64_t mbs,
                                uint32_t key, int batch, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  dim3 grid((unsigned)((m * n + 255) / 256), (unsigned)batch);
  complete_cols_kernel<<<grid, 256, 0, s>>>(a, m, n, abs_, mask, mbs, key);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cholesky factor of G (n x n, n <= 128) with R^{-1}, by the symmetric
// Gaussian elimination of [G | I] (G = L D L^T; R = D^{1/2} L^T,
// R^{-1} = L^{-T} D^{-1/2}), held in registers: thread (ty, tx) of 16 x 64
// holds rows ty + 16 k of the columns tx + 64 s.  The multipliers of pivot j
// are its own row (symmetry).  Two pivots per barrier: the owners of rows j
// and j + 1 publish them (updated through pivot j - 1) in a double-buffered
// LDS pair, and every thread forms row j + 1's update by pivot j itself where
// it needs it (its columns, its rows' multipliers and the second pivot), with
// the same operations as the owner.  Pivots <= thr_rel * max diag(G) (and
// NaN) clear the flag.
__global__ __launch_bounds__(1024) void chol1k_kernel(const double *g, int64_t gbs, double *ro, double *rio,
                                                      int64_t rbs, int n, int *flag, int64_t fstride, int first,
                                                      double thr_rel) {
  constexpr int KR = 8, NS = 4;  // rows per thread, column slots (2n <= 256)
  __shared__ double prow[2][2][256];
  __shared__ double piv[128];
  __shared__ double dmax_s;
  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
  const int p = blockIdx.x;
  const double *G = g + p * gbs;
  const int n2 = 2 * n;
  double w[KR][NS];
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    const int i = ty + 16 * k;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int c = tx + 64 * s;
      double v = 0.0;
      if (i < n && c < n2) v = (c < n) ? G[i * n + c] : ((c - n == i) ? 1.0 : 0.0);
      w[k][s] = v;
    }
  }
  if (ty < 2 && ty < n) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int c = tx + 64 * s;
      if (c < n2) prow[0][ty][c] = w[0][s];
    }
  }
  if (tid == 0) {
    double m = 0.0;
    for (int j = 0; j < n; ++j) m = fmax(m, G[j * n + j]);
    dmax_s = m;
  }
  __syncthreads();
  const double dmax = dmax_s;
  const bool dmax_ok = (dmax > 0.0) && (dmax < 1e300);
  const double thr = thr_rel * dmax;
  int bad = dmax_ok ? 0 : 1;
  for (int j = 0; j < n; j += 2) {
    const double *pj = prow[(j >> 1) & 1][0], *pk = prow[(j >> 1) & 1][1];
    const bool two = j + 1 < n;  // block-uniform
    double d = pj[j];
    if (!(d > thr)) {
      bad = 1;
      d = (thr > 0.0 && thr < 1e300) ? thr : 1.0;
    }
    const double inv = 1.0 / d;
    // pc / pc2: the scaled pivot rows on the columns each pivot updates (left
    // half: columns > j; right half: up to n + j), zero elsewhere, so that
    // the row updates below need no column tests (on the left half they also
    // touch the lower triangle, which is never read or written out)
    double pc[NS], pc2[NS];
    bool act[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int c = tx + 64 * s;
      act[s] = (c < n) ? (c > j) : (c < n2 && c <= n + j);
      pc[s] = act[s] ? pj[c] * inv : 0.0;
    }
    // row j + 1 after pivot j: pk - m pj / d on the columns pivot j touches
    const double m = two ? pj[j + 1] : 0.0;
    double inv2 = 0.0;
    if (two) {
      double d2 = pk[j + 1] - m * (pj[j + 1] * inv);
      if (!(d2 > thr)) {
        bad = 1;
        d2 = (thr > 0.0 && thr < 1e300) ? thr : 1.0;
      }
      if (tid == 0) piv[j + 1] = d2;
      inv2 = 1.0 / d2;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int c = tx + 64 * s;
      const bool act2 = two && ((c < n) ? (c > j + 1) : (c < n2 && c <= n + j + 1));
      const double rk = act[s] ? pk[c] - m * pc[s] : (c < n2 ? pk[c] : 0.0);
      pc2[s] = act2 ? rk * inv2 : 0.0;
    }
    if (tid == 0) piv[j] = d;
    // rows ty + 16 k <= j are final: k below kmin is skipped (wave-uniform)
    const int kmin = (j + 16 - ty) >> 4;  // first k with ty + 16 k > j
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int i = ty + 16 * k;
      if (k >= kmin && i < n) {
        const double mul = pj[i];
        const bool second = two && i > j + 1;
        const double mul2 = second ? pk[i] - m * (pj[i] * inv) : 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          w[k][s] -= mul * pc[s];
          if (second) w[k][s] -= mul2 * pc2[s];
        }
      }
    }
    // the owners of rows j + 2 and j + 3 publish them for the next pair
    double(*nb)[256] = prow[((j >> 1) + 1) & 1];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = j + 2 + h;
      if (r < n && ty == (r & 15)) {
        const int kk = r >> 4;
#pragma unroll
        for (int k = 0; k < KR; ++k)
          if (k == kk) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
              const int c = tx + 64 * s;
              if (c < n2) nb[h][c] = w[k][s];
            }
          }
      }
    }
    __syncthreads();
  }
  double *R = ro + p * rbs, *Ri = rio + p * rbs;
  // R(i, c) = U(i, c) / sqrt(d_i) (c > i), sqrt(d_i) on the diagonal;
  // R^{-1}(c, i) = L^{-1}(i, c) / sqrt(d_i) for c <= i, i.e. from the right half
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    const int i = ty + 16 * k;
    if (i < n) {
      const double si = sqrt(piv[i]);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int c = tx + 64 * s;
        if (c < n) {
          R[i * n + c] = (c > i) ? w[k][s] / si : ((c == i) ? si : 0.0);
        } else if (c < n2) {
          const int cc = c - n;  // L^{-1}(i, cc), nonzero for cc <= i
          Ri[cc * n + i] = (cc <= i) ? w[k][s] / si : 0.0;
        }
      }
    }
  }
  if (tid == 0) {
    int *f = flag + p * fstride;
    const int ok = bad ? 0 : 1;
    *f = first ? ok : (*f & ok);
  }
}

hipError_t launch_chol1k(const double *g, int64_t gbs, double *r, double *rinv, int64_t rbs, int n, int *flag,
                         int64_t fstride, int first, double thr_rel, int batch, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  if (n < 1 || n > 128) return hipErrorInvalidValue;
  chol1k_kernel<<<batch, 1024, 0, s>>>(g, gbs, r, rinv, rbs, n, flag, fstride, first, thr_rel);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Block Gram-Schmidt panel test: W = A_p - Q S1 is a panel's residual after
// its first projection (m x cw), S1 the projection coefficients (c0 x cw).
// A column with ||W_j||^2 <= rel^2 (||S1_j||^2 + ||W_j||^2) lies in the span
// of the previous panels up to rounding: it is marked (mask[j] = 1) and W_j
// is replaced by a random unit vector, so that the panel QR and the second
// projection see a well-conditioned panel.  One 1024-thread block per pair:
// thread (row group tr of 8, column tc of 128).
__global__ __launch_bounds__(1024) void panel_dep_kernel(Mat W, CMat S1, int64_t m, int64_t c0, int cw, int *mask,
                                                         int64_t mbs, double rel, uint32_t key) {
  __shared__ double pw[8][128], ps[8][128];
  __shared__ int dep[128];
  const int tid = threadIdx.x, tc = tid & 127, tr = tid >> 7;
  const int p = blockIdx.x;
  double sw = 0.0, ss = 0.0;
  if (tc < cw) {
    const double *w = W.ptr + p * W.bs + tc * W.cs;
    for (int64_t r = tr; r < m; r += 8) {
      const double v = w[r * W.rs];
      sw += v * v;
    }
    const double *s = S1.ptr + p * S1.bs + tc * S1.cs;
    for (int64_t r = tr; r < c0; r += 8) {
      const double v = s[r * S1.rs];
      ss += v * v;
    }
  }
  pw[tr][tc] = sw;
  ps[tr][tc] = ss;
  __syncthreads();
  if (tr == 0) {
    double a = 0.0, b = 0.0;
    for (int g = 0; g < 8; ++g) {
      a += pw[g][tc];
      b += ps[g][tc];
    }
    const int d = (tc < cw) && !(a > rel * rel * (a + b)) ? 1 : 0;
    dep[tc] = d;
    if (tc < cw) mask[p * mbs + tc] = d;
  }
  __syncthreads();
  if (tc < cw && dep[tc]) {
    double *w = W.ptr + p * W.bs + tc * W.cs;
    const double v = 1.0 / sqrt((double)m);
    for (int64_t r = tr; r < m; r += 8) w[r * W.rs] = (rand_sign(key, tc, r) & 1u) ? -v : v;
  }
}

hipError_t launch_panel_dep(Mat W, CMat S1, int64_t m, int64_t c0, int cw, int *mask, int64_t mbs, double rel,
                            uint32_t key, int batch, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  if (cw < 1 || cw > 128) return hipErrorInvalidValue;
  panel_dep_kernel<<<batch, 1024, 0, s>>>(W, S1, m, c0, cw, mask, mbs, rel, key);
  return hipGetLastError();
}

// Columns j of R (rows x cw, strided) with mask[p * mbs + j] set become zero.
__global__ void zero_masked_cols_kernel(Mat R, int rows, int cw, const int *mask, int64_t mbs) {
  const int p = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cw) return;
  const int r = e / cw, c = e - r * cw;
  if (mask[p * mbs + c]) R.ptr[p * R.bs + r * R.rs + c * R.cs] = 0.0;
}

hipError_t launch_zero_masked_cols(Mat R, int rows, int cw, const int *mask, int64_t mbs, int batch, hipStream_t s) {
  if (batch <= 0 || rows <= 0 || cw <= 0) return hipSuccess;
  dim3 grid((unsigned)((rows * cw + 255) / 256), (unsigned)batch);
  zero_masked_cols_kernel<<<grid, 256, 0, s>>>(R, rows, cw, mask, mbs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// B(r, c) = sum_t sign(r + t k) A(r + t k, c), r < k, c < n, per pair.
// Threads run along whichever of r, c is contiguous in A.
// A pseudo-random permutation of [0, m) (m < 2^31): a bijection of
// [0, 2^bits) built from invertible steps (odd multiplications, xor with a
// right shift, key addition), walked along its cycle until it lands below m.
__device__ __forceinline__ uint32_t perm_row(uint32_t x, uint32_t m, int bits, uint32_t key) {
  const uint32_t mask = (bits >= 32) ? 0xFFFFFFFFu : ((1u << bits) - 1u);
  const int sh = (bits + 1) / 2;
  do {
    x = (x * 0x9E3779B1u + key) & mask;
    x ^= x >> sh;
    x = (x * 0x85EBCA77u + (key >> 7)) & mask;
    x ^= x >> sh;
    x = (x * 0xC2B2AE3Du) & mask;
  } while (x >= m);
  return x;
}

__global__ void sketch_rows_kernel(CMat A, int64_t m, int n, int k, double *b, int64_t bbs, uint32_t key,
                                   int rows_fast) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (e >= (int64_t)k * n) return;
  int r, c;
  if (rows_fast) {
    c = (int)(e / k);
    r = (int)(e - (int64_t)c * k);
  } else {
    r = (int)(e / n);
    c = (int)(e - (int64_t)r * n);
  }
  const double *a = A.ptr + p * A.bs + c * A.cs;
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) < m) ++bits;
  // row t of the sum is row perm(r + t k) of A; eight independent partial
  // sums keep eight loads in flight
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t i = r;
  for (; i + 7 * (int64_t)k < m; i += 8 * (int64_t)k) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t ii = perm_row((uint32_t)(i + u * (int64_t)k), (uint32_t)m, bits, key);
      const double v = a[(int64_t)ii * A.rs];
      acc[u] += (hash32(ii ^ key) & 1u) ? -v : v;
    }
  }
  for (int u = 0; i < m; i += k, ++u) {
    const uint32_t ii = perm_row((uint32_t)i, (uint32_t)m, bits, key);
    const double v = a[(int64_t)ii * A.rs];
    acc[u] += (hash32(ii ^ key) & 1u) ? -v : v;
  }
  b[p * bbs + (int64_t)r * n + c] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

hipError_t launch_sketch_rows(CMat A, int64_t m, int n, int k, double *b, int64_t bbs, uint32_t key, int batch,
                              hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const int64_t tot = (int64_t)k * n;
  dim3 grid((unsigned)((tot + 255) / 256), (unsigned)batch);
  sketch_rows_kernel<<<grid, 256, 0, s>>>(A, m, n, k, b, bbs, key, A.rs == 1 ? 1 : 0);
  return hipGetLastError();
}

}  // namespace hatt
