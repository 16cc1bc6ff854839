// Small dense SVD by one-sided (Hestenes) Jacobi, followed by the
// truncation-rank choice of TT-Rounding.
//
// One-sided Jacobi rotates column pairs of A = R (kr x nc) until all columns
// are mutually orthogonal: A_final = R J with J orthogonal, so
// sigma_j = ||A_final(:, j)|| and U(:, j) = A_final(:, j) / sigma_j.  The
// columns of A_final stay orthogonal to working precision *relative to their
// own norms*, so U is orthonormal even where sigma_j is tiny; the right factor
// is therefore never accumulated: S V^T restricted to the kept rows is formed
// as U_rho^T R, which equals S_rho V_rho^T up to rounding.
//
// A sweep visits every column pair once in the round-robin (circle) order:
// nc' - 1 rounds (nc' = nc rounded up to even) of nc'/2 disjoint pairs.  A
// pair is rotated when |a_p . a_q| > tau ||a_p|| ||a_q|| with
// tau = max(1e-15, kr eps) (below the rounding noise of a kr-term dot product
// the test would keep firing and the sweeps never end); sweeps stop when
// none is.
//   * nc <= 64: one wavefront per matrix, lane c keeps column c in
//     registers; partners are read through LDS.
//   * larger nc: one 256-thread workgroup per matrix, A in LDS, each pair
//     handled by a group of lanes that reduce with shuffles.
#include <mutex>
#include "common.h"

namespace hatt {

// Rotation threshold on |cos| of a column pair's angle (see above).
__device__ __forceinline__ double jacobi_tau(int kr) { return fmax(1e-15, (double)kr * 2.220446049250313e-16); }

// Early stop of every Jacobi kernel: a sweep whose largest squared cosine
// between two columns is at most this rotated by angles whose squares are
// below rounding, so by the quadratic convergence of cyclic Jacobi the
// columns are orthogonal to rounding after it.  Without it, columns that are
// pure rounding noise (rank-deficient R) kept passing the rotation test on
// the noise of their own dot products and ran to the sweep limit.
constexpr double kJacobiStop2 = 1e-16;

// A column whose squared norm is at most this is zero to every Jacobi kernel:
// it is neither rotated nor counted for the early stop, and its singular
// value is reported as 0 (zero U column, zero S V^T row).  Such columns are
// what rotation leaves of the null space of a rank-deficient R; their
// entries square into the subnormal range, where the dot products lose all
// relative accuracy and the pair would rotate on its own rounding until the
// sweep limit.  Entries of a column at the threshold are still around 1e-141,
// so products with them stay well clear of underflow.
constexpr double kJacobiTiny2 = 1e-280;
__device__ __forceinline__ bool jacobi_live(double al, double be) { return al > kJacobiTiny2 && be > kJacobiTiny2; }
__device__ __forceinline__ double jacobi_sigma(double s2) { return s2 > kJacobiTiny2 ? sqrt(s2) : 0.0; }

__device__ __forceinline__ int rr_partner(int c, int t, int np) {
  // round t: position 0 holds index 0, position j >= 1 holds 1 + (j - 1 + t) mod (np - 1);
  // positions k and np - 1 - k are paired
  const int m = np - 1;
  const int pos = (c == 0) ? 0 : 1 + ((c - 1 - t) % m + m) % m;
  const int ppos = np - 1 - pos;
  return (ppos == 0) ? 0 : 1 + (ppos - 1 + t) % m;
}

// Rank rule shared by both kernels (thread-serial, n <= 139).
__device__ int choose_rank(const double *sig_sorted, int kr, int nc, const SvdArgs &a, int p) {
  if (a.rel_keep > 0.0) {
    // eq. HPCRL--2 split: terms with sigma_j > ep ||W||_2, at least one
    int rho = 0;
    const int kmax = min(kr, nc);
    for (int j = 0; j < kmax; ++j) rho += (sig_sorted[j] > a.rel_keep * sig_sorted[0]);
    if (rho > a.ucap) rho = a.ucap;
    if (rho < 1) rho = 1;
    a.rank_out[p * a.rank_bs] = rho;
    return rho;
  }
  double tot2 = 0.0;
  for (int j = 0; j < nc; ++j) tot2 += sig_sorted[j] * sig_sorted[j];
  if (a.first_bond) a.delta2[p] = a.tol2_over_dm1 * tot2;
  const double d2 = a.delta2[p];
  int kmax = min(kr, nc);
  if (a.prev_rank != nullptr) {
    const int64_t lim = a.prev_rank[p * a.rank_bs] * a.n_mode;
    if (lim < kmax) kmax = (int)lim;
  }
  int rho = kmax;
  if (d2 > 0.0) {
    double tail = 0.0;
    for (int j = kmax - 1; j >= 1; --j) {
      const double sj = sig_sorted[j];
      tail += sj * sj;
      if (tail <= d2) rho = j;
      else break;
    }
  }
  if (a.cap > 0 && rho > a.cap) rho = (int)a.cap;
  if (rho > a.ucap) rho = a.ucap;
  if (rho < 1) rho = 1;
  a.rank_out[p * a.rank_bs] = rho;
  return rho;
}

// nc <= 64: one wavefront per matrix (a 64-thread block).  Lane c holds all
// of column c in registers; a round publishes the columns through LDS
// (double-buffered by round parity) and both lanes of a pair form the same
// full-length dot products (the same products summed in the same order), so
// they derive bit-identical rotations without any cross-wave reduction.
template <int KR>
__global__ __launch_bounds__(64) void svd_wave_kernel(SvdArgs a) {
  extern __shared__ double sm[];
  double *xb0 = sm;            // KR x 64, xb[r * 64 + c]
  double *xb1 = sm + KR * 64;
  __shared__ double sig[64];
  __shared__ double sigs[64];
  __shared__ int perm[64];
  __shared__ int s_rho;
  const int lane = threadIdx.x;
  const int p = blockIdx.x;
  const int kr = a.kr, nc = a.nc;
  const double *R = a.r + p * a.rbs;
  double col[KR];
#pragma unroll
  for (int i = 0; i < KR; ++i) col[i] = (lane < nc && i < kr) ? R[i * nc + lane] : 0.0;
  const int np = nc + (nc & 1);
  int buf = 0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rot = 0, big = 0;
    for (int t = 0; t < np - 1; ++t) {
      double *xb = buf ? xb1 : xb0;
      buf ^= 1;
#pragma unroll
      for (int i = 0; i < KR; ++i) xb[i * 64 + lane] = col[i];
      __syncthreads();
      const int q = rr_partner(lane, t, np);
      if (lane < nc && q < nc) {
        double y[KR];
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int i = 0; i < KR; ++i) {
          y[i] = xb[i * 64 + q];
          al += col[i] * col[i];
          be += y[i] * y[i];
          ga += col[i] * y[i];
        }
        // roles: the lower index is "p"
        const bool isp = lane < q;
        const double ap = isp ? al : be, aq = isp ? be : al;
        const bool live = jacobi_live(ap, aq);
        big |= live && (ga * ga > kJacobiStop2 * (ap * aq));
        if (live && ga != 0.0 && fabs(ga) > jacobi_tau(kr) * sqrt(ap * aq)) {
          const double zeta = (aq - ap) / (2.0 * ga);
          const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
          if (isp) {
#pragma unroll
            for (int i = 0; i < KR; ++i) col[i] = cs * col[i] - sn * y[i];
          } else {
#pragma unroll
            for (int i = 0; i < KR; ++i) col[i] = sn * y[i] + cs * col[i];
          }
          rot = 1;
        }
      }
    }
    const int any_big = __syncthreads_or(big);
    if (!__syncthreads_or(rot) || !any_big) break;
  }
  // final columns to xb0, R to xb1, column norms
  double s2 = 0.0;
#pragma unroll
  for (int i = 0; i < KR; ++i) {
    s2 += col[i] * col[i];
    xb0[i * 64 + lane] = col[i];
  }
  for (int e = lane; e < kr * nc; e += 64) xb1[e] = R[e];
  sig[lane] = (lane < nc) ? jacobi_sigma(s2) : -1.0;
  __syncthreads();
  if (lane < nc) {
    int rk = 0;
    const double sc = sig[lane];
    for (int j = 0; j < nc; ++j) rk += (sig[j] > sc) || (sig[j] == sc && j < lane);
    perm[rk] = lane;
    sigs[rk] = sc;
  }
  __syncthreads();
  if (lane == 0) s_rho = choose_rank(sigs, kr, nc, a, p);
  __syncthreads();
  const int rho = s_rho;
  double *U = a.u + p * a.ubs;
  for (int e = lane; e < kr * a.ucap; e += 64) {
    const int r = e / a.ucap, j = e - r * a.ucap;
    double v = 0.0;
    if (j < rho) {
      const double sc = sigs[j];
      v = (sc > 0.0) ? xb0[r * 64 + perm[j]] / sc : 0.0;
    }
    U[e] = v;
  }
  // S V^T rows = U_rho^T R
  double *S = a.svt + p * a.sbs;
  for (int e = lane; e < a.ucap * nc; e += 64) {
    const int j = e / nc, c = e - j * nc;
    double v = 0.0;
    if (j < rho) {
      const double sc = sigs[j];
      if (sc > 0.0) {
        const int cj = perm[j];
        for (int r = 0; r < kr; ++r) v += xb0[r * 64 + cj] * xb1[r * nc + c];
        v *= 1.0 / sc;
      }
    }
    S[e] = v;
  }
}

namespace {
template <int KR>
hipError_t svd_wave_launch(const SvdArgs &a, hipStream_t s) {
  const size_t lds = (size_t)(2 * KR * 64) * sizeof(double);
  static std::once_flag attr_done;
  std::call_once(attr_done, [&] {
    hipFuncSetAttribute((const void *)svd_wave_kernel<KR>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  });
  svd_wave_kernel<KR><<<a.batch, 64, lds, s>>>(a);
  return hipGetLastError();
}
}  // namespace

constexpr int kBlockThreads = 1024;

// One workgroup of kBlockThreads per matrix (64 < nc <= kSvdMaxN, the matrix
// in LDS): up to 16 lanes per column pair, so a rotation step takes a few rows
// per lane.  Writes sigma order, rank and U; S V^T = U^T R is the caller's
// GEMM.
__global__ __launch_bounds__(kBlockThreads) void svd_block_kernel(SvdArgs a, int tpg) {
  extern __shared__ double A[];  // A[c * kr + r]
  __shared__ double sig[kSvdMaxN];
  __shared__ double sigs[kSvdMaxN];
  __shared__ int perm[kSvdMaxN];
  __shared__ int s_rot, s_big;
  __shared__ int s_rho;
  const int kr = a.kr, nc = a.nc;
  const int tid = threadIdx.x;
  const int p = blockIdx.x;
  const double *R = a.r + p * a.rbs;
  for (int e = tid; e < kr * nc; e += kBlockThreads) {
    int r = e / nc, c = e - r * nc;
    A[c * kr + r] = R[e];
  }
  const int np = nc + (nc & 1);
  const int npairs = np / 2;
  const int grp = tid / tpg, gl = tid % tpg;
  const double thr = jacobi_tau(kr);
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) {
      s_rot = 0;
      s_big = 0;
    }
    __syncthreads();
    int myrot = 0, mybig = 0;
    for (int t = 0; t < np - 1; ++t) {
      if (grp < npairs) {
        const int pa = grp, pb = np - 1 - grp;
        int ip = (pa == 0) ? 0 : 1 + (pa - 1 + t) % (np - 1);
        int iq = 1 + (pb - 1 + t) % (np - 1);
        if (ip > iq) { int tmp = ip; ip = iq; iq = tmp; }
        if (iq < nc) {
          double *ap = A + ip * kr, *aq = A + iq * kr;
          double al = 0.0, be = 0.0, ga = 0.0;
          for (int r = gl; r < kr; r += tpg) {
            const double x = ap[r], y = aq[r];
            al += x * x;
            be += y * y;
            ga += x * y;
          }
          for (int off = tpg / 2; off > 0; off >>= 1) {
            al += __shfl_xor(al, off, tpg);
            be += __shfl_xor(be, off, tpg);
            ga += __shfl_xor(ga, off, tpg);
          }
          const bool live = jacobi_live(al, be);
          mybig |= live && (ga * ga > kJacobiStop2 * (al * be));
          if (live && ga != 0.0 && fabs(ga) > thr * sqrt(al * be)) {
            const double zeta = (be - al) / (2.0 * ga);
            const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
            for (int r = gl; r < kr; r += tpg) {
              const double x = ap[r], y = aq[r];
              ap[r] = cs * x - sn * y;
              aq[r] = sn * x + cs * y;
            }
            myrot = 1;
          }
        }
      }
      __syncthreads();
    }
    if (myrot) s_rot = 1;
    if (mybig) s_big = 1;
    __syncthreads();
    if (s_rot == 0 || s_big == 0) break;
    __syncthreads();
  }
  for (int c = tid; c < nc; c += kBlockThreads) {
    double s2 = 0.0;
    for (int r = 0; r < kr; ++r) s2 += A[c * kr + r] * A[c * kr + r];
    sig[c] = jacobi_sigma(s2);
  }
  __syncthreads();
  for (int c = tid; c < nc; c += kBlockThreads) {
    int rk = 0;
    const double sc = sig[c];
    for (int j = 0; j < nc; ++j) rk += (sig[j] > sc) || (sig[j] == sc && j < c);
    perm[rk] = c;
    sigs[rk] = sc;
  }
  __syncthreads();
  if (tid == 0) s_rho = choose_rank(sigs, kr, nc, a, p);
  __syncthreads();
  const int rho = s_rho;
  double *U = a.u + p * a.ubs;
  for (int e = tid; e < kr * a.ucap; e += kBlockThreads) {
    int r = e / a.ucap, j = e - r * a.ucap;
    double v = 0.0;
    if (j < rho) {
      const int c = perm[j];
      const double sc = sigs[j];
      v = (sc > 0.0) ? A[c * kr + r] / sc : 0.0;
    }
    U[e] = v;
  }
}

// ---------------------------------------------------------------------------
// Block one-sided Jacobi in registers (64 < nc <= 128, kr <= 128), one
// workgroup per matrix.  A column is held by a group of LPC lanes (8 or 16),
// so a wave holds CB = 64 / LPC columns of each of two blocks.  Columns are
// grouped in blocks of CB (nb blocks, padded with zero columns to an even
// count); wave w holds the block pair (top[w], bot[w]): lane group g (lanes
// LPC g .. LPC g + LPC - 1) holds column g of each block, lane t of the group
// the rows t + LPC s.  A sweep is
//   * the pairs inside every block: CB - 1 rounds pairing columns g and g ^ x
//     of the same block (both lane groups form the same dot products from
//     the same products in the same order, hence the same rotation);
//   * the pairs across blocks: nb' - 1 block rounds of the circle order
//     (top[0] fixed, the others move one position), in each of which the
//     bot block's columns pass the top block's CB lane groups in CB steps (a
//     shift by one lane group), so every top column meets every bot column
//     once; the blocks move between waves through LDS.
// A pair is rotated under the same test as the other Jacobi kernels.  The
// sums over the lanes of a group use DPP (quad permutes, row half mirror,
// and for 16 lanes the row mirror).
namespace {
template <int CTRL>
__device__ __forceinline__ double svd_dpp(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int LPC>
__device__ __forceinline__ double gsum(double v) {
  v += svd_dpp<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += svd_dpp<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += svd_dpp<0x141>(v);  // row_half_mirror: quads 0 <-> 1 of each 8 lanes
  if (LPC == 16) v += svd_dpp<0x140>(v);  // row_mirror: halves of each 16 lanes
  return v;
}
// 1/x and 1/sqrt(x) from the hardware estimates with Newton steps (the
// estimates are accurate to about 2^-26 relative; each step squares the
// relative error): x > 0, finite.
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}
// Rotation of the pair (x, y) (x plays "p"); returns whether it rotated.
// The rotation is c = 1/sqrt(1+t^2), s = c t, so c^2 + s^2 = 1 to rounding
// whatever the accuracy of t (t only steers convergence).
template <int RPT>
__device__ __forceinline__ bool jrot(double (&x)[RPT], double (&y)[RPT], double al, double be, double ga, double thr) {
  if (ga == 0.0 || !jacobi_live(al, be) || !(ga * ga > (thr * thr) * (al * be))) return false;
  const double zeta = (be - al) * (0.5 * rcp_nr(ga));
  double tt;
  if (fabs(zeta) < 1e150) {
    const double q = fma(zeta, zeta, 1.0);
    const double den = fabs(zeta) + q * rsq_nr(q);  // |zeta| + sqrt(1 + zeta^2)
    tt = (zeta >= 0.0 ? 1.0 : -1.0) * rcp_nr(den);
  } else {
    // t = 1 / (2 zeta) to rounding; none at all for an overflowed zeta
    tt = isfinite(zeta) ? 0.5 * rcp_nr(zeta) : 0.0;
  }
  const double cs = rsq_nr(fma(tt, tt, 1.0)), sn = cs * tt;
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const double u = x[s], v = y[s];
    x[s] = cs * u - sn * v;
    y[s] = sn * u + cs * v;
  }
  return true;
}
}  // namespace

template <int LPC, int RPT>
__global__ __launch_bounds__(LPC * 64) void svd_bj_kernel(SvdArgs a) {
  constexpr int CB = 64 / LPC;  // columns per block
  extern __shared__ double slots[];  // 2 h blocks of CB columns x kr rows: [top 0..h-1 | bot 0..h-1]
  __shared__ double sig[kSvdMaxN];
  __shared__ double sigs[kSvdMaxN];
  __shared__ int perm[kSvdMaxN];
  __shared__ int s_rot, s_big;
  __shared__ int s_rho;
  const int kr = a.kr, nc = a.nc;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane / LPC, t = lane % LPC;
  const int nt = blockDim.x;
  const int p = blockIdx.x;
  const double *R = a.r + p * a.rbs;
  int nb = (nc + CB - 1) / CB;
  nb += nb & 1;
  const int h = nb / 2;
  const bool act = w < h;
  const double thr = jacobi_tau(kr);
  const int bsz = CB * kr;  // doubles per block slot
  double tv[RPT], bv[RPT];
  // initial blocks: top[w] = block w, bot[w] = block nb - 1 - w
  {
    const int ct = CB * w + g, cb = CB * (nb - 1 - w) + g;
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = t + LPC * s;
      tv[s] = (act && r < kr && ct < nc) ? R[r * nc + ct] : 0.0;
      bv[s] = (act && r < kr && cb < nc) ? R[r * nc + cb] : 0.0;
    }
  }
  // A sweep in which no pair had cos^2 above kJacobiStop2 rotated by
  // angles whose squares are below rounding: by the quadratic convergence of
  // cyclic Jacobi the next sweep would find nothing, so it is not run.
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) {
      s_rot = 0;
      s_big = 0;
    }
    int rot = 0, big = 0;
    if (act) {
      // pairs inside each block
      for (int x = 1; x < CB; ++x) {
        const bool isp = g < (g ^ x);
        double pt[RPT], pb[RPT];
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
          pt[s] = __shfl_xor(tv[s], LPC * x);
          pb[s] = __shfl_xor(bv[s], LPC * x);
        }
        double a1 = 0.0, b1 = 0.0, g1 = 0.0, a2 = 0.0, b2 = 0.0, g2 = 0.0;
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
          const double lo1 = isp ? tv[s] : pt[s], hi1 = isp ? pt[s] : tv[s];
          const double lo2 = isp ? bv[s] : pb[s], hi2 = isp ? pb[s] : bv[s];
          a1 += lo1 * lo1;
          b1 += hi1 * hi1;
          g1 += lo1 * hi1;
          a2 += lo2 * lo2;
          b2 += hi2 * hi2;
          g2 += lo2 * hi2;
        }
        a1 = gsum<LPC>(a1);
        b1 = gsum<LPC>(b1);
        g1 = gsum<LPC>(g1);
        a2 = gsum<LPC>(a2);
        b2 = gsum<LPC>(b2);
        g2 = gsum<LPC>(g2);
        big |= (jacobi_live(a1, b1) && g1 * g1 > kJacobiStop2 * (a1 * b1)) |
               (jacobi_live(a2, b2) && g2 * g2 > kJacobiStop2 * (a2 * b2));
        // each lane group updates only its own column of the pair
        if (isp) {
          rot |= jrot<RPT>(tv, pt, a1, b1, g1, thr);
          rot |= jrot<RPT>(bv, pb, a2, b2, g2, thr);
        } else {
          rot |= jrot<RPT>(pt, tv, a1, b1, g1, thr);
          rot |= jrot<RPT>(pb, bv, a2, b2, g2, thr);
        }
      }
    }
    for (int br = 0; br < nb - 1; ++br) {
      if (act) {
        for (int st = 0; st < CB; ++st) {
          double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
          for (int s = 0; s < RPT; ++s) {
            al += tv[s] * tv[s];
            be += bv[s] * bv[s];
            ga += tv[s] * bv[s];
          }
          al = gsum<LPC>(al);
          be = gsum<LPC>(be);
          ga = gsum<LPC>(ga);
          big |= jacobi_live(al, be) && (ga * ga > kJacobiStop2 * (al * be));
          rot |= jrot<RPT>(tv, bv, al, be, ga, thr);
          // the bot columns move on to the next lane group
#pragma unroll
          for (int s = 0; s < RPT; ++s) bv[s] = __shfl(bv[s], (lane + LPC) & 63);
        }
        // circle order: publish both blocks
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
          const int r = t + LPC * s;
          if (r < kr) {
            slots[w * bsz + g * kr + r] = tv[s];
            slots[(h + w) * bsz + g * kr + r] = bv[s];
          }
        }
      }
      __syncthreads();
      if (act) {
        const int st = (w == 0) ? 0 : (w == 1 ? h : w - 1);   // new top: top[0] stays, top[1] <- bot[0]
        const int sb = (w == h - 1) ? (h - 1) : (h + w + 1);  // new bot: bot[h-1] <- top[h-1]
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
          const int r = t + LPC * s;
          tv[s] = (r < kr) ? slots[st * bsz + g * kr + r] : 0.0;
          bv[s] = (r < kr) ? slots[sb * bsz + g * kr + r] : 0.0;
        }
      }
      __syncthreads();
    }
    if (rot) s_rot = 1;
    if (big) s_big = 1;
    __syncthreads();
    if (s_rot == 0 || s_big == 0) break;
    __syncthreads();
  }
  // final columns into the slots (column index CB * slot + g), norms, order
  double *A = slots;  // column c at A + c * kr
  if (act) {
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = t + LPC * s;
      if (r < kr) {
        A[(CB * w + g) * kr + r] = tv[s];
        A[(CB * (h + w) + g) * kr + r] = bv[s];
      }
    }
  }
  __syncthreads();
  const int ncp = CB * nb;
  for (int c = tid; c < ncp; c += nt) {
    double s2 = 0.0;
    for (int r = 0; r < kr; ++r) s2 += A[c * kr + r] * A[c * kr + r];
    sig[c] = jacobi_sigma(s2);
  }
  __syncthreads();
  for (int c = tid; c < ncp; c += nt) {
    int rk = 0;
    const double sc = sig[c];
    for (int j = 0; j < ncp; ++j) rk += (sig[j] > sc) || (sig[j] == sc && j < c);
    perm[rk] = c;
    sigs[rk] = sc;
  }
  __syncthreads();
  if (tid == 0) s_rho = choose_rank(sigs, kr, nc, a, p);
  __syncthreads();
  const int rho = s_rho;
  double *U = a.u + p * a.ubs;
  for (int e = tid; e < kr * a.ucap; e += nt) {
    const int r = e / a.ucap, j = e - r * a.ucap;
    double v = 0.0;
    if (j < rho) {
      const int c = perm[j];
      const double sc = sigs[j];
      v = (sc > 0.0) ? A[c * kr + r] / sc : 0.0;
    }
    U[e] = v;
  }
}

hipError_t launch_svd_trunc(const SvdArgs &a, hipStream_t s) {
  if (a.batch <= 0) return hipSuccess;
  if (a.kr > a.nc || a.kr < 1) return hipErrorInvalidValue;
  if (a.nc <= 64) {
    if (a.kr <= 16) return svd_wave_launch<16>(a, s);
    if (a.kr <= 32) return svd_wave_launch<32>(a, s);
    if (a.kr <= 40) return svd_wave_launch<40>(a, s);
    if (a.kr <= 48) return svd_wave_launch<48>(a, s);
    return svd_wave_launch<64>(a, s);
  }
  if (a.nc <= 128 && a.kr <= 128) {
    // register block Jacobi: the slots hold the whole (padded) matrix; 8
    // lanes per column (blocks of 8 columns, 512 threads), 8, 12 or 16 rows
    // per lane.  (16 lanes per column, with blocks of 4 and twice the waves,
    // measured slower at 128 rows: twice the block rounds and barriers for
    // the same shuffle traffic.)
    static std::once_flag attr_bj;
    std::call_once(attr_bj, [&] {
      const int mx = (int)(128 * 128 * sizeof(double));
      hipFuncSetAttribute((const void *)svd_bj_kernel<8, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
      hipFuncSetAttribute((const void *)svd_bj_kernel<8, 12>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
      hipFuncSetAttribute((const void *)svd_bj_kernel<8, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    });
    int nb = (a.nc + 7) / 8;
    nb += nb & 1;
    const size_t lds = (size_t)nb * 8 * a.kr * sizeof(double);
    if (a.kr <= 64) svd_bj_kernel<8, 8><<<a.batch, 512, lds, s>>>(a);
    else if (a.kr <= 96) svd_bj_kernel<8, 12><<<a.batch, 512, lds, s>>>(a);
    else svd_bj_kernel<8, 16><<<a.batch, 512, lds, s>>>(a);
    return hipGetLastError();
  }
  if (a.nc > kSvdMaxN || (int64_t)a.nc * a.kr > kQrLdsDoubles) return hipErrorInvalidValue;
  const int np = a.nc + (a.nc & 1);
  const int npairs = np / 2;
  int tpg = 16;
  while (tpg > 1 && tpg * npairs > kBlockThreads) tpg >>= 1;
  const size_t lds = (size_t)a.nc * a.kr * sizeof(double);
  static std::once_flag attr_done;  // set once: the maximum a launch may ask for
  std::call_once(attr_done, [&] {
    hipFuncSetAttribute((const void *)svd_block_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)(kQrLdsDoubles * sizeof(double)));
  });
  svd_block_kernel<<<a.batch, kBlockThreads, lds, s>>>(a, tpg);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Block one-sided Jacobi for nc > kSvdMaxN.  Columns are grouped in blocks of
// bw; a round pairs blocks with the circle order and every workgroup fully
// orthogonalises the columns of its two blocks against each other (an inner
// one-sided Jacobi on <= 2 bw columns held in LDS).  A sweep over all block
// pairs that rotates nothing ends the iteration (flags).
int svd_big_block_width(int kr) {
  int bw = kQrLdsDoubles / (2 * std::max(kr, 1));
  if (bw > 32) bw = 32;
  return bw;
}

__global__ void svd_big_prepare_kernel(const double *r, int64_t rbs, int kr, int nc, double *acol, int64_t acs,
                                       int *flags, int batch) {
  const int64_t per = (int64_t)kr * nc, total = per * batch;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / per, rem = e - p * per;
    const int64_t rr = rem / nc, c = rem - rr * nc;
    acol[p * acs + c * kr + rr] = r[p * rbs + rem];
  }
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < 2 * batch) flags[t] = 0;
}

hipError_t launch_svd_big_prepare(const double *r, int64_t rbs, int kr, int nc, double *acol, int64_t acs,
                                  int *flags, int batch, hipStream_t s) {
  const int64_t total = std::max<int64_t>((int64_t)kr * nc * batch, 2 * batch);
  int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  svd_big_prepare_kernel<<<grid, 256, 0, s>>>(r, rbs, kr, nc, acol, acs, flags, batch);
  return hipGetLastError();
}

constexpr int kBigInnerSweeps = 1;

constexpr int kBigRoundThreads = 1024;

__global__ __launch_bounds__(kBigRoundThreads) void svd_big_round_kernel(double *acol, int64_t acs, int kr, int nc, int bw,
                                                            int nb, int t, int *flags) {
  extern __shared__ double A[];  // w columns of length kr
  __shared__ int s_any, s_rot;
  const int p = blockIdx.y;
  if (flags[2 * p + 1]) return;
  const int tid = threadIdx.x;
  const int m = nb - 1;
  const int pa = blockIdx.x, pb = nb - 1 - blockIdx.x;
  const int ba = (pa == 0) ? 0 : 1 + (pa - 1 + t) % m;
  const int bb = 1 + (pb - 1 + t) % m;
  const int a0 = ba * bw, a1 = min(nc, a0 + bw);
  const int b0 = bb * bw, b1 = min(nc, b0 + bw);
  const int wa = max(0, a1 - a0), wb = max(0, b1 - b0);
  const int w = wa + wb;
  if (w < 2) return;
  double *base = acol + p * acs;
  for (int e = tid; e < w * kr; e += kBigRoundThreads) {
    const int c = e / kr, r = e - c * kr;
    const int gc = (c < wa) ? a0 + c : b0 + (c - wa);
    A[e] = base[(int64_t)gc * kr + r];
  }
  if (tid == 0) s_any = 0;
  const int np = w + (w & 1);
  const int npairs = np / 2;
  // up to a full wave per column pair: the pair's dot products and rotation
  // then take few steps per lane and the block has enough waves to hide
  // the LDS latency
  int tpg = 64;
  while (tpg > 1 && tpg * npairs > kBigRoundThreads) tpg >>= 1;
  const double thr = jacobi_tau(kr);
  const int grp = tid / tpg, gl = tid % tpg;
  int mybig = 0;
  __syncthreads();
  // one cyclic sweep over the pairs of the two blocks per round: every
  // outer sweep is then at least one full cyclic Jacobi sweep over all
  // column pairs, and convergence is judged by the outer sweeps
  for (int sweep = 0; sweep < kBigInnerSweeps; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    int myrot = 0;
    for (int tt = 0; tt < np - 1; ++tt) {
      if (grp < npairs) {
        const int qa = grp, qb = np - 1 - grp;
        int ip = (qa == 0) ? 0 : 1 + (qa - 1 + tt) % (np - 1);
        int iq = 1 + (qb - 1 + tt) % (np - 1);
        if (ip > iq) { int tmp = ip; ip = iq; iq = tmp; }
        if (iq < w) {
          double *ap = A + ip * kr, *aq = A + iq * kr;
          double al = 0.0, be = 0.0, ga = 0.0;
          for (int r = gl; r < kr; r += tpg) {
            const double x = ap[r], y = aq[r];
            al += x * x;
            be += y * y;
            ga += x * y;
          }
          for (int off = tpg / 2; off > 0; off >>= 1) {
            al += __shfl_xor(al, off, tpg);
            be += __shfl_xor(be, off, tpg);
            ga += __shfl_xor(ga, off, tpg);
          }
          const bool live = jacobi_live(al, be);
          if (live && ga * ga > kJacobiStop2 * (al * be)) mybig = 1;
          if (live && ga != 0.0 && fabs(ga) > thr * sqrt(al * be)) {
            const double zeta = (be - al) / (2.0 * ga);
            const double t2 = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + t2 * t2), sn = cs * t2;
            for (int r = gl; r < kr; r += tpg) {
              const double x = ap[r], y = aq[r];
              ap[r] = cs * x - sn * y;
              aq[r] = sn * x + cs * y;
            }
            myrot = 1;
          }
        }
      }
      __syncthreads();
    }
    if (myrot) s_rot = 1;
    __syncthreads();
    if (s_rot == 0) break;
    if (tid == 0) s_any = 1;
    __syncthreads();
  }
  for (int e = tid; e < w * kr; e += kBigRoundThreads) {
    const int c = e / kr, r = e - c * kr;
    const int gc = (c < wa) ? a0 + c : b0 + (c - wa);
    base[(int64_t)gc * kr + r] = A[e];
  }
  // bit 0: this round rotated; bit 1: some pair had a squared cosine above
  // the early-stop level
  if (tid == 0 && s_any) atomicOr(flags + 2 * p, 1);
  if (mybig) atomicOr(flags + 2 * p, 2);
}

hipError_t launch_svd_big_round(double *acol, int64_t acs, int kr, int nc, int bw, int nb, int t, int *flags,
                                int batch, hipStream_t s) {
  const size_t lds = (size_t)2 * bw * kr * sizeof(double);
  static std::once_flag attr_done;  // set once: the maximum a launch may ask for
  std::call_once(attr_done, [&] {
    hipFuncSetAttribute((const void *)svd_big_round_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)(kQrLdsDoubles * sizeof(double)));
  });
  svd_big_round_kernel<<<dim3((unsigned)(nb / 2), (unsigned)batch), kBigRoundThreads, lds, s>>>(acol, acs, kr, nc, bw, nb, t,
                                                                                 flags);
  return hipGetLastError();
}

__global__ void svd_big_sweep_end_kernel(int *flags, int batch) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < batch) {
    if (flags[2 * p] == 0 || (flags[2 * p] & 2) == 0) flags[2 * p + 1] = 1;
    flags[2 * p] = 0;
  }
}

hipError_t launch_svd_big_sweep_end(int *flags, int batch, hipStream_t s) {
  svd_big_sweep_end_kernel<<<(batch + 255) / 256, 256, 0, s>>>(flags, batch);
  return hipGetLastError();
}

// Singular values are the column norms of the rotated matrix A V = U S.
// This kernel sorts them, chooses the rank and writes U (kr x ucap, zero
// beyond the kept rank); S V^T = U^T R is a GEMM the caller issues next.
__global__ __launch_bounds__(256) void svd_big_finish_kernel(SvdArgs a, const double *acol, int64_t acs) {
  __shared__ double sig[kSvdBigMaxN];
  __shared__ double sigs[kSvdBigMaxN];
  __shared__ int perm[kSvdBigMaxN];
  __shared__ int s_rho;
  const int kr = a.kr, nc = a.nc;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int p = blockIdx.x;
  const double *A = acol + p * acs;
  for (int c = wv; c < nc; c += 4) {  // one wave per column, coalesced
    const double *col = A + (int64_t)c * kr;
    double s2 = 0.0;
    for (int r = lane; r < kr; r += 64) s2 += col[r] * col[r];
    for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off);
    if (lane == 0) sig[c] = jacobi_sigma(s2);
  }
  __syncthreads();
  for (int c = tid; c < nc; c += 256) {
    int rk = 0;
    const double sc = sig[c];
    for (int j = 0; j < nc; ++j) rk += (sig[j] > sc) || (sig[j] == sc && j < c);
    perm[rk] = c;
    sigs[rk] = sc;
  }
  __syncthreads();
  if (tid == 0) s_rho = choose_rank(sigs, kr, nc, a, p);
  __syncthreads();
  const int rho = s_rho;
  double *U = a.u + p * a.ubs;
  for (int e = tid; e < kr * a.ucap; e += 256) {
    const int r = e / a.ucap, j = e - r * a.ucap;
    double v = 0.0;
    if (j < rho) {
      const double sc = sigs[j];
      v = (sc > 0.0) ? A[(int64_t)perm[j] * kr + r] / sc : 0.0;
    }
    U[e] = v;
  }
}

hipError_t launch_svd_big_finish(const SvdArgs &a, const double *acol, int64_t acs, hipStream_t s) {
  if (a.nc > kSvdBigMaxN) return hipErrorInvalidValue;
  svd_big_finish_kernel<<<a.batch, 256, 0, s>>>(a, acol, acs);
  return hipGetLastError();
}

}  // namespace hatt
