// Small dense SVD by one-sided (Hestenes) Jacobi, one workgroup per matrix,
// followed by the truncation-rank choice of TT-Rounding.
//
// The kr x nc matrix is held column-major in LDS together with V (nc x nc).
// A sweep visits every column pair once using the round-robin (circle)
// ordering: nc' - 1 rounds (nc' = nc rounded up to even) of nc'/2 disjoint
// pairs, each pair handled by a group of lanes inside one wavefront, so the
// three inner products of a pair reduce with cross-lane shuffles.  A pair is
// rotated when |a_p . a_q| > 1e-15 ||a_p|| ||a_q||; sweeps stop when no pair
// needs rotating.  On exit A V^T-rotation gives A_final = R V with orthogonal
// columns, sigma_j = ||A_final(:, j)||, U(:, j) = A_final(:, j) / sigma_j, so
// U diag(sigma) V^T reproduces R exactly up to rounding even for zero or tiny
// sigma_j.
#include "common.h"

namespace hatt {

__global__ __launch_bounds__(256) void svd_trunc_kernel(SvdArgs a, int tpg) {
  extern __shared__ double sm[];
  const int kr = a.kr, nc = a.nc;
  double *A = sm;            // A[c * kr + r]
  double *V = A + nc * kr;   // V[c * nc + r]  (column c of V)
  __shared__ double sig[kSvdMaxN];
  __shared__ int perm[kSvdMaxN];
  __shared__ int s_rot;
  __shared__ int s_rho;
  const int tid = threadIdx.x;
  const int p = blockIdx.x;
  const double *R = a.r + p * a.rbs;
  for (int e = tid; e < kr * nc; e += 256) {
    int r = e / nc, c = e - r * nc;
    A[c * kr + r] = R[e];
  }
  for (int e = tid; e < nc * nc; e += 256) {
    int c = e / nc, r = e - c * nc;
    V[e] = (r == c) ? 1.0 : 0.0;
  }
  const int np = nc + (nc & 1);
  const int npairs = np / 2;
  const int grp = tid / tpg, gl = tid % tpg;
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    int myrot = 0;
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
          if (ga != 0.0 && fabs(ga) > 1e-15 * sqrt(al * be)) {
            const double zeta = (be - al) / (2.0 * ga);
            const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
            for (int r = gl; r < kr; r += tpg) {
              const double x = ap[r], y = aq[r];
              ap[r] = cs * x - sn * y;
              aq[r] = sn * x + cs * y;
            }
            double *vp = V + ip * nc, *vq = V + iq * nc;
            for (int r = gl; r < nc; r += tpg) {
              const double x = vp[r], y = vq[r];
              vp[r] = cs * x - sn * y;
              vq[r] = sn * x + cs * y;
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
    __syncthreads();
  }
  // singular values and descending order (ties keep index order)
  for (int c = tid; c < nc; c += 256) {
    double s2 = 0.0;
    for (int r = 0; r < kr; ++r) s2 += A[c * kr + r] * A[c * kr + r];
    sig[c] = sqrt(s2);
  }
  __syncthreads();
  for (int c = tid; c < nc; c += 256) {
    int rk = 0;
    const double sc = sig[c];
    for (int j = 0; j < nc; ++j) rk += (sig[j] > sc) || (sig[j] == sc && j < c);
    perm[rk] = c;
  }
  __syncthreads();
  if (tid == 0) {
    double tot2 = 0.0;
    for (int j = 0; j < nc; ++j) tot2 += sig[j] * sig[j];
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
        const double sj = sig[perm[j]];
        tail += sj * sj;
        if (tail <= d2) rho = j;
        else break;
      }
    }
    if (a.cap > 0 && rho > a.cap) rho = (int)a.cap;
    if (rho > a.ucap) rho = a.ucap;
    if (rho < 1) rho = 1;
    s_rho = rho;
    a.rank_out[p * a.rank_bs] = rho;
  }
  __syncthreads();
  const int rho = s_rho;
  double *U = a.u + p * a.ubs;
  for (int e = tid; e < kr * a.ucap; e += 256) {
    int r = e / a.ucap, j = e - r * a.ucap;
    double v = 0.0;
    if (j < rho) {
      const int c = perm[j];
      const double sc = sig[c];
      v = (sc > 0.0) ? A[c * kr + r] / sc : 0.0;
    }
    U[e] = v;
  }
  double *S = a.svt + p * a.sbs;
  for (int e = tid; e < a.ucap * nc; e += 256) {
    int j = e / nc, col = e - j * nc;
    double v = 0.0;
    if (j < rho) {
      const int c = perm[j];
      v = sig[c] * V[c * nc + col];
    }
    S[e] = v;
  }
}

hipError_t launch_svd_trunc(const SvdArgs &a, hipStream_t s) {
  if (a.batch <= 0) return hipSuccess;
  if (a.nc > kSvdMaxN || a.kr > a.nc || a.kr < 1) return hipErrorInvalidValue;
  const int np = a.nc + (a.nc & 1);
  const int npairs = np / 2;
  int tpg = 64;
  while (tpg > 1 && tpg * npairs > 256) tpg >>= 1;
  const size_t lds = (size_t)(a.nc * a.kr + a.nc * a.nc) * sizeof(double);
  hipFuncSetAttribute((const void *)svd_trunc_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)lds);
  svd_trunc_kernel<<<a.batch, 256, lds, s>>>(a, tpg);
  return hipGetLastError();
}

}  // namespace hatt
