// Batched, strided FP64 GEMM on the CDNA matrix cores
// (v_mfma_f64_16x16x4_f64), with an optional deterministic split-K.
//
// Tile: 64 x 64 outputs per 256-thread workgroup, K staged through LDS in
// slabs of 16.  Each of the 4 waves owns a 32 x 32 quadrant = 2 x 2 MFMA
// blocks of 16 x 16; one MFMA consumes a 16 x 4 slice of A and a 4 x 16 slice
// of B, one double per lane each (lane l holds A(l%16, l/16) and
// B(l/16, l%16)); its 16 x 16 result sits 4 doubles per lane, lane l holding
// rows l/16 + 4v, v = 0..3, of column l%16 (rows interleaved by 4, checked
// on gfx950 with a one-wave probe).
// Operand tiles are loaded with the thread mapping that makes the unit-stride
// dimension of each operand contiguous across lanes.
#include "common.h"

namespace hatt {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, LDA_S = BM + 1, LDB_S = BN + 1;

__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmArgs g) {
  __shared__ double As[BK * LDA_S];  // As[k * LDA_S + m]
  __shared__ double Bs[BK * LDB_S];  // Bs[k * LDB_S + n]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int64_t m0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
  const int ks = g.ksplit;
  const int p = blockIdx.z / ks, kc = blockIdx.z - (blockIdx.z / ks) * ks;
  int64_t kchunk = (g.K + ks - 1) / ks;
  kchunk = ((kchunk + BK - 1) / BK) * BK;
  const int64_t kbeg = kc * kchunk;
  const int64_t kend = std::min<int64_t>(g.K, kbeg + kchunk);

  const double *Ab = g.A.ptr + p * g.A.bs;
  const double *Bb = g.B.ptr + p * g.B.bs;
  const bool a_kfast = (g.A.cs == 1);
  const bool b_nfast = (g.B.cs == 1) || (g.B.rs != 1);

  d4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      int mm, kk;
      if (a_kfast) { kk = e & 15; mm = e >> 4; }
      else { mm = e & 63; kk = e >> 6; }
      const int64_t gm = m0 + mm, gk = k0 + kk;
      double v = 0.0;
      if (gm < g.M && gk < kend) v = Ab[gm * g.A.rs + gk * g.A.cs];
      As[kk * LDA_S + mm] = v;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      int nn, kk;
      if (b_nfast) { nn = e & 63; kk = e >> 6; }
      else { kk = e & 15; nn = e >> 4; }
      const int64_t gn = n0 + nn, gk = k0 + kk;
      double v = 0.0;
      if (gn < g.N && gk < kend) v = Bb[gk * g.B.rs + gn * g.B.cs];
      Bs[kk * LDB_S + nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4), c16 = lane & 15;
      double av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = As[kr * LDA_S + wm + i * 16 + c16];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = Bs[kr * LDB_S + wn + j * 16 + c16];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  const int rq = lane >> 4, cq = lane & 15;
  if (ks == 1) {
    double *Cb = g.C.ptr + p * g.C.bs;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t gm = m0 + wm + i * 16 + rq + 4 * v, gn = n0 + wn + j * 16 + cq;
          if (gm < g.M && gn < g.N) {
            double *cp = Cb + gm * g.C.rs + gn * g.C.cs;
            double r = g.alpha * acc[i][j][v];
            if (g.beta != 0.0) r += g.beta * (*cp);
            *cp = r;
          }
        }
  } else {
    double *Pb = g.part + ((int64_t)p * ks + kc) * g.M * g.N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t gm = m0 + wm + i * 16 + rq + 4 * v, gn = n0 + wn + j * 16 + cq;
          if (gm < g.M && gn < g.N) Pb[gm * g.N + gn] = g.alpha * acc[i][j][v];
        }
  }
}

// Sum of the ksplit partial products in chunk order (bitwise reproducible).
__global__ void splitk_reduce_kernel(GemmArgs g) {
  const int64_t per = g.M * g.N, total = per * g.batch;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / per, rem = e - p * per;
    const int64_t r = rem / g.N, c = rem - r * g.N;
    const double *src = g.part + p * g.ksplit * per + rem;
    double acc = 0.0;
    for (int t = 0; t < g.ksplit; ++t) acc += src[t * per];
    double *cp = g.C.ptr + p * g.C.bs + r * g.C.rs + c * g.C.cs;
    if (g.beta != 0.0) acc += g.beta * (*cp);
    *cp = acc;
  }
}

int gemm_pick_ksplit(int64_t M, int64_t N, int64_t K, int batch) {
  const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN) * (int64_t)batch;
  int ks = 1;
  // aim for ~2 workgroups per CU while keeping >= 4 K slabs per chunk
  while (tiles * ks < 512 && K / ((int64_t)(ks * 2) * BK) >= 4 && ks < 64) ks *= 2;
  return ks;
}

hipError_t launch_gemm(const GemmArgs &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  GemmArgs a = g;
  if (a.K <= 0) {
    // C = beta C
    a.ksplit = 1;
  }
  if (a.ksplit < 1) a.ksplit = 1;
  if (a.ksplit > 1 && a.part == nullptr) a.ksplit = 1;
  dim3 grid((unsigned)((a.M + BM - 1) / BM), (unsigned)((a.N + BN - 1) / BN),
            (unsigned)(a.batch * a.ksplit));
  gemm_f64_kernel<<<grid, 256, 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.ksplit == 1) return e;
  const int64_t total = a.M * a.N * a.batch;
  int rg = (int)std::min<int64_t>((total + 255) / 256, 65536);
  splitk_reduce_kernel<<<rg, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace hatt
