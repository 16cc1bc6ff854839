// Batched, strided FP64 GEMM on the CDNA matrix cores
// (v_mfma_f64_16x16x4_f64), with an optional deterministic split-K.
//
// Tile: 64 x 64 (or 64 x 32, 32 x 64, 32 x 32 for thin operands) outputs per
// 256-thread workgroup, K staged through LDS in slabs of 32.  Each of the 4
// waves owns a quadrant made of 16 x 16 MFMA blocks; one MFMA consumes a 16 x 4 slice of A and a 4 x 16 slice
// of B, one double per lane each (lane l holds A(l%16, l/16) and
// B(l/16, l%16)); its 16 x 16 result sits 4 doubles per lane, lane l holding
// rows l/16 + 4v, v = 0..3, of column l%16 (rows interleaved by 4, checked
// on gfx950 with a one-wave probe).
// Operand tiles are loaded with the thread mapping that makes the unit-stride
// dimension of each operand contiguous across lanes.
#include "common.h"
#include "stage.h"

namespace hatt {

constexpr int BK = 32;

// BM x BN output tile, 4 waves in a 2 x 2 grid, each wave (BM/2) x (BN/2) as
// (BM/32) x (BN/32) MFMA blocks of 16 x 16.  The next K slab is fetched into
// registers while the MFMAs consume the current one from LDS.  CT is the
// compute type (FP64 or FP32 matrix cores, FP32 accumulating in FP32); TA,
// TB, TC are the storage types of the operands (converted on load / store).
template <int BM, int BN, typename CT, typename TA, typename TB, typename TC, int WL = 0>
__device__ __forceinline__ void gemm_body(const GemmArgs &g) {
  using acc_t = typename std::conditional<std::is_same<CT, double>::value, d4_t, f4_t>::type;
  constexpr int LDA_S = BM + 1, LDB_S = BN + 1;
  // wave layout WL: 0 = 2 x 2 quadrants; 1 = four waves stacked along M
  // (each BM/4 rows x BN), for thin N; 2 = side by side along N, for thin M.
  // With a thin side whole 16-wide blocks are dead padding; these layouts
  // give every wave the same number of live blocks.
  static_assert(WL == 0 || (WL == 1 && BM == 64) || (WL == 2 && BN == 64), "wave layout");
  constexpr int MI = WL == 0 ? BM / 32 : (WL == 1 ? BM / 64 : BM / 16);
  constexpr int NJ = WL == 0 ? BN / 32 : (WL == 1 ? BN / 16 : BN / 64);
  constexpr int A_PER = BM * BK / 256, B_PER = BN * BK / 256;
  __shared__ CT As[BK * LDA_S];  // As[k * LDA_S + m]
  __shared__ CT Bs[BK * LDB_S];  // Bs[k * LDB_S + n]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = WL == 0 ? (wave >> 1) * (BM / 2) : (WL == 1 ? wave * (BM / 4) : 0);
  const int wn = WL == 0 ? (wave & 1) * (BN / 2) : (WL == 2 ? wave * (BN / 4) : 0);
  const int64_t m0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
  const int ks = g.ksplit;
  const int p = blockIdx.z / ks, kc = blockIdx.z - (blockIdx.z / ks) * ks;
  if (g.run_flag != nullptr && g.run_flag[p * g.run_flag_stride] != g.run_when) return;
  int64_t kchunk = (g.K + ks - 1) / ks;
  kchunk = ((kchunk + BK - 1) / BK) * BK;
  const int64_t kbeg = kc * kchunk;
  const int64_t kend = std::min<int64_t>(g.K, kbeg + kchunk);

  const TA *Ab = reinterpret_cast<const TA *>(static_cast<const void *>(g.A.ptr)) + p * g.A.bs;
  const TB *Bb = reinterpret_cast<const TB *>(static_cast<const void *>(g.B.ptr)) + p * g.B.bs;
  const bool a_kfast = (g.A.cs == 1);
  const bool b_nfast = (g.B.cs == 1) || (g.B.rs != 1);

  // Per-thread load slots t = 0..PER-1 are element tid + 256 t of the slab
  // tile; along the unit-stride dimension they share one index, so each
  // operand needs one base pointer and one per-slot stride.
  const int64_t rem0 = kend - kbeg;
  const TA *abase;
  const TB *bbase;
  int64_t astep, bstep;  // pointer distance between slots t and t + 1
  int a_lds0, a_ldsd, b_lds0, b_ldsd;
  int a_fix, a_var0, a_vard, a_lim, b_fix, b_var0, b_vard, b_lim;  // bound checks, see fetch
  if (a_kfast) {
    const int kk = tid % BK, mm = tid / BK;
    abase = Ab + (m0 + mm) * g.A.rs + (kbeg + kk) * g.A.cs;
    astep = (256 / BK) * g.A.rs;
    a_lds0 = kk * LDA_S + mm;
    a_ldsd = 256 / BK;
    a_fix = kk;                      // k index: fixed, checked against the slab's remaining K
    a_var0 = (int)std::min<int64_t>(m0 + mm, 1 << 30);
    a_vard = 256 / BK;               // m index grows with t
    a_lim = (int)std::min<int64_t>(g.M, 1 << 30);
  } else {
    const int mm = tid % BM, kk = tid / BM;
    abase = Ab + (m0 + mm) * g.A.rs + (kbeg + kk) * g.A.cs;
    astep = (256 / BM) * g.A.cs;
    a_lds0 = kk * LDA_S + mm;
    a_ldsd = (256 / BM) * LDA_S;
    a_fix = (m0 + mm < g.M) ? -1 : (1 << 30);  // -1: the m index is inside
    a_var0 = kk;
    a_vard = 256 / BM;               // k index grows with t
    a_lim = 0;
  }
  if (b_nfast) {
    const int nn = tid % BN, kk = tid / BN;
    bbase = Bb + (kbeg + kk) * g.B.rs + (n0 + nn) * g.B.cs;
    bstep = (256 / BN) * g.B.rs;
    b_lds0 = kk * LDB_S + nn;
    b_ldsd = (256 / BN) * LDB_S;
    b_fix = (n0 + nn < g.N) ? -1 : (1 << 30);
    b_var0 = kk;
    b_vard = 256 / BN;
    b_lim = 0;
  } else {
    const int kk = tid % BK, nn = tid / BK;
    bbase = Bb + (kbeg + kk) * g.B.rs + (n0 + nn) * g.B.cs;
    bstep = (256 / BK) * g.B.cs;
    b_lds0 = kk * LDB_S + nn;
    b_ldsd = 256 / BK;
    b_fix = kk;
    b_var0 = (int)std::min<int64_t>(n0 + nn, 1 << 30);
    b_vard = 256 / BK;
    b_lim = (int)std::min<int64_t>(g.N, 1 << 30);
  }
  (void)rem0;
  const int64_t a_kstep = BK * g.A.cs, b_kstep = BK * g.B.rs;
  CT ra[A_PER], rb[B_PER];
  // slot t is in range when: k-fast layout: fixed k < rem and m (n) < limit;
  // m-fast (n-fast) layout: the fixed m (n) is inside and k < rem.
  auto fetch = [&](int64_t k0, int64_t slab) {
    const int rem = (int)std::min<int64_t>(kend - k0, 1 << 30);
    const TA *pa = abase + slab * a_kstep;
    const TB *pb = bbase + slab * b_kstep;
#pragma unroll
    for (int t = 0; t < A_PER; ++t) {
      const int v = a_var0 + t * a_vard;
      const bool ok = a_kfast ? (a_fix < rem && v < a_lim) : (a_fix < 0 && v < rem);
      ra[t] = to_ct<CT>(ok ? (double)pa[t * astep] : 0.0);
    }
#pragma unroll
    for (int t = 0; t < B_PER; ++t) {
      const int v = b_var0 + t * b_vard;
      const bool ok = b_nfast ? (b_fix < 0 && v < rem) : (b_fix < rem && v < b_lim);
      rb[t] = to_ct<CT>(ok ? (double)pb[t * bstep] : 0.0);
    }
  };
  auto park = [&]() {
#pragma unroll
    for (int t = 0; t < A_PER; ++t) As[a_lds0 + t * a_ldsd] = ra[t];
#pragma unroll
    for (int t = 0; t < B_PER; ++t) Bs[b_lds0 + t * b_ldsd] = rb[t];
  };

  acc_t acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  if (kbeg < kend) {
    fetch(kbeg, 0);
    park();
  }
  __syncthreads();
  // 16 x 16 blocks of this wave that lie wholly in the padding beyond M or N
  // are skipped (their products are zero and never stored); so are the K
  // steps of a partial last slab past the valid K.  Both tests are uniform
  // across the wave.
  bool live_m[MI], live_n[NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i) live_m[i] = m0 + wm + i * 16 < g.M;
#pragma unroll
  for (int j = 0; j < NJ; ++j) live_n[j] = n0 + wn + j * 16 < g.N;
  // FP64 with a thin side (wave layouts 1 and 2): a last block of that side
  // with at most 8 live columns (rows) is formed as one or two 4-wide strips
  // by the four-block 4 x 4 x 4 MFMA (the wave's other operand fragment is
  // reused as is; the strip's operand is read replicated across the four
  // blocks) at a quarter of a 16 x 16 block's cost per strip.
  constexpr bool REM = std::is_same<CT, double>::value && WL != 0;
  int rem_blk = 0, rem_cnt = 0;  // wave-uniform
  double racc[2] = {0.0, 0.0};
  if constexpr (REM) {
    const int64_t edge = (WL == 1) ? g.N - n0 - wn : g.M - m0 - wm;
    if (edge > 0 && edge < 64 && (edge & 15) >= 1 && (edge & 15) <= 8) {
      rem_blk = (int)(edge >> 4);
      rem_cnt = (int)(((edge & 15) + 3) >> 2);
      if (WL == 1) {
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          if (j == rem_blk) live_n[j] = false;
      } else {
#pragma unroll
        for (int i = 0; i < MI; ++i)
          if (i == rem_blk) live_m[i] = false;
      }
    }
  }
  int64_t slab = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK, ++slab) {
    const bool more = k0 + BK < kend;
    if (more) fetch(k0 + BK, slab + 1);
    const int kval = (int)std::min<int64_t>(BK, kend - k0);
    if constexpr (is_bf16<CT>::value) {
      // BF16: one K-16 MFMA per block and 16 K values of the slab (the slab
      // is zero beyond the valid K)
#pragma unroll
      for (int kk = 0; kk < BK; kk += 16) {
        if (kk >= kval) break;
        const int q = lane >> 4, c16 = lane & 15;
        CT av[MI][4], bv[NJ][4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int kr = kk + 4 * e + q;
#pragma unroll
          for (int i = 0; i < MI; ++i) av[i][e] = As[kr * LDA_S + wm + i * 16 + c16];
#pragma unroll
          for (int j = 0; j < NJ; ++j) bv[j][e] = Bs[kr * LDB_S + wn + j * 16 + c16];
        }
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j)
            if (live_m[i] && live_n[j]) acc[i][j] = mfma16_bf16(av[i], bv[j], acc[i][j]);
      }
    } else {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      if (kk >= kval) break;
      const int kr = kk + (lane >> 4), c16 = lane & 15;
      CT av[MI], bv[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i) av[i] = As[kr * LDA_S + wm + i * 16 + c16];
#pragma unroll
      for (int j = 0; j < NJ; ++j) bv[j] = Bs[kr * LDB_S + wn + j * 16 + c16];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          if (live_m[i] && live_n[j]) acc[i][j] = mfma16(av[i], bv[j], acc[i][j]);
      if constexpr (REM) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (q < rem_cnt) {
            if (WL == 1) {
              const double x = (double)Bs[kr * LDB_S + wn + rem_blk * 16 + 4 * q + (lane & 3)];
              racc[q] = mfma4((double)av[0], x, racc[q]);
            } else {
              const double x = (double)As[kr * LDA_S + wm + rem_blk * 16 + 4 * q + (lane & 3)];
              racc[q] = mfma4(x, (double)bv[0], racc[q]);
            }
          }
        }
      }
    }
    }
    __syncthreads();
    if (more) {
      park();
      __syncthreads();
    }
  }

  const int rq = lane >> 4, cq = lane & 15;
  // strip q's result of this lane (row, column within the tile)
  auto rem_at = [&](int q, int64_t *gm, int64_t *gn) {
    if (WL == 1) {
      *gm = m0 + wm + 4 * ((lane >> 2) & 3) + rq;
      *gn = n0 + wn + rem_blk * 16 + 4 * q + (lane & 3);
    } else {
      *gm = m0 + wm + rem_blk * 16 + 4 * q + rq;
      *gn = n0 + wn + cq;
    }
  };
  if (ks == 1) {
    TC *Cb = reinterpret_cast<TC *>(static_cast<void *>(g.C.ptr)) + p * g.C.bs;
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t gm = m0 + wm + i * 16 + mfma_row<CT>(rq, v), gn = n0 + wn + j * 16 + cq;
          // a strip-formed block is stored by the strips alone
          if (live_m[i] && live_n[j] && gm < g.M && gn < g.N) {
            TC *cp = Cb + gm * g.C.rs + gn * g.C.cs;
            double r = g.alpha * (double)acc[i][j][v];
            if (g.beta != 0.0) r += g.beta * (double)(*cp);
            *cp = (TC)r;
          }
        }
    if constexpr (REM) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        int64_t gm, gn;
        rem_at(q, &gm, &gn);
        if (q < rem_cnt && gm < g.M && gn < g.N) {
          TC *cp = Cb + gm * g.C.rs + gn * g.C.cs;
          double r = g.alpha * racc[q];
          if (g.beta != 0.0) r += g.beta * (double)(*cp);
          *cp = (TC)r;
        }
      }
    }
  } else {  // split-K partials, FP64 whatever the compute type
    double *Pb = g.part + ((int64_t)p * ks + kc) * g.M * g.N;
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t gm = m0 + wm + i * 16 + mfma_row<CT>(rq, v), gn = n0 + wn + j * 16 + cq;
          if (live_m[i] && live_n[j] && gm < g.M && gn < g.N) Pb[gm * g.N + gn] = g.alpha * (double)acc[i][j][v];
        }
    if constexpr (REM) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        int64_t gm, gn;
        rem_at(q, &gm, &gn);
        if (q < rem_cnt && gm < g.M && gn < g.N) Pb[gm * g.N + gn] = g.alpha * racc[q];
      }
    }
  }
}

template <int BM, int BN, int WL>
__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmArgs g) {
  gemm_body<BM, BN, double, double, double, double, WL>(g);
}

// FP32 matrix cores, FP32 accumulation; operands stored as FP32 or FP64.
template <int BM, int BN, typename TA, typename TB, typename TC, int WL>
__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmArgs g) {
  gemm_body<BM, BN, float, TA, TB, TC, WL>(g);
}

// BF16 matrix cores, FP32 accumulation; operands stored as FP32 or FP64 and
// rounded to BF16 when staged.
template <int BM, int BN, typename TA, typename TB, typename TC, int WL>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
  gemm_body<BM, BN, __bf16, TA, TB, TC, WL>(g);
}

// Sum of the ksplit partial products in chunk order (bitwise reproducible).
__global__ void splitk_reduce_kernel(GemmArgs g) {
  const int64_t per = g.M * g.N, total = per * g.batch;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / per, rem = e - p * per;
    if (g.run_flag != nullptr && g.run_flag[p * g.run_flag_stride] != g.run_when) continue;
    const int64_t r = rem / g.N, c = rem - r * g.N;
    const double *src = g.part + p * g.ksplit * per + rem;
    double acc = 0.0;
    for (int t = 0; t < g.ksplit; ++t) acc += src[t * per];
    const int64_t off = p * g.C.bs + r * g.C.rs + c * g.C.cs;
    if (g.c_f32) {  // FP32 storage of C (the low-precision range finding)
      float *cp = reinterpret_cast<float *>(static_cast<void *>(g.C.ptr)) + off;
      if (g.beta != 0.0) acc += g.beta * (double)(*cp);
      *cp = (float)acc;
    } else {
      double *cp = g.C.ptr + off;
      if (g.beta != 0.0) acc += g.beta * (*cp);
      *cp = acc;
    }
  }
}

// Thin-N GEMM (32 < N <= 48, C = alpha A B + beta C; FP64, or FP32 matrix
// cores for the FP32 range finding; the launcher also runs products thin in
// M here, transposed): a workgroup forms 64 MI rows of C, each wave 16 MI of
// them (MI 16-row MFMA blocks) across all N columns.  A goes from global
// memory straight into the MFMA operand registers with no LDS round trip.
// Inside each 16-wide K chunk the K order
// is permuted so that loads stay coalesced: with A k-fast a lane's four
// values are consecutive in memory (k = 4 (lane / 16) + t at MFMA step t),
// with A m-fast 16 lanes read 16 consecutive rows (k = 4 t + lane / 16).  B's
// chunk is staged through a double-buffered LDS tile and read with the same
// permutation, so every product pairs A(m, k) with B(k, n) as in the plain
// sum.  A's loads run two chunks ahead in a ring of three register sets, B's
// one chunk ahead (issued first, so that waiting for B leaves A in flight);
// one barrier per chunk.  Columns 32..N-1 form a third 16-wide block
// (FULL2, N > 40) or one or two 4-wide strips of the four-block 4 x 4 x 4
// MFMA (N <= 40), whose A operand is the 16 x 16 x 4 one's.
namespace {
constexpr int kThinCh = 16, kThinLdb = 49;
// 16-row blocks per wave: two for k-fast A (its loads are the longer-latency
// ones; two blocks share each B fragment read), one for m-fast A (more waves
// per SIMD)
constexpr int thin_mi(bool ak) { return ak ? 2 : 1; }
}

// CT is the compute type (FP64, or FP32 matrix cores accumulating in FP32,
// always with a full third column block); TA, TB, TC are the storage types.
template <int MI, bool AK, bool FULL2, typename CT, typename TA, typename TB, typename TC>
__device__ __forceinline__ void thin_body(const GemmArgs &g) {
  constexpr bool F64 = std::is_same<CT, double>::value;
  static_assert(F64 || FULL2, "the 4 x 4 x 4 strips are FP64 only");
  using acc_t = typename std::conditional<F64, d4_t, f4_t>::type;
  constexpr int CH = kThinCh, LDB = kThinLdb, NB = FULL2 ? 3 : 2;
  __shared__ CT Bs[2][CH * LDB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, kq = lane >> 4;
  const int ks = g.ksplit;
  const int p = blockIdx.z / ks, kc = blockIdx.z - (blockIdx.z / ks) * ks;
  if (g.run_flag != nullptr && g.run_flag[p * g.run_flag_stride] != g.run_when) return;
  int64_t kchunk = (g.K + ks - 1) / ks;
  kchunk = ((kchunk + CH - 1) / CH) * CH;
  const int64_t kbeg = kc * kchunk;
  const int64_t kend = std::min<int64_t>(g.K, kbeg + kchunk);
  const int nch = kend > kbeg ? (int)((kend - kbeg + CH - 1) / CH) : 0;
  const int64_t m0 = (int64_t)blockIdx.x * (64 * MI) + wave * (16 * MI);
  const int M = (int)g.M, N = (int)g.N;  // the launcher checks that offsets fit in 32 bits

  bool live[MI];
#pragma unroll
  for (int i = 0; i < MI; ++i) live[i] = m0 + 16 * i < g.M;
  // columns 32..N-1 without FULL2: strips of 4 (one or two), wave-uniform
  const int rem_cnt = FULL2 ? 0 : (N - 32 + 3) / 4;

  // A: per-lane offsets of the row part (rows past M read row M-1; their
  // results are never stored) and of the permuted k index at step t.
  const TA *Ab = reinterpret_cast<const TA *>(static_cast<const void *>(g.A.ptr)) + p * g.A.bs + kbeg * g.A.cs;
  const int ars = (int)g.A.rs, acs = (int)g.A.cs;
  int a_row[MI];
#pragma unroll
  for (int i = 0; i < MI; ++i) {
    const int row = (int)std::min<int64_t>(m0 + 16 * i + r, g.M - 1);
    a_row[i] = AK ? row * ars : row;
  }
  auto kidx = [&](int t) { return AK ? 4 * kq + t : 4 * t + kq; };

  // B: three elements per thread per chunk; k-fast B is walked along k.
  const TB *Bb = reinterpret_cast<const TB *>(static_cast<const void *>(g.B.ptr)) + p * g.B.bs + kbeg * g.B.rs;
  const bool b_kfast = g.B.rs == 1 && g.B.cs != 1;
  const int brs = (int)g.B.rs;
  int b_k[3], b_noff[3], b_loff[3];  // b_k: the k index, or CH for a column past N
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int e = tid + 256 * u;  // 768 = 16 x 48 elements
    const int bk = b_kfast ? (e & 15) : e / 48, bn = b_kfast ? (e >> 4) : e % 48;
    b_k[u] = bn < N ? bk : CH;
    b_noff[u] = std::min(bn, N - 1) * (int)g.B.cs;
    b_loff[u] = bk * LDB + bn;
  }

  // Every load of the chunk loop is unconditional and in bounds: indices past
  // the valid K of a partial last chunk are clamped to its last valid k, and
  // the values they bring are zeroed where they are used (B when parked, A
  // before its MFMAs), so no load waits on a branch.
  auto chunk_rem = [&](int c) { return (int)std::min<int64_t>(kend - kbeg - (int64_t)CH * c, CH); };
  typedef CT Frag[MI][4];
  auto fetchA = [&](int c, Frag &dst) {
    const TA *base = Ab + (int64_t)(CH * c) * acs;
    const int last = chunk_rem(c) - 1;
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int kk = std::min(kidx(t), last);
        dst[i][t] = (CT)base[a_row[i] + (AK ? kk : kk * acs)];
      }
  };
  TB rb[3];
  auto fetchB = [&](int c) {
    const TB *base = Bb + (int64_t)(CH * c) * g.B.rs;
    const int last = chunk_rem(c) - 1;
#pragma unroll
    for (int u = 0; u < 3; ++u) rb[u] = base[std::min(b_k[u], last) * brs + b_noff[u]];
  };
  auto parkB = [&](int c, int buf) {
    CT *dst = Bs[buf];
    const int rem = chunk_rem(c);
#pragma unroll
    for (int u = 0; u < 3; ++u) dst[b_loff[u]] = b_k[u] < rem ? (CT)rb[u] : (CT)0;
  };

  acc_t acc[MI][NB];
  double racc[MI][2];
#pragma unroll
  for (int i = 0; i < MI; ++i) {
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
    racc[i][0] = racc[i][1] = 0.0;
  }
  auto mult = [&](int s, const Frag &a) {
    const CT *bs = Bs[s & 1];
    const int rem = chunk_rem(s);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const CT *bp = bs + kidx(t) * LDB;
      CT bv[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) bv[j] = bp[16 * j + r];
      double x[2] = {0.0, 0.0};
      if constexpr (!FULL2) {
#pragma unroll
        for (int q = 0; q < 2; ++q) x[q] = (double)bp[32 + 4 * q + (lane & 3)];
      }
      const bool kin = kidx(t) < rem;
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        if (!live[i]) continue;  // wave-uniform
        const CT av = kin ? a[i][t] : (CT)0;
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = mfma16(av, bv[j], acc[i][j]);
        if constexpr (!FULL2) {
#pragma unroll
          for (int q = 0; q < 2; ++q)
            if (q < rem_cnt) racc[i][q] = mfma4((double)av, x[q], racc[i][q]);
        }
      }
    }
  };

  Frag a0, a1, a2;
  if (nch > 0) {
    fetchB(0);
    fetchA(0, a0);
    fetchA(std::min(1, nch - 1), a1);
    parkB(0, 0);
  }
  __syncthreads();
  // chunk s: B(s + 1) and A(s + 2) are fetched (the last chunk again past
  // the end), chunk s is multiplied, B(s + 1) is parked in the other LDS
  // buffer, one barrier
  auto step = [&](int s, const Frag &cur, Frag &ahead) {
    const int c1 = std::min(s + 1, nch - 1);
    fetchB(c1);
    fetchA(std::min(s + 2, nch - 1), ahead);
    mult(s, cur);
    parkB(c1, (s + 1) & 1);
    __syncthreads();
  };
  for (int s = 0; s < nch; s += 3) {
    step(s, a0, a2);
    if (s + 1 >= nch) break;
    step(s + 1, a1, a0);
    if (s + 2 >= nch) break;
    step(s + 2, a2, a1);
  }

  auto strip_at = [&](int q, int i, int64_t *gm, int *gn) {
    *gm = m0 + 16 * i + 4 * ((lane >> 2) & 3) + kq;
    *gn = 32 + 4 * q + (lane & 3);
  };
  if (ks == 1) {
    TC *Cb = reinterpret_cast<TC *>(static_cast<void *>(g.C.ptr)) + p * g.C.bs;
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      if (!live[i]) continue;
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t gm = m0 + 16 * i + mfma_row<CT>(kq, v);
          const int gn = 16 * j + r;
          if (gm < M && gn < N) {
            TC *cp = Cb + gm * g.C.rs + gn * g.C.cs;
            double y = g.alpha * (double)acc[i][j][v];
            if (g.beta != 0.0) y += g.beta * (double)(*cp);
            *cp = (TC)y;
          }
        }
      if constexpr (!FULL2) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          int64_t gm;
          int gn;
          strip_at(q, i, &gm, &gn);
          if (q < rem_cnt && gm < M && gn < N) {
            TC *cp = Cb + gm * g.C.rs + gn * g.C.cs;
            double y = g.alpha * racc[i][q];
            if (g.beta != 0.0) y += g.beta * (double)(*cp);
            *cp = (TC)y;
          }
        }
      }
    }
  } else if constexpr (F64) {  // split-K partials (the FP32 form runs unsplit)
    double *Pb = g.part + ((int64_t)p * ks + kc) * g.M * g.N;
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      if (!live[i]) continue;
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t gm = m0 + 16 * i + mfma_row<CT>(kq, v);
          const int gn = 16 * j + r;
          if (gm < M && gn < N) Pb[g.part_t ? gn * g.M + gm : gm * N + gn] = g.alpha * acc[i][j][v];
        }
      if constexpr (!FULL2) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          int64_t gm;
          int gn;
          strip_at(q, i, &gm, &gn);
          if (q < rem_cnt && gm < M && gn < N) Pb[g.part_t ? gn * g.M + gm : gm * N + gn] = g.alpha * racc[i][q];
        }
      }
    }
  }
}

template <int MI, bool AK, bool FULL2>
__global__ __launch_bounds__(256) void gemm_thin_f64_kernel(GemmArgs g) {
  thin_body<MI, AK, FULL2, double, double, double, double>(g);
}

template <int MI, bool AK, typename TA, typename TB, typename TC>
__global__ __launch_bounds__(256) void gemm_thin_f32_kernel(GemmArgs g) {
  thin_body<MI, AK, true, float, TA, TB, TC>(g);
}

// The thin kernel's variant for g (bit 1: A k-fast, bit 0: a full third
// column block, always set for the FP32 form), or -1 when it does not apply:
// 32 < N <= 48 with more than 32 rows, A with a unit stride, every per-pair
// offset within 32 bits, and FP64 operands or one of the FP32 path's
// storage combinations (unsplit).
static int thin_variant(const GemmArgs &g) {
  if (g.prec) {
    const int combo = g.a_f32 * 4 + g.b_f32 * 2 + g.c_f32;
    if ((combo != 5 && combo != 2 && combo != 7) || g.ksplit > 1) return -1;
  } else if (g.a_f32 || g.b_f32 || g.c_f32) {
    return -1;
  }
  if (!(g.N > 32 && g.N <= 48 && g.M > 32)) return -1;
  const bool ak = g.A.cs == 1;
  if (!ak && g.A.rs != 1) return -1;
  if (g.A.rs < 0 || g.A.cs < 0 || g.B.rs < 0 || g.B.cs < 0) return -1;
  const int64_t lim = (int64_t)1 << 30;
  const int64_t kpad = g.K + kThinCh;
  if (g.M >= lim || (g.M - 1) * g.A.rs + kpad * g.A.cs >= lim) return -1;
  if (kpad * g.B.rs + 48 * g.B.cs >= lim) return -1;
  return (ak ? 2 : 0) | ((g.prec || g.N > 40) ? 1 : 0);
}

// Arguments and variant of the thin kernel for g: g itself when it is thin
// in N; for 32 < M <= 48 and N > 48 the transposed product C^T = B^T A^T
// (operands, their storage types and C with their strides swapped, split-K
// partials still written in g's M x N layout); -1 when neither applies.
static int thin_args(const GemmArgs &g, GemmArgs *t) {
  *t = g;
  int v = thin_variant(g);
  if (v >= 0 || !(g.M > 32 && g.M <= 48 && g.N > 48)) return v;
  t->A = CMat{g.B.ptr, g.B.cs, g.B.rs, g.B.bs};
  t->B = CMat{g.A.ptr, g.A.cs, g.A.rs, g.A.bs};
  t->C = Mat{g.C.ptr, g.C.cs, g.C.rs, g.C.bs};
  t->a_f32 = g.b_f32;
  t->b_f32 = g.a_f32;
  t->M = g.N;
  t->N = g.M;
  t->part_t = 1;
  v = thin_variant(*t);
  if (v < 0) *t = g;
  return v;
}

static const char *tname(int f32) { return f32 ? "float" : "double"; }

void gemm_kernel_name(const GemmArgs &g, char *buf, size_t n) {
  GemmArgs t;
  const int v = (g.prec == 2) ? -1 : thin_args(g, &t);
  const char *ak = (v & 2) ? "true" : "false";
  if (v >= 0 && !g.prec) {
    snprintf(buf, n, "gemm_thin_f64_kernel<%d, %s, %s>", thin_mi(v & 2), ak, (v & 1) ? "true" : "false");
    return;
  }
  if (v >= 0) {
    snprintf(buf, n, "gemm_thin_f32_kernel<%d, %s, %s, %s, %s>", thin_mi(v & 2), ak, tname(t.a_f32),
             tname(t.b_f32), tname(t.c_f32));
    return;
  }
  int bm, bn, wl;
  gemm_tile(g.M, g.N, &bm, &bn, &wl);
  if (g.prec)
    snprintf(buf, n, "%s<%d, %d, %s, %s, %s, %d>", g.prec == 2 ? "gemm_bf16_kernel" : "gemm_f32_kernel", bm, bn,
             tname(g.a_f32), tname(g.b_f32), tname(g.c_f32), wl);
  else
    snprintf(buf, n, "gemm_f64_kernel<%d, %d, %d>", bm, bn, wl);
}

// Tile shape: 32 rows or columns when that side of C is at most 32 wide
// (less padding for the thin operands of the sweep), else 64.
void gemm_tile(int64_t M, int64_t N, int *bm, int *bn, int *wl) {
  *bm = (M <= 32) ? 32 : 64;
  *bn = (N <= 32) ? 32 : 64;
  // one 64-wide tile for 32 < N <= 48 (A is fetched once; the dead fourth
  // column block is skipped), its waves stacked along M; likewise along N for
  // 32 < M <= 48
  *wl = 0;
  if (*bm == 64 && *bn == 64) *wl = (N <= 48) ? 1 : ((M <= 48) ? 2 : 0);
}

int gemm_pick_ksplit(int64_t M, int64_t N, int64_t K, int batch) {
  int bm, bn, wl;
  gemm_tile(M, N, &bm, &bn, &wl);
  const int64_t tiles = ((M + bm - 1) / bm) * ((N + bn - 1) / bn) * (int64_t)batch;
  int ks = 1;
  // aim for ~8 workgroups per CU (latency hiding) while keeping >= 4 K slabs per chunk
  while (tiles * ks < 2048 && K / ((int64_t)(ks * 2) * BK) >= 4 && ks < 64) ks *= 2;
  return ks;
}

hipError_t launch_gemm(const GemmArgs &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  GemmArgs a = g;
  if (a.K <= 0) a.ksplit = 1;  // C = beta C
  if (a.ksplit < 1) a.ksplit = 1;
  if (a.ksplit > 1 && a.part == nullptr) a.ksplit = 1;
  int bm, bn, wl;
  gemm_tile(a.M, a.N, &bm, &bn, &wl);

  dim3 grid((unsigned)((a.M + bm - 1) / bm), (unsigned)((a.N + bn - 1) / bn), (unsigned)(a.batch * a.ksplit));
  GemmArgs t;
  const int thin = (a.prec == 2) ? -1 : thin_args(a, &t);  // no thin BF16 kernel
  if (thin >= 0) {
    const int rows = 64 * thin_mi(thin & 2);
    dim3 tg((unsigned)((t.M + rows - 1) / rows), 1, (unsigned)(t.batch * t.ksplit));
    if (t.prec) {
      const int combo = t.a_f32 * 4 + t.b_f32 * 2 + t.c_f32;
#define HATT_THIN32(TA, TB, TC)                                                               \
  do {                                                                                        \
    if (thin & 2) gemm_thin_f32_kernel<thin_mi(true), true, TA, TB, TC><<<tg, 256, 0, s>>>(t); \
    else gemm_thin_f32_kernel<thin_mi(false), false, TA, TB, TC><<<tg, 256, 0, s>>>(t);        \
  } while (0)
      if (combo == 5) HATT_THIN32(float, double, float);
      else if (combo == 2) HATT_THIN32(double, float, double);
      else HATT_THIN32(float, float, float);
#undef HATT_THIN32
    } else if (thin == 3) gemm_thin_f64_kernel<thin_mi(true), true, true><<<tg, 256, 0, s>>>(t);
    else if (thin == 2) gemm_thin_f64_kernel<thin_mi(true), true, false><<<tg, 256, 0, s>>>(t);
    else if (thin == 1) gemm_thin_f64_kernel<thin_mi(false), false, true><<<tg, 256, 0, s>>>(t);
    else gemm_thin_f64_kernel<thin_mi(false), false, false><<<tg, 256, 0, s>>>(t);
  } else if (!a.prec) {
    if (a.a_f32 || a.b_f32 || a.c_f32) return hipErrorInvalidValue;
    if (bm == 64 && bn == 64) {
      if (wl == 1) gemm_f64_kernel<64, 64, 1><<<grid, 256, 0, s>>>(a);
      else if (wl == 2) gemm_f64_kernel<64, 64, 2><<<grid, 256, 0, s>>>(a);
      else gemm_f64_kernel<64, 64, 0><<<grid, 256, 0, s>>>(a);
    } else if (bm == 64) gemm_f64_kernel<64, 32, 0><<<grid, 256, 0, s>>>(a);
    else if (bn == 64) gemm_f64_kernel<32, 64, 0><<<grid, 256, 0, s>>>(a);
    else gemm_f64_kernel<32, 32, 0><<<grid, 256, 0, s>>>(a);
  } else if (a.prec == 2) {
    // BF16 range finding: W_L (FP32) x sketch (FP64) -> W (FP32)
    if (a.a_f32 != 1 || a.b_f32 != 0 || a.c_f32 != 1) return hipErrorInvalidValue;
    if (bm == 64 && bn == 64) {
      if (wl == 1) gemm_bf16_kernel<64, 64, float, double, float, 1><<<grid, 256, 0, s>>>(a);
      else if (wl == 2) gemm_bf16_kernel<64, 64, float, double, float, 2><<<grid, 256, 0, s>>>(a);
      else gemm_bf16_kernel<64, 64, float, double, float, 0><<<grid, 256, 0, s>>>(a);
    } else if (bm == 64) gemm_bf16_kernel<64, 32, float, double, float, 0><<<grid, 256, 0, s>>>(a);
    else if (bn == 64) gemm_bf16_kernel<32, 64, float, double, float, 0><<<grid, 256, 0, s>>>(a);
    else gemm_bf16_kernel<32, 32, float, double, float, 0><<<grid, 256, 0, s>>>(a);
  } else {
    const int combo = a.a_f32 * 4 + a.b_f32 * 2 + a.c_f32;
#define HATT_GEMM32(TA, TB, TC)                                                              \
  do {                                                                                       \
    if (bm == 64 && bn == 64) {                                                              \
      if (wl == 1) gemm_f32_kernel<64, 64, TA, TB, TC, 1><<<grid, 256, 0, s>>>(a);           \
      else if (wl == 2) gemm_f32_kernel<64, 64, TA, TB, TC, 2><<<grid, 256, 0, s>>>(a);      \
      else gemm_f32_kernel<64, 64, TA, TB, TC, 0><<<grid, 256, 0, s>>>(a);                   \
    } else if (bm == 64) gemm_f32_kernel<64, 32, TA, TB, TC, 0><<<grid, 256, 0, s>>>(a);     \
    else if (bn == 64) gemm_f32_kernel<32, 64, TA, TB, TC, 0><<<grid, 256, 0, s>>>(a);       \
    else gemm_f32_kernel<32, 32, TA, TB, TC, 0><<<grid, 256, 0, s>>>(a);                     \
  } while (0)
    if (combo == 5) HATT_GEMM32(float, double, float);       // W_L (f32) x sketch (f64) -> W (f32)
    else if (combo == 2) HATT_GEMM32(double, float, double); // X (f64) x W (f32) -> Y (f64)
    else if (combo == 7) HATT_GEMM32(float, float, float);
    else return hipErrorInvalidValue;
#undef HATT_GEMM32
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.ksplit == 1 || a.no_reduce) return e;
  return launch_splitk_reduce(a, s);
}

hipError_t launch_splitk_reduce(const GemmArgs &a, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0 || a.batch <= 0 || a.ksplit <= 1) return hipSuccess;
  const int64_t total = a.M * a.N * a.batch;
  int rg = (int)std::min<int64_t>((total + 255) / 256, 65536);
  splitk_reduce_kernel<<<rg, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace hatt
