// Elementwise and small-contraction kernels: Philox sketch, PKP expansion,
// the last-core sketch of HPCRL and the "sandwich" contraction that carries
// both the W_L columns of HPCRL (eq. WLWR) and the PKP-free core update of
// the HaTT sweep (eq. M*core0).
#include <mutex>
#include "common.h"
#include "stage.h"

namespace hatt {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 products
// with the published multipliers, Weyl key schedule between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    uint32_t lo0 = m0 * c[0], hi0 = __umulhi(m0, c[0]);
    uint32_t lo1 = m1 * c[2], hi1 = __umulhi(m1, c[2]);
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
  // ((a >> 5) 2^26 + (b >> 6) + 1/2) 2^-53, strictly inside (0, 1)
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 0.5) * (1.0 / 9007199254740992.0);
}

__global__ void sketch_fill_kernel(uint64_t seed, uint32_t core, int64_t count, double scale,
                                   double *__restrict__ out) {
  const int64_t npairs = (count + 1) / 2;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npairs;
       p += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c[4] = {(uint32_t)(p & 0xFFFFFFFFu), (uint32_t)((uint64_t)p >> 32), core, 0x5A7Cu};
    philox4x32_10(c, (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32));
    const double ua = u53(c[0], c[1]);
    const double ub = u53(c[2], c[3]);
    const double rad = sqrt(-2.0 * log(ua)) * scale;
    const double ang = 6.283185307179586476925286766559 * ub;
    const double g0 = rad * cos(ang), g1 = rad * sin(ang);
    out[2 * p] = g0;
    if (2 * p + 1 < count) out[2 * p + 1] = g1;
  }
}

hipError_t launch_sketch_fill(uint64_t seed, int core, int64_t count, double scale, double *out,
                              hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t npairs = (count + 1) / 2;
  int grid = (int)std::min<int64_t>((npairs + 255) / 256, 8192);
  sketch_fill_kernel<<<grid, 256, 0, s>>>(seed, (uint32_t)core, count, scale, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// PKP expansion (Sec. 2.2).  Memory bound: one thread per output element,
// consecutive threads write consecutive (a', b') so stores coalesce; inputs
// are small and stay in cache.
__global__ void pkp_kernel(PkpArgs a) {
  const int64_t cols = a.r1 * a.s1;
  const int64_t per = a.r0 * a.s0 * a.n * cols;
  const int64_t total = per * a.batch;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / per;
    int64_t rem = e - p * per;
    const int64_t col = rem % cols;
    rem /= cols;
    const int64_t i = rem % a.n;
    const int64_t row = rem / a.n;
    const int64_t ra = row / a.s0, sb = row - ra * a.s0;
    const int64_t ca = col / a.s1, cb = col - ca * a.s1;
    const double xv = a.x[p * a.xs + (ra * a.n + i) * a.r1 + ca];
    const double yv = a.y[p * a.ys + (sb * a.n + i) * a.s1 + cb];
    a.out[p * a.os + (row * a.n + i) * cols + col] = xv * yv;
  }
}

hipError_t launch_pkp(const PkpArgs &a, hipStream_t s) {
  const int64_t total = a.r0 * a.s0 * a.n * a.r1 * a.s1 * a.batch;
  if (total <= 0) return hipSuccess;
  int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  pkp_kernel<<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sandwich contraction out_{i,g} = YL_i C_g ZR_i for a chunk of GC values of
// g per workgroup, slice i = blockIdx.x.  YL_i and ZR_i are staged once in
// LDS, the GC matrices C_g next to them; the product is formed as
// T = C_g ZR_i (RI x SO) and then YL_i T.  Two LDS layouts: with g innermost
// when the output is contiguous in g (the W_L columns of HPCRL), else with
// the column index innermost (the core update, contiguous in (a', b')).
// Every LDS access pattern is either a broadcast or unit stride.
template <bool GFAST>
__global__ __launch_bounds__(256) void sandwich_kernel(SandwichArgs a, int GC) {
  extern __shared__ double sm[];
  const int RA = a.RA, RI = a.RI, SI = a.SI, SO = a.SO;
  double *YL = sm;                  // RA x RI      YL[a'*RI + a]
  double *ZR = YL + RA * RI;        // SI x SO      ZR[b*SO + b']
  double *Cs = ZR + SI * SO;        // GC x RI x SI
  double *Ts = Cs + GC * RI * SI;   // GC x RI x SO
  const int tid = threadIdx.x;
  const int64_t i = blockIdx.x;
  const int64_t g0 = (int64_t)blockIdx.y * GC;
  const int p = blockIdx.z;
  const int gc = (int)std::min<int64_t>(GC, a.G - g0);
  if (gc <= 0) return;

  const double *yl = a.yl + p * a.ylb + i * a.yli;
  if (a.ylc == 1) {
    for (int e = tid; e < RA * RI; e += 256) {
      int ap = e / RI, aa = e - ap * RI;
      YL[e] = yl[ap * a.ylr + aa];
    }
  } else {
    for (int e = tid; e < RA * RI; e += 256) {
      int aa = e / RA, ap = e - aa * RA;
      YL[ap * RI + aa] = yl[ap * a.ylr + aa * a.ylc];
    }
  }
  const double *zr = a.zr + p * a.zrb + i * a.zri;
  if (a.zrc == 1) {
    for (int e = tid; e < SI * SO; e += 256) {
      int b = e / SO, bp = e - b * SO;
      ZR[e] = zr[b * a.zrr + bp];
    }
  } else {
    for (int e = tid; e < SI * SO; e += 256) {
      int bp = e / SI, b = e - bp * SI;
      ZR[b * SO + bp] = zr[b * a.zrr + bp * a.zrc];
    }
  }
  const double *cbase = a.c + p * a.cb + g0 * a.cg;
  const int nC = gc * RI * SI;
  if (GFAST) {
    // Cs[(a*SI + b)*GC + gg], digits (gg, b, a)
    Rad3 d(tid, 256, gc, SI);
    for (int e = tid; e < nC; e += 256, d.next())
      Cs[(d.i2 * SI + d.i1) * GC + d.i0] = cbase[d.i0 * a.cg + d.i2 * a.ca + d.i1 * a.cbb];
  } else {
    // Cs[(gg*RI + a)*SI + b], digits (b, a, gg)
    Rad3 d(tid, 256, SI, RI);
    for (int e = tid; e < nC; e += 256, d.next())
      Cs[e] = cbase[d.i2 * a.cg + d.i1 * a.ca + d.i0 * a.cbb];
  }
  __syncthreads();

  // T = C_g ZR  (RI x SO per g)
  const int nT = gc * RI * SO;
  if (GFAST) {
    Rad3 d(tid, 256, gc, SO);  // digits (gg, b', a)
    for (int e = tid; e < nT; e += 256, d.next()) {
      const double *cr = Cs + d.i2 * SI * GC + d.i0;
      const double *zc = ZR + d.i1;
      double acc = 0.0;
      for (int b = 0; b < SI; ++b) acc += cr[b * GC] * zc[b * SO];
      Ts[(d.i2 * SO + d.i1) * GC + d.i0] = acc;
    }
  } else {
    Rad3 d(tid, 256, SO, RI);  // digits (b', a, gg)
    for (int e = tid; e < nT; e += 256, d.next()) {
      const double *cr = Cs + (d.i2 * RI + d.i1) * SI;
      const double *zc = ZR + d.i0;
      double acc = 0.0;
      for (int b = 0; b < SI; ++b) acc += cr[b] * zc[b * SO];
      Ts[e] = acc;
    }
  }
  __syncthreads();

  // out = YL T  (RA x SO per g)
  double *obase = a.o + p * a.ob + i * a.oi + g0 * a.og;
  const int nO = gc * RA * SO;
  if (GFAST) {
    Rad3 d(tid, 256, gc, SO);  // digits (gg, b', a')
    for (int e = tid; e < nO; e += 256, d.next()) {
      const double *yr = YL + d.i2 * RI;
      const double *tc = Ts + d.i1 * GC + d.i0;
      double acc = 0.0;
      for (int aa = 0; aa < RI; ++aa) acc += yr[aa] * tc[aa * SO * GC];
      obase[d.i0 * a.og + d.i2 * a.oa + d.i1 * a.obb] = acc;
    }
  } else {
    Rad3 d(tid, 256, SO, RA);  // digits (b', a', gg)
    for (int e = tid; e < nO; e += 256, d.next()) {
      const double *yr = YL + d.i1 * RI;
      const double *tc = Ts + d.i2 * RI * SO + d.i0;
      double acc = 0.0;
      for (int aa = 0; aa < RI; ++aa) acc += yr[aa] * tc[aa * SO];
      obase[d.i2 * a.og + d.i1 * a.oa + d.i0 * a.obb] = acc;
    }
  }
}

// Register-blocked variant for ranks up to MAXR.  Thread (g, b') keeps the
// b'-columns of ZR (SI x BPT) and of T_g = C_g ZR (RI x BPT) in registers;
// rows of C_g and of YL are read from LDS as double2 words that every lane
// working on the same g (stage 1) or every lane (stage 2) shares, so one LDS
// instruction feeds 2 * BPT FMAs.  Rows are zero-padded to even length.
// LANE_G: lanes run along g (outputs with g fastest), else along b'.
template <int MAXR, int BPT, bool LANE_G>
__global__ __launch_bounds__(256) void sandwich_reg_kernel(SandwichArgs a, int GC, int TPG) {
  extern __shared__ double sm[];
  const int RA = a.RA, RI = a.RI, SI = a.SI, SO = a.SO;
  const int RIp = (RI + 1) & ~1, SIp = (SI + 1) & ~1;
  const int cgs = RI * SIp + 2;          // per-g stride of the C chunk (padding breaks bank aliasing)
  const int zsz = (SI * SO + 1) & ~1;
  double *YL = sm;                       // RA x RIp
  double *ZR = YL + RA * RIp;            // SI x SO
  double *Cs = ZR + zsz;                 // GC x cgs
  const int tid = threadIdx.x;
  const int64_t i = blockIdx.x;
  const int64_t g0 = (int64_t)blockIdx.y * GC;
  const int p = blockIdx.z;
  const int gc = (int)std::min<int64_t>(GC, a.G - g0);
  if (gc <= 0) return;

  const double *yl = a.yl + p * a.ylb + i * a.yli;
  stage_lds<4>(RA * RIp, Rad3(tid, 256, RIp, RA), YL,  // digits (a, a')
               [&](const Rad3 &d) { return (d.i0 < RI) ? yl[d.i1 * a.ylr + d.i0 * a.ylc] : 0.0; },
               [&](const Rad3 &d) { return d.i1 * RIp + d.i0; });
  const double *zr = a.zr + p * a.zrb + i * a.zri;
  stage_lds<4>(SI * SO, Rad3(tid, 256, SO, SI), ZR,  // digits (b', b)
               [&](const Rad3 &d) { return zr[d.i1 * a.zrr + d.i0 * a.zrc]; },
               [&](const Rad3 &d) { return d.i1 * SO + d.i0; });
  const double *cbase = a.c + p * a.cb + g0 * a.cg;
  const int per = RI * SIp;
  if (a.cg == 1) {
    // g is the fastest index of C in memory: consecutive threads take consecutive g
    stage_lds<8>(gc * per, Rad3(tid, 256, gc, SIp), Cs,  // digits (g, b, a)
                 [&](const Rad3 &d) {
                   return (d.i1 < SI) ? cbase[d.i0 * a.cg + d.i2 * a.ca + d.i1 * a.cbb] : 0.0;
                 },
                 [&](const Rad3 &d) { return d.i0 * cgs + d.i2 * SIp + d.i1; });
  } else {
    stage_lds<8>(gc * per, Rad3(tid, 256, SIp, RI), Cs,  // digits (b, a, g)
                 [&](const Rad3 &d) {
                   return (d.i0 < SI) ? cbase[d.i2 * a.cg + d.i1 * a.ca + d.i0 * a.cbb] : 0.0;
                 },
                 [&](const Rad3 &d) { return d.i2 * cgs + d.i1 * SIp + d.i0; });
  }
  __syncthreads();

  int tg, tb;
  if (LANE_G) {
    tg = tid % GC;
    tb = tid / GC;
  } else {
    tb = tid % TPG;
    tg = tid / TPG;
  }
  if (tg >= gc || tb >= TPG) return;
  const int bp0 = tb * BPT;

  double zc[MAXR][BPT];
#pragma unroll
  for (int b = 0; b < MAXR; ++b)
#pragma unroll
    for (int j = 0; j < BPT; ++j) zc[b][j] = (b < SI && bp0 + j < SO) ? ZR[b * SO + bp0 + j] : 0.0;

  // stage 1: T_g(:, b') = C_g ZR(:, b')
  double t[MAXR][BPT];
  const double *cg = Cs + tg * cgs;
#pragma unroll
  for (int aa = 0; aa < MAXR; ++aa) {
#pragma unroll
    for (int j = 0; j < BPT; ++j) t[aa][j] = 0.0;
    if (aa < RI) {
      const double *crow = cg + aa * SIp;
#pragma unroll
      for (int b = 0; b < MAXR; b += 2) {
        if (b < SIp) {
          const double2 c2 = *reinterpret_cast<const double2 *>(crow + b);
#pragma unroll
          for (int j = 0; j < BPT; ++j) t[aa][j] = fma(c2.x, zc[b][j], fma(c2.y, zc[b + 1][j], t[aa][j]));
        }
      }
    }
  }
  // stage 2: out(a', b') = YL(a', :) T_g(:, b')
  double *obase = a.o + p * a.ob + i * a.oi + (g0 + tg) * a.og;
  for (int ap = 0; ap < RA; ++ap) {
    const double *yrow = YL + ap * RIp;
    double acc[BPT];
#pragma unroll
    for (int j = 0; j < BPT; ++j) acc[j] = 0.0;
#pragma unroll
    for (int aa = 0; aa < MAXR; aa += 2) {
      if (aa < RIp) {
        const double2 y2 = *reinterpret_cast<const double2 *>(yrow + aa);
#pragma unroll
        for (int j = 0; j < BPT; ++j) acc[j] = fma(y2.x, t[aa][j], fma(y2.y, t[aa + 1][j], acc[j]));
      }
    }
#pragma unroll
    for (int j = 0; j < BPT; ++j)
      if (bp0 + j < SO) obase[ap * a.oa + (bp0 + j) * a.obb] = acc[j];
  }
}

namespace {
template <int MAXR, int BPT, bool LG>
hipError_t sandwich_reg_launch(const SandwichArgs &a, hipStream_t s, int64_t budget) {
  const int RIp = (a.RI + 1) & ~1, SIp = (a.SI + 1) & ~1;
  const int64_t cgs = (int64_t)a.RI * SIp + 2;
  const int64_t fixed = (int64_t)a.RA * RIp + (((int64_t)a.SI * a.SO + 1) & ~1);
  const int TPG = (a.SO + BPT - 1) / BPT;
  int64_t gmax = std::min<int64_t>(256 / TPG, (budget - fixed) / cgs);
  if (gmax < 1) return hipErrorInvalidValue;
  const int64_t chunks = (a.G + gmax - 1) / gmax;
  const int64_t GC = (a.G + chunks - 1) / chunks;
  const size_t lds = (size_t)(fixed + GC * cgs) * sizeof(double);
  static std::once_flag attr_done;
  std::call_once(attr_done, [&] {
    hipFuncSetAttribute((const void *)sandwich_reg_kernel<MAXR, BPT, LG>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)(budget * sizeof(double)));
  });
  dim3 grid((unsigned)a.n, (unsigned)chunks, (unsigned)a.batch);
  sandwich_reg_kernel<MAXR, BPT, LG><<<grid, 256, lds, s>>>(a, (int)GC, TPG);
  return hipGetLastError();
}

template <bool LG>
hipError_t sandwich_reg_dispatch(const SandwichArgs &a, hipStream_t s, int64_t budget, bool *done) {
  const int m = std::max(std::max(a.RI, a.SI), 1);
  *done = (a.SO <= 256);  // one g's threads must fit a block
  if (!*done) return hipSuccess;
  if (m <= 16) return sandwich_reg_launch<16, 2, LG>(a, s, budget);
  if (m <= 24) return sandwich_reg_launch<24, 2, LG>(a, s, budget);
  if (m <= 32) return sandwich_reg_launch<32, 1, LG>(a, s, budget);
  if (m <= 48) return sandwich_reg_launch<48, 1, LG>(a, s, budget);
  *done = false;
  return hipSuccess;
}
}  // namespace

bool g_sandwich_reg = true;
bool g_sandwich_mfma = true;

const char *sandwich_kernel_name(const SandwichArgs &a, const SwForce *force) {
  const int64_t budget = 19456;
  SwPlan pl;
  const bool valu = force != nullptr && force->valu && !a.prec;
  if ((a.prec || g_sandwich_mfma) && !valu && sandwich_mfma_plan(a, kSandwichLdsDoubles, &pl, force))
    return sandwich_mfma_name(a, pl);
  if (a.prec) return "none (the low-precision sandwich needs the matrix-core plan)";
  const int RIp = (a.RI + 1) & ~1, SIp = (a.SI + 1) & ~1;
  const int64_t fixed = (int64_t)a.RA * RIp + (((int64_t)a.SI * a.SO + 1) & ~1);
  const int m = std::max(std::max(a.RI, a.SI), 1);
  const bool lg = (a.og == 1);
  if (g_sandwich_reg && fixed + (int64_t)a.RI * SIp + 2 <= budget && a.SO <= 256 && m <= 48) {
    if (m <= 16) return lg ? "sandwich_reg_kernel<16, 2, true>" : "sandwich_reg_kernel<16, 2, false>";
    if (m <= 24) return lg ? "sandwich_reg_kernel<24, 2, true>" : "sandwich_reg_kernel<24, 2, false>";
    if (m <= 32) return lg ? "sandwich_reg_kernel<32, 1, true>" : "sandwich_reg_kernel<32, 1, false>";
    return lg ? "sandwich_reg_kernel<48, 1, true>" : "sandwich_reg_kernel<48, 1, false>";
  }
  return lg ? "sandwich_kernel<true>" : "sandwich_kernel<false>";
}

bool sandwich_supported(const SandwichArgs &a) {
  if (a.n <= 0 || a.G <= 0 || a.batch <= 0) return true;
  const int64_t budget = 19456;
  SwPlan pl;
  if ((g_sandwich_mfma || a.prec) && sandwich_mfma_plan(a, kSandwichLdsDoubles, &pl)) return true;
  if (a.prec) return false;
  // the scalar kernel is the last resort: one YL and ZR slice and at least one
  // sketch column of intermediates must fit in LDS
  const int64_t fixed = (int64_t)a.RA * a.RI + (int64_t)a.SI * a.SO;
  const int64_t perg = (int64_t)a.RI * a.SI + (int64_t)a.RI * a.SO;
  const int64_t gc = std::min<int64_t>(8, (budget - fixed) / perg);
  return gc >= 1 && a.n < (1LL << 31) && (a.G + gc - 1) / gc <= 65535 && a.batch <= 65535;
}

hipError_t launch_sandwich(const SandwichArgs &a, hipStream_t s, const SwForce *force) {
  if (a.n <= 0 || a.G <= 0 || a.batch <= 0) return hipSuccess;
  const int64_t budget = 19456;  // doubles of dynamic LDS
  const bool valu = force != nullptr && force->valu && !a.prec;
  if ((g_sandwich_mfma && !valu) || a.prec) {
    SwPlan pl;
    if (sandwich_mfma_plan(a, kSandwichLdsDoubles, &pl, force)) return launch_sandwich_mfma(a, pl, s);
    if (a.prec) return hipErrorInvalidValue;  // the FP32 / BF16 variants exist only on the matrix cores
  }
  if (g_sandwich_reg) {
    const int RIp = (a.RI + 1) & ~1, SIp = (a.SI + 1) & ~1;
    const int64_t fixed = (int64_t)a.RA * RIp + (((int64_t)a.SI * a.SO + 1) & ~1);
    if (fixed + (int64_t)a.RI * SIp + 2 <= budget) {
      bool done = false;
      hipError_t e = (a.og == 1) ? sandwich_reg_dispatch<true>(a, s, budget, &done)
                                 : sandwich_reg_dispatch<false>(a, s, budget, &done);
      if (done) return e;
    }
  }
  const int64_t fixed = (int64_t)a.RA * a.RI + (int64_t)a.SI * a.SO;
  const int64_t perg = (int64_t)a.RI * a.SI + (int64_t)a.RI * a.SO;
  int64_t gc = std::min<int64_t>(8, (budget - fixed) / perg);
  if (gc < 1) return hipErrorInvalidValue;
  gc = std::min<int64_t>(gc, a.G);
  const size_t lds = (size_t)(fixed + gc * perg) * sizeof(double);
  dim3 grid((unsigned)a.n, (unsigned)((a.G + gc - 1) / gc), (unsigned)a.batch);
  static std::once_flag attr_done;  // set once: the maximum a launch may ask for
  std::call_once(attr_done, [&] {
    hipFuncSetAttribute((const void *)sandwich_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)(budget * sizeof(double)));
    hipFuncSetAttribute((const void *)sandwich_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)(budget * sizeof(double)));
  });
  if (a.og == 1) sandwich_kernel<true><<<grid, 256, lds, s>>>(a, (int)gc);
  else sandwich_kernel<false><<<grid, 256, lds, s>>>(a, (int)gc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// x[p * bs + k] *= alpha[p] (invert = 0) or /= alpha[p] (invert = 1), k < count.
__global__ void scale_by_kernel(double *x, int64_t count, int64_t bs, const double *alpha, int invert) {
  const int p = blockIdx.y;
  const double a = invert ? 1.0 / alpha[p] : alpha[p];
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x)
    x[p * bs + k] *= a;
}

hipError_t launch_scale_by(double *x, int64_t count, int64_t bs, const double *alpha, int invert, int batch,
                           hipStream_t s) {
  if (count <= 0 || batch <= 0) return hipSuccess;
  dim3 grid((unsigned)std::min<int64_t>((count + 255) / 256, 4096), (unsigned)batch);
  scale_by_kernel<<<grid, 256, 0, s>>>(x, count, bs, alpha, invert);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ void copy_kernel(CMat src, Mat dst, int64_t M, int64_t N, int batch) {
  const int64_t per = M * N, total = per * batch;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / per, rem = e - p * per;
    const int64_t r = rem / N, c = rem - r * N;
    dst.ptr[p * dst.bs + r * dst.rs + c * dst.cs] = src.ptr[p * src.bs + r * src.rs + c * src.cs];
  }
}

__global__ void cast_f32_kernel(const double *src, int64_t sbs, float *dst, int64_t dbs, int64_t count, int batch) {
  const int64_t total = count * batch;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / count, k = e - p * count;
    dst[p * dbs + k] = (float)src[p * sbs + k];
  }
}

hipError_t launch_cast_f32(const double *src, int64_t sbs, float *dst, int64_t dbs, int64_t count, int batch,
                           hipStream_t s) {
  const int64_t total = count * batch;
  if (total <= 0) return hipSuccess;
  int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  cast_f32_kernel<<<grid, 256, 0, s>>>(src, sbs, dst, dbs, count, batch);
  return hipGetLastError();
}

// flag[p] = 1, then 0 for every train p with a non-finite entry among its
// first `count` doubles (pair stride `stride`).  Every block scans a slice
// of one train and only ever stores 0, so the blocks need no ordering.
__global__ void finite_init_kernel(int *flag, int batch) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < batch) flag[p] = 1;
}

__global__ void finite_check_kernel(const double *data, int64_t count, int64_t stride, int *flag) {
  const int p = blockIdx.y;
  const double *a = data + p * stride;
  int bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(a[e]);
  if (__syncthreads_or(bad) && threadIdx.x == 0) flag[p] = 0;
}

hipError_t launch_finite_check(const double *data, int64_t count, int64_t stride, int batch, int *flag,
                               hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  finite_init_kernel<<<(batch + 255) / 256, 256, 0, s>>>(flag, batch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || count <= 0) return e;
  const int64_t blocks = std::min<int64_t>((count + 4095) / 4096, 1024);
  finite_check_kernel<<<dim3((unsigned)blocks, (unsigned)batch), 256, 0, s>>>(data, count, stride, flag);
  return hipGetLastError();
}

// Reversal of a train: core k (r0 x n x r1, row-major) becomes core d-1-k
// (r1 x n x r0) of the destination, dst(b, i, a) = src(a, i, b).  For each
// mode index i that is a transpose of an r0 x r1 matrix: a block moves one
// 32 x 32 tile through LDS, reading along b and writing along a, so both
// sides are coalesced.  blockIdx.x = tile (a-tile, b-tile, i), y = core,
// z = pair; blocks past a core's tile count return.
__global__ __launch_bounds__(256) void tt_reverse_kernel(RevArgs a) {
  __shared__ double tile[32][33];
  const int k = blockIdx.y, p = blockIdx.z;
  const int r0 = a.r0[k], n = a.n[k], r1 = a.r1[k];
  const int ta = (r0 + 31) / 32, tb = (r1 + 31) / 32;
  const int64_t t = blockIdx.x;
  if (t >= (int64_t)ta * tb * n) return;
  const int i = (int)(t / (ta * tb));
  const int rem = (int)(t - (int64_t)i * ta * tb);
  const int a0 = (rem / tb) * 32, b0 = (rem - (rem / tb) * tb) * 32;
  const double *src = a.src + p * a.sstride + a.soff[k];
  double *dst = a.dst + p * a.dstride + a.doff[k];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int aa = a0 + ty + 8 * u, bb = b0 + tx;
    if (aa < r0 && bb < r1) tile[ty + 8 * u][tx] = src[((int64_t)aa * n + i) * r1 + bb];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int bb = b0 + ty + 8 * u, aa = a0 + tx;
    if (aa < r0 && bb < r1) dst[((int64_t)bb * n + i) * r0 + aa] = tile[tx][ty + 8 * u];
  }
}

hipError_t launch_tt_reverse(const RevArgs &a, int64_t max_tiles, int batch, hipStream_t s) {
  if (batch <= 0 || a.d <= 0) return hipSuccess;
  if (a.d > kRevMaxCores || max_tiles <= 0 || max_tiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  tt_reverse_kernel<<<dim3((unsigned)max_tiles, (unsigned)a.d, (unsigned)batch), 256, 0, s>>>(a);
  return hipGetLastError();
}

// dst[p][k] = src[p][d - k], k = 0..d (the kept ranks of a reversed train).
__global__ void rank_reverse_kernel(const int64_t *src, int64_t *dst, int d, int batch) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)batch * (d + 1)) return;
  const int64_t p = e / (d + 1);
  const int k = (int)(e - p * (d + 1));
  dst[e] = src[p * (d + 1) + (d - k)];
}

hipError_t launch_rank_reverse(const int64_t *src, int64_t *dst, int d, int batch, hipStream_t s) {
  const int64_t tot = (int64_t)batch * (d + 1);
  if (tot <= 0) return hipSuccess;
  rank_reverse_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(src, dst, d, batch);
  return hipGetLastError();
}

__global__ void cast_f64_kernel(const float *src, int64_t sbs, double *dst, int64_t dbs, int64_t count, int batch) {
  const int64_t total = count * batch;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / count, k = e - p * count;
    dst[p * dbs + k] = (double)src[p * sbs + k];
  }
}

hipError_t launch_cast_f64(const float *src, int64_t sbs, double *dst, int64_t dbs, int64_t count, int batch,
                           hipStream_t s) {
  const int64_t total = count * batch;
  if (total <= 0) return hipSuccess;
  int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  cast_f64_kernel<<<grid, 256, 0, s>>>(src, sbs, dst, dbs, count, batch);
  return hipGetLastError();
}

// Per pair, multiply w[p * bs .. + count) by the power of two that brings its
// largest magnitude into [1, 2) (exact: only the exponents change).  One
// block per pair.
__global__ __launch_bounds__(256) void rescale_pow2_kernel(float *w, int64_t count, int64_t bs) {
  __shared__ float part[256];
  float *v = w + (int64_t)blockIdx.x * bs;
  float m = 0.f;
  for (int64_t e = threadIdx.x; e < count; e += 256) m = fmaxf(m, fabsf(v[e]));
  part[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) part[threadIdx.x] = fmaxf(part[threadIdx.x], part[threadIdx.x + h]);
    __syncthreads();
  }
  m = part[0];
  if (!(m > 0.f) || !(m < INFINITY)) return;  // zero or non-finite: leave as is
  int ex;
  (void)frexpf(m, &ex);                       // m = f 2^ex, f in [0.5, 1)
  const float sc = ldexpf(1.f, 1 - ex);        // m sc in [1, 2)
  for (int64_t e = threadIdx.x; e < count; e += 256) v[e] *= sc;
}

hipError_t launch_rescale_pow2(float *w, int64_t count, int64_t bs, int batch, hipStream_t s) {
  if (count <= 0 || batch <= 0) return hipSuccess;
  rescale_pow2_kernel<<<batch, 256, 0, s>>>(w, count, bs);
  return hipGetLastError();
}

hipError_t launch_copy(CMat src, Mat dst, int64_t M, int64_t N, int batch, hipStream_t s) {
  const int64_t total = M * N * batch;
  if (total <= 0) return hipSuccess;
  int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  copy_kernel<<<grid, 256, 0, s>>>(src, dst, M, N, batch);
  return hipGetLastError();
}

__global__ void add_kernel(CMat src, Mat dst, int64_t M, int64_t N, int batch) {
  const int64_t per = M * N, total = per * batch;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / per, rem = e - p * per;
    const int64_t r = rem / N, c = rem - r * N;
    dst.ptr[p * dst.bs + r * dst.rs + c * dst.cs] += src.ptr[p * src.bs + r * src.rs + c * src.cs];
  }
}

hipError_t launch_add(CMat src, Mat dst, int64_t M, int64_t N, int batch, hipStream_t s) {
  const int64_t total = M * N * batch;
  if (total <= 0) return hipSuccess;
  int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  add_kernel<<<grid, 256, 0, s>>>(src, dst, M, N, batch);
  return hipGetLastError();
}

__global__ void fill_kernel(double *p, int64_t count, double v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}
__global__ void fill_i64_kernel(int64_t *p, int64_t count, int64_t v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

hipError_t launch_fill(double *p, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int grid = (int)std::min<int64_t>((count + 255) / 256, 65536);
  fill_kernel<<<grid, 256, 0, s>>>(p, count, v);
  return hipGetLastError();
}
hipError_t launch_fill_i64(int64_t *p, int64_t count, int64_t v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int grid = (int)std::min<int64_t>((count + 255) / 256, 65536);
  fill_i64_kernel<<<grid, 256, 0, s>>>(p, count, v);
  return hipGetLastError();
}

struct RankPattern {
  int64_t v[kMaxRankPattern];
};
__global__ void rank_pattern_kernel(int64_t *dst, int batch, int len, RankPattern pat) {
  const int64_t total = (int64_t)batch * len;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = pat.v[e % len];
}

hipError_t launch_rank_pattern(int64_t *dst, int batch, int len, const int64_t *host_pattern, hipStream_t s) {
  if (len > kMaxRankPattern) return hipErrorInvalidValue;
  RankPattern pat;
  for (int k = 0; k < len; ++k) pat.v[k] = host_pattern[k];
  const int64_t total = (int64_t)batch * len;
  if (total <= 0) return hipSuccess;
  int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
  rank_pattern_kernel<<<grid, 256, 0, s>>>(dst, batch, len, pat);
  return hipGetLastError();
}

// Frobenius norm of each pair's contiguous block, fixed reduction order.
__global__ __launch_bounds__(256) void block_norm_kernel(const double *x, int64_t count, int64_t bs,
                                                         double *out) {
  __shared__ double red[256];
  const int p = blockIdx.x;
  const double *xp = x + p * bs;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < count; e += 256) acc += xp[e] * xp[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p] = sqrt(red[0]);
}

hipError_t launch_block_norm(const double *x, int64_t count, int64_t bs, double *out, int batch,
                             hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  block_norm_kernel<<<batch, 256, 0, s>>>(x, count, bs, out);
  return hipGetLastError();
}

}  // namespace hatt
