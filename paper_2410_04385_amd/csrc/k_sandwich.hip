// The sandwich contraction on the FP64 matrix cores.
//
// For one pair p, one mode index i and a chunk of GC sketch columns g, the
// kernel forms out_g = YL_i C_g ZR_i (RA x RI, RI x SI, SI x SO) as two
// products (the same operation as sandwich_kernel, see common.h):
//   stage 1  T = [C_g0; C_g1; ...] ZR      rows (g, a) stacked, K = SI
//   stage 2  out = YL [T_g0 | T_g1 | ...]  columns (g, b') side by side, K = RI
// Both run on v_mfma_f64_16x16x4f64 (16 x 16 output blocks, K steps of 4);
// every operand sits in LDS, zero-padded to whole blocks.  Stage 1 stacks the
// g blocks along M and stage 2 along N, so only the short dimension of each
// product is padded to 16.  The column order of stage 2 is chosen so that the
// 16 lanes of an output row segment store to consecutive addresses:
// (b', g) with g fastest when the output is contiguous in g, (g, b') otherwise
// (the column-major W_L of HPCRL and the core update, both contiguous in b').
#include <mutex>
#include "common.h"
#include "stage.h"

namespace hatt {

namespace {
__host__ __device__ inline int rup(int x, int m) { return (x + m - 1) / m * m; }
}  // namespace

// K steps of the generic kernel's MFMA chains: up to 32 (K <= 128), run in
// unrolled chunks of 16.
constexpr int kSwMaxKSteps = 32;

// Register slots per thread for the next chunk of sketch columns in the
// slice-major kernel (its chunk holds at most 256 * kSlicePf C entries).
constexpr int kSlicePf = 24;

bool g_sandwich_slice = true;

// Slice-major plan (FP64, output not contiguous in g): LDS holds YL and ZR of
// one slice, a chunk of GC sketch columns C_g (rows (g, a), K = b) and the
// stage-1 result T; the block walks its gpb sketch columns chunk by chunk.
static bool sandwich_slice_plan(const SandwichArgs &a, int64_t budget, SwPlan *pl) {
  if (a.prec != 0 || a.og == 1) return false;
  const int RI4 = rup(a.RI, 4), SI4 = rup(a.SI, 4);
  const int SO16 = rup(a.SO, 16), RA16 = rup(a.RA, 16);
  if (RI4 > 4 * kSwMaxKSteps || SI4 > 4 * kSwMaxKSteps) return false;
  const int ldc = SI4 + 1, ldz = SO16 + 1, ldy = RI4 + 1;
  const int64_t fixed = (int64_t)RA16 * ldy + (int64_t)SI4 * ldz;
  int best = 0, bm1 = 0, bldt = 0;
  for (int gc = (int)std::min<int64_t>(8, a.G); gc >= 1; --gc) {
    const int m1 = rup(gc * a.RI, 16), ldt = rup(gc * a.SO, 16) + 1;
    if ((int64_t)m1 * SI4 > 256LL * kSlicePf) continue;
    if (fixed + (int64_t)m1 * ldc + (int64_t)RI4 * ldt <= budget) {
      best = gc;
      bm1 = m1;
      bldt = ldt;
      break;
    }
  }
  if (best == 0) return false;
  // output and C offsets within a block are 32-bit
  const int64_t omax = (int64_t)(best - 1) * std::llabs(a.og) + (int64_t)(a.SO - 1) * std::llabs(a.obb) +
                       (int64_t)(a.RA - 1) * std::llabs(a.oa);
  const int64_t cmax = (int64_t)(best - 1) * std::llabs(a.cg) + (int64_t)(a.RI - 1) * std::llabs(a.ca) +
                       (int64_t)(a.SI - 1) * std::llabs(a.cbb);
  if (omax >= (1LL << 31) || cmax >= (1LL << 31) || bm1 >= (1 << 16) || bldt >= (1 << 16)) return false;
  pl->slice = 1;
  pl->ks = 0;
  pl->rem = 0;
  pl->nbuf = 1;
  pl->pf = 0;
  pl->GC = best;
  pl->RI4 = RI4;
  pl->SI4 = SI4;
  pl->SO16 = SO16;
  pl->RA16 = RA16;
  pl->ldc = ldc;
  pl->ldz = ldz;
  pl->ldy = ldy;
  pl->ldt = bldt;
  pl->M1 = bm1;
  pl->fd_ri = make_fastdiv(a.RI);
  pl->fd_so = make_fastdiv(a.SO);
  pl->fd_gc = make_fastdiv(best);
  pl->lds_doubles = fixed + (int64_t)bm1 * ldc + (int64_t)RI4 * bldt;
  // one slice per block; split g only when the slices alone leave the CUs idle
  const int64_t slices = a.n * (int64_t)a.batch;
  const int64_t chunks = (a.G + best - 1) / best;
  int64_t gbl = std::max<int64_t>(1, std::min<int64_t>(chunks, (512 + slices - 1) / slices));
  const int64_t cpb = (chunks + gbl - 1) / gbl;
  pl->gpb = (int)(cpb * best);
  pl->gblocks = (int)((a.G + pl->gpb - 1) / pl->gpb);
  pl->ipb = 1;
  pl->iblocks = (int)a.n;
  pl->chunks = pl->gblocks;
  return pl->iblocks >= 1 && a.n < (1LL << 31) && pl->gblocks <= 65535;
}

// Largest K-step count with a register-blocked instantiation, and its fetch
// slots per thread for the next slice's YL / ZR entries.
constexpr int kSwKsMax = 8;
__host__ __device__ constexpr int sw_ks_slots(int ks) { return ks <= 2 ? 2 : (ks <= 4 ? 4 : 8); }

bool sandwich_mfma_plan(const SandwichArgs &a, int64_t budget, SwPlan *pl, const SwForce *force) {
  // K edges: whole K steps of 4, or whole K-16 BF16 MFMAs.  The budget is
  // given in doubles; BF16 plans count 2-byte elements, so they get four per
  // double (FP32 plans keep the FP64 element count)
  const int kq = (a.prec == 2) ? 16 : 4;
  const int64_t per_double = (a.prec == 2) ? 4 : 1;
  budget *= per_double;
  const int RI4 = rup(a.RI, kq), SI4 = rup(a.SI, kq);
  const int SO16 = rup(a.SO, 16), RA16 = rup(a.RA, 16);
  const int ldc = SI4 + 1, ldz = SO16 + 1, ldy = RI4 + 1;
  const int64_t yz = (int64_t)SI4 * ldz + (int64_t)RA16 * ldy;  // one YL + ZR buffer
  // the register prefetch of the next slice needs every YL / ZR slot to fit
  // kSwPrefetch slots per thread (else each slice is staged directly)
  bool pf = (int64_t)RA16 * RI4 + (int64_t)SI4 * SO16 <= kSwPrefetch * 256;
  int nbuf = 2;
  auto lds_for = [&](int gc, int *ldt, int *m1) {
    *m1 = rup(gc * a.RI, 16);
    *ldt = rup(gc * a.SO, 16) + 1;
    return (int64_t)(*m1) * ldc + nbuf * yz + (int64_t)RI4 * (*ldt);
  };
  // largest chunk (<= 16 columns) that keeps two blocks per CU, unless one
  // block per CU takes at least twice as many columns of a chunk below four
  // (the slices are then staged for too little work); failing both, one
  // YL / ZR buffer (the next slice is staged after this one's products,
  // large factor ranks)
  auto largest = [&](int64_t lim) {
    for (int gc = (int)std::min<int64_t>(16, a.G); gc >= 1; --gc) {
      int ldt, m1;
      if (lds_for(gc, &ldt, &m1) <= lim) return gc;
    }
    return 0;
  };
  int best = largest(std::min<int64_t>(budget, 9728 * per_double));
  if (best < 4) {
    const int one = largest(budget);
    if (one > 0 && (best == 0 || one >= 2 * best)) best = one;
  }
  if (best == 0) {
    nbuf = 1;
    best = largest(budget);
  }
  if (best == 0) return false;
  if (force != nullptr && force->gc_div > 1) best = std::max(1, best / force->gc_div);
  pl->nbuf = nbuf;
  if (nbuf == 1) pf = false;
  const int64_t chunks = (a.G + best - 1) / best;
  const int GC = (int)((a.G + chunks - 1) / chunks);  // balanced chunks
  int ldt, m1;
  pl->lds_doubles = lds_for(GC, &ldt, &m1);
  pl->GC = GC;
  pl->chunks = (int)chunks;
  pl->RI4 = RI4;
  pl->SI4 = SI4;
  pl->SO16 = SO16;
  pl->RA16 = RA16;
  pl->ldc = ldc;
  pl->ldz = ldz;
  pl->ldy = ldy;
  pl->ldt = ldt;
  pl->M1 = m1;
  pl->fd_ri = make_fastdiv(a.RI);
  pl->fd_so = make_fastdiv(a.SO);
  pl->fd_gc = make_fastdiv(GC);
  // the multiply-high decodes need row / column indices below 2^16 and divisors <= 4096
  if (m1 >= (1 << 16) || ldt >= (1 << 16) || a.RI > 4096 || a.SO > 4096) return false;
  if (RI4 > 4 * kSwMaxKSteps || SI4 > 4 * kSwMaxKSteps) return false;  // K steps of the MFMA loops
  // slices per block: about 2048 blocks in the grid; C is staged once per block
  const int64_t others = chunks * (int64_t)a.batch;
  int64_t ipb = std::max<int64_t>(1, (a.n * others) / 2048);
  ipb = std::min<int64_t>(ipb, a.n);
  pl->iblocks = (int)((a.n + ipb - 1) / ipb);
  pl->ipb = (int)((a.n + pl->iblocks - 1) / pl->iblocks);  // balanced
  // prefetch offsets are 32-bit
  const int64_t ymax = (int64_t)(a.RA - 1) * std::llabs(a.ylr) + (int64_t)(a.RI - 1) * std::llabs(a.ylc);
  const int64_t zmax = (int64_t)(a.SI - 1) * std::llabs(a.zrr) + (int64_t)(a.SO - 1) * std::llabs(a.zrc);
  const bool off32 = ymax < (1LL << 31) && zmax < (1LL << 31);
  pf = pf && off32;
  pl->pf = pf ? 1 : 0;
  // register-blocked kernel: equal K steps, every valid YL / ZR entry in a
  // fetch slot, block counts that divide the four waves, 32-bit output offsets
  pl->ks = 0;
  const int64_t omax = (a.G - 1) * std::llabs(a.og) + (int64_t)(a.SO - 1) * std::llabs(a.obb) +
                       (int64_t)(a.RA - 1) * std::llabs(a.oa);
  if (off32 && omax < (1LL << 31) && RI4 == SI4 && RI4 / 4 <= kSwKsMax && 4 % (SO16 / 16) == 0 &&
      4 % (RA16 / 16) == 0 && (int64_t)a.RA * a.RI + (int64_t)a.SI * a.SO <= 256LL * sw_ks_slots(RI4 / 4))
    pl->ks = RI4 / 4;
  if (pl->nbuf != 2 || a.prec == 2) pl->ks = 0;  // the register-blocked kernel has no BF16 form
  if (force != nullptr && force->no_ks) pl->ks = 0;
  pl->rem = (pl->ks > 0 && a.prec == 0 && a.og != 1 && a.SO >= 17 && a.SO <= 20 && a.RA >= 17 && a.RA <= 20) ? 1 : 0;
  pl->slice = 0;
  // large factor ranks leave room for a single YL / ZR slice buffer next to
  // the sketch columns: there the slice-major kernel stages each slice once
  // and streams the sketch columns instead
  if (g_sandwich_slice && pl->ks == 0 && pl->nbuf == 1 && !(force != nullptr && force->no_slice)) {
    SwPlan sp = *pl;
    if (sandwich_slice_plan(a, budget, &sp)) *pl = sp;
  }
  return true;
}

// Two 16 x 16 output blocks per pass (two accumulation chains in flight):
// c0 += A0 B0, c1 += A1 B1 over K steps of 4 (A rows advance by lda_k per
// step, B rows by ldb_k).  Both chains always run; a caller without a second
// block passes the first block's operands twice and drops c1.
template <typename CT, typename ACC>
__device__ __forceinline__ void mfma_pair(const CT *a0, const CT *b0, const CT *a1, const CT *b1, int lda_k,
                                          int ldb_k, int ksteps, ACC &c0, ACC &c1) {
  for (int k0 = 0; k0 < ksteps; k0 += 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if (k0 + k < ksteps) {
        const int kk = k0 + k;
        const CT x0 = a0[kk * lda_k], y0 = b0[kk * ldb_k];
        const CT x1 = a1[kk * lda_k], y1 = b1[kk * ldb_k];
        c0 = mfma16(x0, y0, c0);
        c1 = mfma16(x1, y1, c1);
      }
    }
  }
}

// BF16: the same chains with one K-16 MFMA per four K steps (ksteps is a
// multiple of 4: the BF16 plans pad K to 16 with zeros).
template <typename ACC>
__device__ __forceinline__ void mfma_pair(const __bf16 *a0, const __bf16 *b0, const __bf16 *a1, const __bf16 *b1,
                                          int lda_k, int ldb_k, int ksteps, ACC &c0, ACC &c1) {
  for (int k0 = 0; k0 < ksteps; k0 += 4) {
    __bf16 x0[4], y0[4], x1[4], y1[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      x0[e] = a0[(k0 + e) * lda_k];
      y0[e] = b0[(k0 + e) * ldb_k];
      x1[e] = a1[(k0 + e) * lda_k];
      y1[e] = b1[(k0 + e) * ldb_k];
    }
    c0 = mfma16_bf16(x0, y0, c0);
    c1 = mfma16_bf16(x1, y1, c1);
  }
}

// One chain, for a wave whose last tile has no partner.
template <typename CT, typename ACC>
__device__ __forceinline__ void mfma_one(const CT *a0, const CT *b0, int lda_k, int ldb_k, int ksteps, ACC &c0) {
  for (int k0 = 0; k0 < ksteps; k0 += 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if (k0 + k < ksteps) c0 = mfma16(a0[(k0 + k) * lda_k], b0[(k0 + k) * ldb_k], c0);
    }
  }
}
template <typename ACC>
__device__ __forceinline__ void mfma_one(const __bf16 *a0, const __bf16 *b0, int lda_k, int ldb_k, int ksteps,
                                         ACC &c0) {
  for (int k0 = 0; k0 < ksteps; k0 += 4) {
    __bf16 x0[4], y0[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      x0[e] = a0[(k0 + e) * lda_k];
      y0[e] = b0[(k0 + e) * ldb_k];
    }
    c0 = mfma16_bf16(x0, y0, c0);
  }
}

// CT: compute and LDS type (FP64, or FP32 / BF16 for the low-precision
// range finding); C and the output are stored in ST (CT, FP32 for BF16), YL
// and ZR (cores of x and y) in FP64.
template <bool LG, typename CT>
__global__ __launch_bounds__(256) void sandwich_mfma_kernel(SandwichArgs a, SwPlan pl) {
  using acc_t = typename std::conditional<std::is_same<CT, double>::value, d4_t, f4_t>::type;
  using ST = typename std::conditional<is_bf16<CT>::value, float, CT>::type;
  extern __shared__ double smraw[];
  CT *sm = reinterpret_cast<CT *>(smraw);
  const int RA = a.RA, RI = a.RI, SI = a.SI, SO = a.SO;
  const int GC = pl.GC;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: tile loops stay scalar
  const int r16 = lane & 15, q4 = lane >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * pl.ipb;
  const int64_t i1 = std::min<int64_t>(a.n, i0 + pl.ipb);
  const int64_t g0 = (int64_t)blockIdx.y * GC;
  const int p = blockIdx.z;
  const int gc = (int)std::min<int64_t>(GC, a.G - g0);
  if (gc <= 0 || i0 >= i1) return;
  const int yzs = pl.SI4 * pl.ldz + pl.RA16 * pl.ldy;
  CT *Cs = sm;                               // pl.M1 rows (g, a) x ldc, K = b
  CT *YZ0 = Cs + pl.M1 * pl.ldc;             // [ZR: SI4 x ldz | YL: RA16 x ldy], two buffers
  CT *Ts = YZ0 + pl.nbuf * yzs;              // RI4 rows (a) x ldt, N = stage-2 columns
  const int M1 = gc * RI;                    // valid stage-1 rows
  const int M1p = rup(M1, 16);

  // ---- C chunk (fixed for all slices of this block), zero K padding
  const ST *cbase = reinterpret_cast<const ST *>(static_cast<const void *>(a.c)) + p * a.cb + g0 * a.cg;
  if (a.cg == 1) {  // g fastest in memory: consecutive threads take consecutive g
    stage_lds<8>(gc * RI * pl.SI4, Rad3(tid, 256, gc, pl.SI4), Cs,  // digits (g, b, a)
                 [&](const Rad3 &d) {
                   return (d.i1 < SI) ? (double)cbase[d.i0 * a.cg + d.i2 * a.ca + d.i1 * a.cbb] : 0.0;
                 },
                 [&](const Rad3 &d) { return (d.i0 * RI + d.i2) * pl.ldc + d.i1; });
  } else {
    stage_lds<8>(gc * RI * pl.SI4, Rad3(tid, 256, pl.SI4, RI), Cs,  // digits (b, a, g)
                 [&](const Rad3 &d) {
                   return (d.i0 < SI) ? (double)cbase[d.i2 * a.cg + d.i1 * a.ca + d.i0 * a.cbb] : 0.0;
                 },
                 [&](const Rad3 &d) { return (d.i2 * RI + d.i1) * pl.ldc + d.i0; });
  }
  for (int e = tid; e < (M1p - M1) * pl.SI4; e += 256) {
    const int r = M1 + e / pl.SI4, k = e - (e / pl.SI4) * pl.SI4;
    Cs[r * pl.ldc + k] = to_ct<CT>(0.0);
  }
  // rows a >= RI of T are K padding of stage 2: zero once
  for (int e = tid; e < (pl.RI4 - RI) * pl.ldt; e += 256) Ts[RI * pl.ldt + e] = to_ct<CT>(0.0);

  // ---- YL / ZR slots of this thread: slot u is element tid + 256 u of the
  // padded [ZR | YL] grid; kind 0 = zero padding, 1 = ZR entry, 2 = YL entry
  int pf_lds[kSwPrefetch], pf_off[kSwPrefetch];
  int pf_kind = 0;
  const int nz = pl.SI4 * pl.SO16, ny = pl.RA16 * pl.RI4;
#pragma unroll
  for (int u = 0; u < kSwPrefetch; ++u) {
    const int e = tid + 256 * u;
    pf_lds[u] = -1;
    pf_off[u] = 0;
    if (e < nz) {
      const int b = e / pl.SO16, bp = e - b * pl.SO16;
      pf_lds[u] = b * pl.ldz + bp;
      if (b < SI && bp < SO) {
        pf_kind |= 1 << (2 * u);
        pf_off[u] = (int)(b * a.zrr + bp * a.zrc);
      }
    } else if (e < nz + ny) {
      const int f = e - nz, ap = f / pl.RI4, k = f - ap * pl.RI4;
      pf_lds[u] = pl.SI4 * pl.ldz + ap * pl.ldy + k;
      if (ap < RA && k < RI) {
        pf_kind |= 2 << (2 * u);
        pf_off[u] = (int)(ap * a.ylr + k * a.ylc);
      }
    }
  }
  const double *zrp = a.zr + p * a.zrb;
  const double *ylp = a.yl + p * a.ylb;
  double pf[kSwPrefetch];
  auto fetch = [&](int64_t i) {
    const double *zr = zrp + i * a.zri, *yl = ylp + i * a.yli;
#pragma unroll
    for (int u = 0; u < kSwPrefetch; ++u) {
      const int k = (pf_kind >> (2 * u)) & 3;
      pf[u] = (k == 1) ? zr[pf_off[u]] : ((k == 2) ? yl[pf_off[u]] : 0.0);
    }
  };
  auto park = [&](CT *buf) {
#pragma unroll
    for (int u = 0; u < kSwPrefetch; ++u)
      if (pf_lds[u] >= 0) buf[pf_lds[u]] = to_ct<CT>(pf[u]);
  };
  // without the register prefetch: stage slice i straight into buf
  auto stage_direct = [&](int64_t i, CT *buf) {
    const double *zr = zrp + i * a.zri, *yl = ylp + i * a.yli;
    stage_lds<4>(pl.SI4 * pl.SO16, Rad3(tid, 256, pl.SO16, pl.SI4), buf,  // digits (b', b)
                 [&](const Rad3 &d) {
                   return (d.i1 < SI && d.i0 < SO) ? zr[(int64_t)d.i1 * a.zrr + (int64_t)d.i0 * a.zrc] : 0.0;
                 },
                 [&](const Rad3 &d) { return d.i1 * pl.ldz + d.i0; });
    stage_lds<4>(pl.RA16 * pl.RI4, Rad3(tid, 256, pl.RI4, pl.RA16), buf + pl.SI4 * pl.ldz,  // digits (a, a')
                 [&](const Rad3 &d) {
                   return (d.i1 < RA && d.i0 < RI) ? yl[(int64_t)d.i1 * a.ylr + (int64_t)d.i0 * a.ylc] : 0.0;
                 },
                 [&](const Rad3 &d) { return d.i1 * pl.ldy + d.i0; });
  };
  const bool pfr = pl.pf != 0;
  if (pfr) {
    fetch(i0);
    park(YZ0);
  } else {
    stage_direct(i0, YZ0);
  }
  __syncthreads();

  const int nt1 = pl.SO16 / 16, tiles1 = (M1p / 16) * nt1;
  const int ncols = LG ? SO * GC : gc * SO;
  const int nt2 = rup(ncols, 16) / 16, tiles2 = (pl.RA16 / 16) * nt2;
  int buf = 0;
  for (int64_t i = i0; i < i1; ++i) {
    const bool more = i + 1 < i1;
    if (more && pfr) fetch(i + 1);  // in flight during the MFMAs below
    const CT *ZRs = YZ0 + buf * yzs;
    const CT *YLs = ZRs + pl.SI4 * pl.ldz;

    // ---- stage 1: T(g, a; b') = sum_b C_g(a, b) ZR(b, b'), scattered into Ts
    for (int t = wave; t < tiles1; t += 8) {
      const int t2 = t + 4;
      const bool two = t2 < tiles1;
      const int tm0 = (t / nt1) * 16, tn0 = (t - (t / nt1) * nt1) * 16;
      const int tm1 = two ? (t2 / nt1) * 16 : tm0, tn1 = two ? (t2 - (t2 / nt1) * nt1) * 16 : tn0;
      acc_t c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
      if (two)  // wave-uniform: the tile index derives from the wave number only
        mfma_pair(Cs + (tm0 + r16) * pl.ldc + q4, ZRs + q4 * pl.ldz + tn0 + r16, Cs + (tm1 + r16) * pl.ldc + q4,
                  ZRs + q4 * pl.ldz + tn1 + r16, 4, 4 * pl.ldz, pl.SI4 / 4, c0, c1);
      else
        mfma_one(Cs + (tm0 + r16) * pl.ldc + q4, ZRs + q4 * pl.ldz + tn0 + r16, 4, 4 * pl.ldz, pl.SI4 / 4, c0);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (u == 1 && !two) break;
        const acc_t &c = u ? c1 : c0;
        const int tm = u ? tm1 : tm0, bq = (u ? tn1 : tn0) + r16;
        if (bq < SO) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = tm + mfma_row<CT>(q4, v);
            if (row < M1) {
              const int g = fdiv(row, pl.fd_ri), aa = row - g * RI;
              const int col = LG ? bq * GC + g : g * SO + bq;
              Ts[aa * pl.ldt + col] = to_ct<CT>(c[v]);
            }
          }
        }
      }
    }
    __syncthreads();

    // ---- stage 2: out(a', col) = sum_a YL(a', a) T(a, col)
    ST *obase = reinterpret_cast<ST *>(static_cast<void *>(a.o)) + p * a.ob + i * a.oi + g0 * a.og;
    for (int t = wave; t < tiles2; t += 8) {
      const int t2 = t + 4;
      const bool two = t2 < tiles2;
      const int tm0 = (t / nt2) * 16, tn0 = (t - (t / nt2) * nt2) * 16;
      const int tm1 = two ? (t2 / nt2) * 16 : tm0, tn1 = two ? (t2 - (t2 / nt2) * nt2) * 16 : tn0;
      acc_t c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
      if (two)
        mfma_pair(YLs + (tm0 + r16) * pl.ldy + q4, Ts + q4 * pl.ldt + tn0 + r16, YLs + (tm1 + r16) * pl.ldy + q4,
                  Ts + q4 * pl.ldt + tn1 + r16, 4, 4 * pl.ldt, pl.RI4 / 4, c0, c1);
      else
        mfma_one(YLs + (tm0 + r16) * pl.ldy + q4, Ts + q4 * pl.ldt + tn0 + r16, 4, 4 * pl.ldt, pl.RI4 / 4, c0);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (u == 1 && !two) break;
        const acc_t &c = u ? c1 : c0;
        const int tm = u ? tm1 : tm0, col = (u ? tn1 : tn0) + r16;
        int g, bq;
        if (LG) {
          bq = fdiv(col, pl.fd_gc);
          g = col - bq * GC;
        } else {
          g = fdiv(col, pl.fd_so);
          bq = col - g * SO;
        }
        if (col < ncols && g < gc) {
          ST *o = obase + g * a.og + bq * a.obb + (int64_t)tm * a.oa;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int rr = mfma_row<CT>(q4, v);
            if (tm + rr < RA) o[(int64_t)rr * a.oa] = (ST)c[v];
          }
        }
      }
    }
    if (more) {
      if (pl.nbuf == 1) {
        __syncthreads();  // every wave is done with this slice's YL / ZR
        stage_direct(i + 1, YZ0);
      } else if (pfr) {
        park(YZ0 + (buf ^ 1) * yzs);
      } else {
        stage_direct(i + 1, YZ0 + (buf ^ 1) * yzs);
      }
    }
    __syncthreads();  // Ts and the YL / ZR buffer are reused by the next slice
    if (pl.nbuf == 2) buf ^= 1;
  }
}

// Slice-major form of sandwich_mfma_kernel (FP64, the (g, b') column order)
// for large factor ranks: the block owns one mode index i, stages YL_i and
// ZR_i once, and walks its sketch columns GC at a time.  Each chunk's C
// entries are fetched into registers while the previous chunk's stage 1
// runs and parked in LDS once that stage is done, so the loads overlap the
// matrix-core work.  Stage 1 stacks the chunk's g blocks along M (rows
// (g, a), K = b), stage 2 places their results side by side along N
// (columns (g, b'), K = a), as in sandwich_mfma_kernel.
__global__ __launch_bounds__(256) void sandwich_slice_kernel(SandwichArgs a, SwPlan pl) {
  extern __shared__ double sm[];
  const int RA = a.RA, RI = a.RI, SI = a.SI, SO = a.SO;
  const int GC = pl.GC;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r16 = lane & 15, q4 = lane >> 4;
  const int64_t i = blockIdx.x;
  const int64_t gb0 = (int64_t)blockIdx.y * pl.gpb;
  const int64_t gb1 = std::min<int64_t>(a.G, gb0 + pl.gpb);
  const int p = blockIdx.z;
  if (i >= a.n || gb0 >= gb1) return;
  double *YLs = sm;                              // RA16 rows (a') x ldy, K = a
  double *ZRs = YLs + pl.RA16 * pl.ldy;          // SI4 rows (b) x ldz
  double *Cs = ZRs + pl.SI4 * pl.ldz;            // M1 rows (g, a) x ldc, K = b
  double *Ts = Cs + pl.M1 * pl.ldc;              // RI4 rows (a) x ldt, columns (g, b')
  {
    const double *zr = a.zr + p * a.zrb + i * a.zri, *yl = a.yl + p * a.ylb + i * a.yli;
    stage_lds<4>(pl.SI4 * pl.SO16, Rad3(tid, 256, pl.SO16, pl.SI4), ZRs,  // digits (b', b)
                 [&](const Rad3 &d) {
                   return (d.i1 < SI && d.i0 < SO) ? zr[(int64_t)d.i1 * a.zrr + (int64_t)d.i0 * a.zrc] : 0.0;
                 },
                 [&](const Rad3 &d) { return d.i1 * pl.ldz + d.i0; });
    stage_lds<4>(pl.RA16 * pl.RI4, Rad3(tid, 256, pl.RI4, pl.RA16), YLs,  // digits (a, a')
                 [&](const Rad3 &d) {
                   return (d.i1 < RA && d.i0 < RI) ? yl[(int64_t)d.i1 * a.ylr + (int64_t)d.i0 * a.ylc] : 0.0;
                 },
                 [&](const Rad3 &d) { return d.i1 * pl.ldy + d.i0; });
  }
  // rows a >= RI of T are K padding of stage 2
  for (int e = tid; e < (pl.RI4 - RI) * pl.ldt; e += 256) Ts[RI * pl.ldt + e] = 0.0;

  // C slots of this thread: slot u is entry tid + 256 u of the chunk's
  // (row, b) grid, row = g RI + a; stored at Cs[row * ldc + b], read from
  // C_{g0+g}(a, b) (zero for b >= SI or a row beyond the chunk)
  const int nce = pl.M1 * pl.SI4;
  // (a row beyond a short last chunk is one whose LDS index reaches gc RI ldc)
  int c_lds[kSlicePf], c_off[kSlicePf];
  unsigned c_ok = 0;
#pragma unroll
  for (int u = 0; u < kSlicePf; ++u) {
    const int e = tid + 256 * u;
    c_lds[u] = -1;
    c_off[u] = 0;
    if (e < nce) {
      const int row = e / pl.SI4, b = e - row * pl.SI4;
      c_lds[u] = row * pl.ldc + b;
      const int g = fdiv(row, pl.fd_ri), aa = row - g * RI;
      if (b < SI && g < GC) {
        c_ok |= 1u << u;
        c_off[u] = (int)(g * a.cg + aa * a.ca + b * a.cbb);
      }
    }
  }
  const double *cbase = a.c + p * a.cb;
  double cf[kSlicePf];
  auto cfetch = [&](int64_t g0, int gc) {
    const double *cp = cbase + g0 * a.cg;
    const int lim = gc * RI * pl.ldc;
#pragma unroll
    for (int u = 0; u < kSlicePf; ++u) cf[u] = (((c_ok >> u) & 1u) && c_lds[u] < lim) ? cp[c_off[u]] : 0.0;
  };
  auto cpark = [&]() {
#pragma unroll
    for (int u = 0; u < kSlicePf; ++u)
      if (c_lds[u] >= 0) Cs[c_lds[u]] = cf[u];
  };
  int gcur = (int)std::min<int64_t>(GC, gb1 - gb0);
  cfetch(gb0, gcur);
  cpark();
  __syncthreads();

  const int nt1 = pl.SO16 / 16;
  double *obase0 = a.o + p * a.ob + i * a.oi;
  for (int64_t g0 = gb0; g0 < gb1; g0 += GC) {
    const int gc = gcur;
    const int64_t gn = g0 + GC;
    const bool more = gn < gb1;
    int gnext = 0;
    if (more) {
      gnext = (int)std::min<int64_t>(GC, gb1 - gn);
      cfetch(gn, gnext);  // in flight during stage 1
    }
    const int M1 = gc * RI, M1p = rup(M1, 16);
    const int tiles1 = (M1p / 16) * nt1;
    // ---- stage 1: T(a; g, b') = sum_b C_g(a, b) ZR(b, b')
    for (int t = wave; t < tiles1; t += 8) {
      const int t2 = t + 4;
      const bool two = t2 < tiles1;
      const int tm0 = (t / nt1) * 16, tn0 = (t - (t / nt1) * nt1) * 16;
      const int tm1 = two ? (t2 / nt1) * 16 : tm0, tn1 = two ? (t2 - (t2 / nt1) * nt1) * 16 : tn0;
      d4_t c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
      if (two)
        mfma_pair(Cs + (tm0 + r16) * pl.ldc + q4, ZRs + q4 * pl.ldz + tn0 + r16, Cs + (tm1 + r16) * pl.ldc + q4,
                  ZRs + q4 * pl.ldz + tn1 + r16, 4, 4 * pl.ldz, pl.SI4 / 4, c0, c1);
      else
        mfma_one(Cs + (tm0 + r16) * pl.ldc + q4, ZRs + q4 * pl.ldz + tn0 + r16, 4, 4 * pl.ldz, pl.SI4 / 4, c0);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (u == 1 && !two) break;
        const d4_t &c = u ? c1 : c0;
        const int tm = u ? tm1 : tm0, bq = (u ? tn1 : tn0) + r16;
        if (bq < SO) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = tm + mfma_row<double>(q4, v);
            if (row < M1) {
              const int g = fdiv(row, pl.fd_ri), aa = row - g * RI;
              Ts[aa * pl.ldt + g * SO + bq] = c[v];
            }
          }
        }
      }
    }
    __syncthreads();  // T complete; C of this chunk no longer read
    if (more) cpark();
    // ---- stage 2: out(a'; g, b') = sum_a YL(a', a) T(a; g, b')
    const int ncols = gc * SO;
    const int nt2 = rup(ncols, 16) / 16, tiles2 = (pl.RA16 / 16) * nt2;
    double *obase = obase0 + g0 * a.og;
    for (int t = wave; t < tiles2; t += 8) {
      const int t2 = t + 4;
      const bool two = t2 < tiles2;
      const int tm0 = (t / nt2) * 16, tn0 = (t - (t / nt2) * nt2) * 16;
      const int tm1 = two ? (t2 / nt2) * 16 : tm0, tn1 = two ? (t2 - (t2 / nt2) * nt2) * 16 : tn0;
      d4_t c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
      if (two)
        mfma_pair(YLs + (tm0 + r16) * pl.ldy + q4, Ts + q4 * pl.ldt + tn0 + r16, YLs + (tm1 + r16) * pl.ldy + q4,
                  Ts + q4 * pl.ldt + tn1 + r16, 4, 4 * pl.ldt, pl.RI4 / 4, c0, c1);
      else
        mfma_one(YLs + (tm0 + r16) * pl.ldy + q4, Ts + q4 * pl.ldt + tn0 + r16, 4, 4 * pl.ldt, pl.RI4 / 4, c0);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (u == 1 && !two) break;
        const d4_t &c = u ? c1 : c0;
        const int tm = u ? tm1 : tm0, col = (u ? tn1 : tn0) + r16;
        const int g = fdiv(col, pl.fd_so), bq = col - g * SO;
        if (col < ncols) {
          double *o = obase + g * a.og + bq * a.obb + (int64_t)tm * a.oa;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int rr = mfma_row<double>(q4, v);
            if (tm + rr < RA) o[(int64_t)rr * a.oa] = c[v];
          }
        }
      }
    }
    __syncthreads();  // T and the parked C chunk: next chunk
    gcur = gnext;
  }
}

// Register-blocked variant for KS K steps on both products (K padded to
// 4 KS), same LDS layout and grid as sandwich_mfma_kernel, for shapes whose
// stage-1 column-block count and stage-2 row-block count divide 4.  Wave w
// keeps one ZR block column (stage 1) and one YL block row (stage 2) in
// registers for the whole slice and takes every fourth block of the other
// operand; the fragments of its next block are read while the KS MFMAs of
// the current one run.  Block walks advance by fixed pointer steps and the
// epilogues decode one index per block (a row's (g, a) changes by at most
// one wrap between the four rows a lane holds), so address arithmetic stays
// well below the MFMA time.  Only the valid YL / ZR entries are fetched (the
// padding of both buffers is zeroed once).  The next slice's entries are
// parked after stage 1 and the one after that is fetched before stage 2, so
// the fetch registers stay live across the stage-2 stores and the wait for
// them (vector loads and stores share one counter) comes a whole stage 1
// after the last store.  In the remainder form (REM: FP64, 17 to 20 columns
// of ZR and rows of YL) a wave holds both the full 16-block and the 4-wide
// remainder of the held operand and takes every fourth block row (stage 1)
// or block column (stage 2) of the other, forming the remainder with the
// four-block 4 x 4 x 4 MFMA on the same fragments.

// Blocks j = 0 .. count-1 of one product on one wave: the moving operand's
// fragment of block j starts at p + j dp (K steps sk apart), the held operand
// is h; MA: the moving operand is A.
template <int KS, bool MA, typename ACC, typename CT, class EP>
__device__ __forceinline__ void ks_blocks(int count, const CT (&h)[KS], const CT *p, int dp, int sk, EP ep) {
  CT x0[KS], x1[KS];
  auto load = [&](int j, CT(&x)[KS]) {
    const CT *q = p + j * dp;
#pragma unroll
    for (int k = 0; k < KS; ++k) x[k] = q[k * sk];
  };
  auto mma = [&](const CT(&x)[KS]) {
    ACC c = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < KS; ++k) c = MA ? mfma16(x[k], h[k], c) : mfma16(h[k], x[k], c);
    return c;
  };
  if (count <= 0) return;
  load(0, x0);
  for (int j = 0;; j += 2) {
    if (j + 1 < count) load(j + 1, x1);
    ep(j, mma(x0));
    if (j + 1 >= count) return;
    if (j + 2 < count) load(j + 2, x0);
    ep(j + 1, mma(x1));
    if (j + 2 >= count) return;
  }
}

// As ks_blocks, for FP64 products with one full 16-block and a remainder of
// at most 4 on the held side: each block of the moving operand feeds a
// 16 x 16 x 4 chain with h and a 4 x 4 x 4 chain with hr (the held
// remainder, laid out for the four-block MFMA), interleaved step by step so
// the short chain's latency hides behind the long one.
template <int KS, bool MA, class EP>
__device__ __forceinline__ void ks_blocks_rem(int count, const double (&h)[KS], const double (&hr)[KS],
                                              const double *p, int dp, int sk, EP ep) {
  double x0[KS], x1[KS];
  auto load = [&](int j, double(&x)[KS]) {
    const double *q = p + j * dp;
#pragma unroll
    for (int k = 0; k < KS; ++k) x[k] = q[k * sk];
  };
  auto mma = [&](const double(&x)[KS], d4_t &c, double &cr) {
    c = d4_t{0, 0, 0, 0};
    cr = 0.0;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      c = MA ? mfma16(x[k], h[k], c) : mfma16(h[k], x[k], c);
      cr = MA ? mfma4(x[k], hr[k], cr) : mfma4(hr[k], x[k], cr);
    }
  };
  if (count <= 0) return;
  d4_t c;
  double cr;
  load(0, x0);
  for (int j = 0;; j += 2) {
    if (j + 1 < count) load(j + 1, x1);
    mma(x0, c, cr);
    ep(j, c, cr);
    if (j + 1 >= count) return;
    if (j + 2 < count) load(j + 2, x0);
    mma(x1, c, cr);
    ep(j + 1, c, cr);
    if (j + 2 >= count) return;
  }
}

template <bool LG, typename CT, int KS, bool REM>
__global__ __launch_bounds__(256) void sandwich_ks_kernel(SandwichArgs a, SwPlan pl) {
  using acc_t = typename std::conditional<std::is_same<CT, double>::value, d4_t, f4_t>::type;
  constexpr bool F64 = std::is_same<CT, double>::value;
  constexpr int K4 = 4 * KS, NSL = sw_ks_slots(KS);
  constexpr int DV = F64 ? 4 : 1;                  // row step between a lane's four results
  constexpr bool ONE_WRAP = 4 * KS - 3 > 3 * DV;   // RI >= 4 KS - 3 exceeds the largest step
  static_assert(!REM || (F64 && !LG), "the remainder form is built for FP64 with the (g, b') column order");
  extern __shared__ double smraw[];
  CT *sm = reinterpret_cast<CT *>(smraw);
  const int RA = a.RA, RI = a.RI, SI = a.SI, SO = a.SO;
  const int GC = pl.GC;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r16 = lane & 15, q4 = lane >> 4;
  const int r0 = F64 ? q4 : 4 * q4;                // first result row of this lane
  const int64_t i0 = (int64_t)blockIdx.x * pl.ipb;
  const int64_t i1 = std::min<int64_t>(a.n, i0 + pl.ipb);
  const int64_t g0 = (int64_t)blockIdx.y * GC;
  const int p = blockIdx.z;
  const int gc = (int)std::min<int64_t>(GC, a.G - g0);
  if (gc <= 0 || i0 >= i1) return;
  const int ldc = pl.ldc, ldz = pl.ldz, ldy = pl.ldy, ldt = pl.ldt;
  const int yzs = K4 * ldz + pl.RA16 * ldy;
  CT *Cs = sm;                    // pl.M1 rows (g, a) x ldc, K = b
  CT *YZ0 = Cs + pl.M1 * ldc;     // [ZR: K4 x ldz | YL: RA16 x ldy], two buffers
  CT *Ts = YZ0 + 2 * yzs;         // K4 rows (a) x ldt, N = stage-2 columns
  const int M1 = gc * RI, M1p = rup(M1, 16);

  // ---- C chunk, zero K padding (as in sandwich_mfma_kernel)
  const CT *cbase = reinterpret_cast<const CT *>(static_cast<const void *>(a.c)) + p * a.cb + g0 * a.cg;
  if (a.cg == 1) {
    stage_lds<8>(gc * RI * K4, Rad3(tid, 256, gc, K4), Cs,
                 [&](const Rad3 &d) {
                   return (d.i1 < SI) ? (double)cbase[d.i0 * a.cg + d.i2 * a.ca + d.i1 * a.cbb] : 0.0;
                 },
                 [&](const Rad3 &d) { return (d.i0 * RI + d.i2) * ldc + d.i1; });
  } else {
    stage_lds<8>(gc * RI * K4, Rad3(tid, 256, K4, RI), Cs,
                 [&](const Rad3 &d) {
                   return (d.i0 < SI) ? (double)cbase[d.i2 * a.cg + d.i1 * a.ca + d.i0 * a.cbb] : 0.0;
                 },
                 [&](const Rad3 &d) { return (d.i2 * RI + d.i1) * ldc + d.i0; });
  }
  for (int e = tid; e < (M1p - M1) * K4; e += 256) {
    const int r = M1 + e / K4, k = e - (e / K4) * K4;
    Cs[r * ldc + k] = (CT)0;
  }
  for (int e = tid; e < (K4 - RI) * ldt; e += 256) Ts[RI * ldt + e] = (CT)0;
  for (int e = tid; e < 2 * yzs; e += 256) YZ0[e] = (CT)0;

  // ---- fetch slots: slot u of this thread is valid entry tid + 256 u of
  // [ZR (SI x SO) | YL (RA x RI)]
  const int nz = SI * SO, nv = nz + RA * RI;
  int s_lds[NSL], s_off[NSL];
  unsigned s_zr = 0;
#pragma unroll
  for (int u = 0; u < NSL; ++u) {
    const int e = tid + 256 * u;
    s_lds[u] = -1;
    s_off[u] = 0;
    if (e < nz) {
      const int b = e / SO, bp = e - b * SO;
      s_lds[u] = b * ldz + bp;
      s_off[u] = (int)(b * a.zrr + bp * a.zrc);
      s_zr |= 1u << u;
    } else if (e < nv) {
      const int f = e - nz, ap = f / RI, k = f - ap * RI;
      s_lds[u] = K4 * ldz + ap * ldy + k;
      s_off[u] = (int)(ap * a.ylr + k * a.ylc);
    }
  }
  const double *zrp = a.zr + p * a.zrb;
  const double *ylp = a.yl + p * a.ylb;
  double pf[NSL];
  auto fetch = [&](int64_t i) {
    const double *zr = zrp + i * a.zri, *yl = ylp + i * a.yli;
#pragma unroll
    for (int u = 0; u < NSL; ++u)
      if (256 * u < nv) pf[u] = (((s_zr >> u) & 1u) ? zr : yl)[s_off[u]];
  };
  auto park = [&](CT *buf) {
#pragma unroll
    for (int u = 0; u < NSL; ++u)
      if (256 * u < nv && s_lds[u] >= 0) buf[s_lds[u]] = (CT)pf[u];
  };
  __syncthreads();  // padding zeroed before the first valid entries land
  fetch(i0);
  park(YZ0);
  if (i0 + 1 < i1) fetch(i0 + 1);
  __syncthreads();

  // ---- stage-1 walk: ZR block column tn1 held, block rows tm1 + j st1
  const int nt1 = pl.SO16 / 16, mt1 = M1p / 16;
  const int tn1 = wave % nt1, st1 = 4 / nt1, tm1 = wave / nt1;
  const int cnt1 = tm1 < mt1 ? (mt1 - tm1 + st1 - 1) / st1 : 0;
  const int bq1 = tn1 * 16 + r16;               // this lane's b'
  const int col1 = LG ? bq1 * GC : bq1;          // T column of (g = 0, b')
  const int gst1 = LG ? 1 : SO;                  // T column step per g
  const int tdelta = gst1 - RI * ldt;            // T offset change of one wrap (a -= RI, g += 1)
  // ---- stage-2 walk: YL block row tm2 held, block columns tn2 + j st2
  const int ncols = LG ? SO * GC : gc * SO;
  const int mt2 = pl.RA16 / 16, nt2 = rup(ncols, 16) / 16;
  const int tm2 = wave % mt2, st2 = 4 / mt2, tn2 = wave / mt2;
  const int cnt2 = tn2 < nt2 ? (nt2 - tn2 + st2 - 1) / st2 : 0;
  const int og = (int)a.og, obb = (int)a.obb, oa = (int)a.oa;  // 32-bit: checked by the plan
  unsigned rows2 = 0;  // results v of this lane inside RA
#pragma unroll
  for (int v = 0; v < 4; ++v)
    if (tm2 * 16 + r0 + v * DV < RA) rows2 |= 1u << v;

  int buf = 0;
  for (int64_t i = i0; i < i1; ++i) {
    const CT *ZRs = YZ0 + buf * yzs;
    const CT *YLs = ZRs + K4 * ldz;

    // ---- stage 1: T(g, a; b') = sum_b C_g(a, b) ZR(b, b')
    if constexpr (REM) {
      // block rows wave + 4 j, each with columns 0..15 (16 x 16) and 16..SO-1 (4 x 4)
      double hb[KS], hr[KS];
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        hb[k] = ZRs[(4 * k + q4) * ldz + r16];
        hr[k] = ZRs[(4 * k + q4) * ldz + 16 + (lane & 3)];
      }
      const int cnt = wave < mt1 ? (mt1 - wave + 3) / 4 : 0;
      const int rrow = 4 * ((lane >> 2) & 3) + q4, rcol = 16 + (lane & 3);  // remainder result of this lane
      auto ep = [&](int j, const d4_t &c, double cr) {
        const int tm = (wave + 4 * j) * 16, row0 = tm + q4;
        const int g = fdiv(row0, pl.fd_ri), aa = row0 - g * RI;
        const int t0 = aa * ldt + r16 + g * SO;
        const bool full = tm + 16 <= M1;  // wave-uniform
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row0 + 4 * v;
          int t;
          if (ONE_WRAP) {
            t = t0 + 4 * v * ldt + ((aa + 4 * v >= RI) ? tdelta : 0);
          } else {
            const int gv = fdiv(row, pl.fd_ri);
            t = (row - gv * RI) * ldt + gv * SO + r16;
          }
          if (full || row < M1) Ts[t] = c[v];
        }
        const int row = tm + rrow;
        if (rcol < SO && row < M1) {
          const int gr = fdiv(row, pl.fd_ri);
          Ts[(row - gr * RI) * ldt + gr * SO + rcol] = cr;
        }
      };
      ks_blocks_rem<KS, true>(cnt, hb, hr, Cs + (wave * 16 + r16) * ldc + q4, 64 * ldc, 4, ep);
    } else {
      CT hb[KS];
      const CT *xb = ZRs + q4 * ldz + bq1;
#pragma unroll
      for (int k = 0; k < KS; ++k) hb[k] = xb[k * 4 * ldz];
      auto ep = [&](int j, const acc_t &c) {
        if (bq1 >= SO) return;
        const int tm = (tm1 + j * st1) * 16, row0 = tm + r0;
        const int g = fdiv(row0, pl.fd_ri), aa = row0 - g * RI;
        const int t0 = aa * ldt + col1 + g * gst1;
        const bool full = tm + 16 <= M1;  // wave-uniform
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row0 + v * DV;
          int t;
          if (ONE_WRAP) {
            t = t0 + v * DV * ldt + ((aa + v * DV >= RI) ? tdelta : 0);
          } else {
            const int gv = fdiv(row, pl.fd_ri);
            t = (row - gv * RI) * ldt + col1 + gv * gst1;
          }
          if (full || row < M1) Ts[t] = c[v];
        }
      };
      ks_blocks<KS, true, acc_t>(cnt1, hb, Cs + (tm1 * 16 + r16) * ldc + q4, st1 * 16 * ldc, 4, ep);
    }
    if (i + 1 < i1) {
      park(YZ0 + (buf ^ 1) * yzs);
      if (i + 2 < i1) fetch(i + 2);
    }
    __syncthreads();

    // ---- stage 2: out(a', col) = sum_a YL(a', a) T(a, col)
    if constexpr (REM) {
      // block columns wave + 4 j, each with rows 0..15 (16 x 16) and 16..RA-1 (4 x 4)
      double ha[KS], har[KS];
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        ha[k] = YLs[r16 * ldy + 4 * k + q4];
        har[k] = YLs[(16 + (lane & 3)) * ldy + 4 * k + q4];
      }
      const int cnt = wave < nt2 ? (nt2 - wave + 3) / 4 : 0;
      double *ob = a.o + p * a.ob + i * a.oi + g0 * a.og + (int64_t)q4 * a.oa;
      const bool rrow_ok = 16 + q4 < RA;  // remainder result row of this lane
      auto ep = [&](int j, const d4_t &c, double cr) {
        const int col = (wave + 4 * j) * 16 + r16;
        const int g = fdiv(col, pl.fd_so), bq = col - g * SO;
        if (col < ncols) {
          double *o = ob + (g * og + bq * obb);
#pragma unroll
          for (int v = 0; v < 4; ++v) o[v * 4 * oa] = c[v];
          if (rrow_ok) o[16 * oa] = cr;
        }
      };
      ks_blocks_rem<KS, false>(cnt, ha, har, Ts + q4 * ldt + wave * 16 + r16, 64, 4 * ldt, ep);
    } else {
      CT ha[KS];
      const CT *xa = YLs + (tm2 * 16 + r16) * ldy + q4;
#pragma unroll
      for (int k = 0; k < KS; ++k) ha[k] = xa[k * 4];
      CT *ob = reinterpret_cast<CT *>(static_cast<void *>(a.o)) + p * a.ob + i * a.oi + g0 * a.og +
               (int64_t)(tm2 * 16 + r0) * a.oa;
      auto ep = [&](int j, const acc_t &c) {
        const int col = (tn2 + j * st2) * 16 + r16;
        int g, bq;
        if (LG) {
          bq = fdiv(col, pl.fd_gc);
          g = col - bq * GC;
        } else {
          g = fdiv(col, pl.fd_so);
          bq = col - g * SO;
        }
        if (col < ncols && g < gc) {
          CT *o = ob + (g * og + bq * obb);
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if ((rows2 >> v) & 1u) o[v * DV * oa] = c[v];
        }
      };
      ks_blocks<KS, false, acc_t>(cnt2, ha, Ts + q4 * ldt + tn2 * 16 + r16, st2 * 16, 4 * ldt, ep);
    }
    __syncthreads();  // Ts and this slice's buffer are rewritten next
    buf ^= 1;
  }
}

namespace {
template <bool LG, typename CT, int KS, bool REM>
void ks_attr(int mx) {
  (void)hipFuncSetAttribute((const void *)sandwich_ks_kernel<LG, CT, KS, REM>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, mx);
}
template <int KS>
void ks_attrs(int mx) {
  ks_attr<true, double, KS, false>(mx);
  ks_attr<false, double, KS, false>(mx);
  ks_attr<true, float, KS, false>(mx);
  ks_attr<false, float, KS, false>(mx);
  ks_attr<false, double, KS, true>(mx);
}
template <bool LG, typename CT, bool REM>
void ks_launch(const SandwichArgs &a, const SwPlan &pl, dim3 grid, size_t lds, hipStream_t s) {
  switch (pl.ks) {
    case 1: sandwich_ks_kernel<LG, CT, 1, REM><<<grid, 256, lds, s>>>(a, pl); break;
    case 2: sandwich_ks_kernel<LG, CT, 2, REM><<<grid, 256, lds, s>>>(a, pl); break;
    case 3: sandwich_ks_kernel<LG, CT, 3, REM><<<grid, 256, lds, s>>>(a, pl); break;
    case 4: sandwich_ks_kernel<LG, CT, 4, REM><<<grid, 256, lds, s>>>(a, pl); break;
    case 5: sandwich_ks_kernel<LG, CT, 5, REM><<<grid, 256, lds, s>>>(a, pl); break;
    case 6: sandwich_ks_kernel<LG, CT, 6, REM><<<grid, 256, lds, s>>>(a, pl); break;
    case 7: sandwich_ks_kernel<LG, CT, 7, REM><<<grid, 256, lds, s>>>(a, pl); break;
    default: sandwich_ks_kernel<LG, CT, 8, REM><<<grid, 256, lds, s>>>(a, pl); break;
  }
}
static_assert(kSwKsMax == 8, "ks_launch instantiates K-step counts 1 to 8");
}  // namespace

bool g_sandwich_ks = true;

const char *sandwich_mfma_name(const SandwichArgs &a, const SwPlan &pl) {
  // [remainder form, FP32, (b', g) order][K steps - 1]
  static const char *const ks_names[2][2][2][kSwKsMax] = {
      {{{"sandwich_ks_kernel<false, double, 1, false>", "sandwich_ks_kernel<false, double, 2, false>",
         "sandwich_ks_kernel<false, double, 3, false>", "sandwich_ks_kernel<false, double, 4, false>",
         "sandwich_ks_kernel<false, double, 5, false>", "sandwich_ks_kernel<false, double, 6, false>",
         "sandwich_ks_kernel<false, double, 7, false>", "sandwich_ks_kernel<false, double, 8, false>"},
        {"sandwich_ks_kernel<true, double, 1, false>", "sandwich_ks_kernel<true, double, 2, false>",
         "sandwich_ks_kernel<true, double, 3, false>", "sandwich_ks_kernel<true, double, 4, false>",
         "sandwich_ks_kernel<true, double, 5, false>", "sandwich_ks_kernel<true, double, 6, false>",
         "sandwich_ks_kernel<true, double, 7, false>", "sandwich_ks_kernel<true, double, 8, false>"}},
       {{"sandwich_ks_kernel<false, float, 1, false>", "sandwich_ks_kernel<false, float, 2, false>",
         "sandwich_ks_kernel<false, float, 3, false>", "sandwich_ks_kernel<false, float, 4, false>",
         "sandwich_ks_kernel<false, float, 5, false>", "sandwich_ks_kernel<false, float, 6, false>",
         "sandwich_ks_kernel<false, float, 7, false>", "sandwich_ks_kernel<false, float, 8, false>"},
        {"sandwich_ks_kernel<true, float, 1, false>", "sandwich_ks_kernel<true, float, 2, false>",
         "sandwich_ks_kernel<true, float, 3, false>", "sandwich_ks_kernel<true, float, 4, false>",
         "sandwich_ks_kernel<true, float, 5, false>", "sandwich_ks_kernel<true, float, 6, false>",
         "sandwich_ks_kernel<true, float, 7, false>", "sandwich_ks_kernel<true, float, 8, false>"}}},
      {{{"sandwich_ks_kernel<false, double, 1, true>", "sandwich_ks_kernel<false, double, 2, true>",
         "sandwich_ks_kernel<false, double, 3, true>", "sandwich_ks_kernel<false, double, 4, true>",
         "sandwich_ks_kernel<false, double, 5, true>", "sandwich_ks_kernel<false, double, 6, true>",
         "sandwich_ks_kernel<false, double, 7, true>", "sandwich_ks_kernel<false, double, 8, true>"},
        {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr}},
       {{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr},
        {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr}}}};
  const int lg = a.og == 1 ? 1 : 0, f = a.prec ? 1 : 0;
  if (pl.slice) return "sandwich_slice_kernel";
  if (g_sandwich_ks && pl.ks >= 1 && pl.ks <= kSwKsMax) {
    const int r = (pl.rem && !f && !lg) ? 1 : 0;
    return ks_names[r][f][lg][pl.ks - 1];
  }
  if (a.prec == 2) return lg ? "sandwich_mfma_kernel<true, __bf16>" : "sandwich_mfma_kernel<false, __bf16>";
  if (a.prec) return lg ? "sandwich_mfma_kernel<true, float>" : "sandwich_mfma_kernel<false, float>";
  return lg ? "sandwich_mfma_kernel<true, double>" : "sandwich_mfma_kernel<false, double>";
}

hipError_t launch_sandwich_mfma(const SandwichArgs &a, const SwPlan &pl, hipStream_t s) {
  const size_t esz = a.prec == 2 ? sizeof(__bf16) : (a.prec ? sizeof(float) : sizeof(double));
  const size_t lds = (size_t)pl.lds_doubles * esz;
  static std::once_flag attr_done;  // set once: the maximum a launch may ask for
  std::call_once(attr_done, [&] {
    const int mx = (int)(kSandwichLdsDoubles * sizeof(double));
    (void)hipFuncSetAttribute((const void *)sandwich_mfma_kernel<true, double>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void *)sandwich_mfma_kernel<false, double>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void *)sandwich_mfma_kernel<true, float>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void *)sandwich_mfma_kernel<false, float>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void *)sandwich_mfma_kernel<true, __bf16>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void *)sandwich_mfma_kernel<false, __bf16>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    ks_attrs<1>(mx);
    ks_attrs<2>(mx);
    ks_attrs<3>(mx);
    ks_attrs<4>(mx);
    ks_attrs<5>(mx);
    ks_attrs<6>(mx);
    ks_attrs<7>(mx);
    ks_attrs<8>(mx);
    (void)hipFuncSetAttribute((const void *)sandwich_slice_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
  });
  if (pl.slice) {
    sandwich_slice_kernel<<<dim3((unsigned)pl.iblocks, (unsigned)pl.gblocks, (unsigned)a.batch), 256, lds, s>>>(a, pl);
    return hipGetLastError();
  }
  dim3 grid((unsigned)pl.iblocks, (unsigned)pl.chunks, (unsigned)a.batch);
  const bool ks = g_sandwich_ks && pl.ks >= 1 && pl.ks <= kSwKsMax;
  if (a.prec == 2) {
    if (a.og == 1) sandwich_mfma_kernel<true, __bf16><<<grid, 256, lds, s>>>(a, pl);
    else sandwich_mfma_kernel<false, __bf16><<<grid, 256, lds, s>>>(a, pl);
  } else if (a.prec) {
    if (ks) {
      if (a.og == 1) ks_launch<true, float, false>(a, pl, grid, lds, s);
      else ks_launch<false, float, false>(a, pl, grid, lds, s);
    } else if (a.og == 1) {
      sandwich_mfma_kernel<true, float><<<grid, 256, lds, s>>>(a, pl);
    } else {
      sandwich_mfma_kernel<false, float><<<grid, 256, lds, s>>>(a, pl);
    }
  } else {
    if (ks) {
      if (a.og == 1) ks_launch<true, double, false>(a, pl, grid, lds, s);
      else if (pl.rem) ks_launch<false, double, true>(a, pl, grid, lds, s);
      else ks_launch<false, double, false>(a, pl, grid, lds, s);
    } else if (a.og == 1) {
      sandwich_mfma_kernel<true, double><<<grid, 256, lds, s>>>(a, pl);
    } else {
      sandwich_mfma_kernel<false, double><<<grid, 256, lds, s>>>(a, pl);
    }
  }
  return hipGetLastError();
}

}  // namespace hatt
