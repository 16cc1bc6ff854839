// Internal declarations shared by the host orchestration and the kernel
// translation units of libhatt.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace hatt {

// Largest column count of one TSQR panel and of the in-LDS Jacobi SVD.
constexpr int kQrMaxCols = 128;
constexpr int kSvdMaxN = 139;
// Largest column count of the block Jacobi SVD over global memory: its
// finishing kernel sorts the singular values in static LDS (20 bytes per
// column, within the 64 KiB of static LDS a kernel may declare).  3072
// columns hold every bond product r_k s_k of the uneven batches (<= 48 x 48).
constexpr int kSvdBigMaxN = 3072;
// Doubles of dynamic LDS a TSQR block may use (of the 160 KiB per CU).
constexpr int kQrLdsDoubles = 19456;

// ---------------------------------------------------------------------------
// Strided matrix view used by the generic kernels: element (r, c) of pair p
// lives at ptr[p * bs + r * rs + c * cs].
struct Mat {
  double *ptr;
  int64_t rs, cs, bs;
};
struct CMat {
  const double *ptr;
  int64_t rs, cs, bs;
};

// ---- sketch / elementwise kernels (k_basic.hip) ---------------------------
hipError_t launch_sketch_fill(uint64_t seed, int core, int64_t count, double scale, double *out,
                              hipStream_t s);

// A(a s0 + b, i, a' s1 + b') = X(a, i, a') Y(b, i, b') for `batch` pairs.
struct PkpArgs {
  const double *x;
  const double *y;
  double *out;
  int64_t r0, r1, s0, s1, n;
  int64_t xs, ys, os;  // batch strides (elements)
  int batch;
};
hipError_t launch_pkp(const PkpArgs &a, hipStream_t s);

// Sandwich: out_{i,g}(a', b') = sum_{a,b} YL_i(a', a) C_g(a, b) ZR_i(b, b')
// for i < n, g < G.  All operands strided; see hatt.cpp for the two uses
// (W_L columns of HPCRL and the PKP-free core update).
struct SandwichArgs {
  const double *yl;  // YL_i(a', a) = yl[p*ylb + i*yli + a'*ylr + a*ylc]
  int64_t ylb, yli, ylr, ylc;
  const double *zr;  // ZR_i(b, b') = zr[p*zrb + i*zri + b*zrr + b'*zrc]
  int64_t zrb, zri, zrr, zrc;
  const double *c;   // C_g(a, b) = c[p*cb + g*cg + a*ca + b*cbb]
  int64_t cb, cg, ca, cbb;
  double *o;         // out = o[p*ob + i*oi + g*og + a'*oa + b'*obb]
  int64_t ob, oi, og, oa, obb;
  int RA, RI, SI, SO;  // YL is RA x RI, C is RI x SI, ZR is SI x SO
  int64_t n, G;
  int batch;
  int prec;            // 1: C and out are FP32 and the products run on the FP32 matrix cores;
                       // 2: C and out are FP32, the products run on the BF16 matrix cores
};
// Overrides of the sandwich kernel choice (the autotuner's candidates):
// no_ks / no_slice rule out the register-blocked / slice-major kernels,
// gc_div divides the chunk of sketch columns per block, valu takes the
// vector-ALU kernels instead of the matrix-core plan (FP64 only).
struct SwForce {
  int no_ks = 0, no_slice = 0, gc_div = 1, valu = 0;
};
hipError_t launch_sandwich(const SandwichArgs &a, hipStream_t s, const SwForce *force = nullptr);
// Whether launch_sandwich has a kernel for these shapes (checked on the host
// before anything is enqueued).
bool sandwich_supported(const SandwichArgs &a);
// Matrix-core variant (k_sandwich.hip): block and LDS plan for a chunk of GC
// sketch columns per workgroup; false when even one column does not fit.
// Division by a launch constant d as a multiply-high: q = (x * m) >> 32 with
// m = ceil(2^32 / d) equals floor(x / d) for 0 <= x < 2^16 and 1 < d <= 4096
// (checked exhaustively); m = 0 marks d = 1.
struct FastDiv {
  uint32_t m;
  int d;
};
inline FastDiv make_fastdiv(int d) {
  FastDiv f;
  f.d = d;
  f.m = (d <= 1) ? 0u : (uint32_t)(((1ull << 32) + (uint64_t)d - 1) / (uint64_t)d);
  return f;
}
constexpr int64_t kSandwichLdsDoubles = 19456;
constexpr int kSwPrefetch = 8;  // register slots per thread for the next slice's YL / ZR
struct SwPlan {
  int GC, chunks;
  int ipb, iblocks;           // mode indices per block, blocks along i
  int pf;                     // 1: next slice's YL / ZR prefetched into registers
  int RI4, SI4, SO16, RA16;   // padded sizes (K edges to 4, M/N edges to 16)
  int ldc, ldz, ldy, ldt, M1; // LDS row strides; padded stage-1 row count
  int64_t lds_doubles;
  FastDiv fd_ri, fd_so, fd_gc; // index decodes of the stage-1 rows and stage-2 columns
  int ks;                     // K steps of both products when they are equal and a
                              // register-blocked instantiation covers them, else 0
  int rem;                    // 1: FP64, b' and a' ranges of 17 to 20 (one full 16-block and a
                              // remainder of at most 4, formed by the 4 x 4 x 4 MFMA)
  int nbuf;                   // YL / ZR slice buffers: 2 (next slice staged during this one) or 1
  int slice;                  // 1: slice-major kernel (one mode index per block, YL / ZR staged
                              // once, the sketch columns streamed in chunks of GC)
  int gpb, gblocks;           // slice-major: sketch columns per block, blocks along g
};
bool sandwich_mfma_plan(const SandwichArgs &a, int64_t budget, SwPlan *pl, const SwForce *force = nullptr);
hipError_t launch_sandwich_mfma(const SandwichArgs &a, const SwPlan &pl, hipStream_t s);
// Name of the compiled kernel launch_sandwich_mfma runs for this plan.
const char *sandwich_mfma_name(const SandwichArgs &a, const SwPlan &pl);
// Name of the compiled kernel launch_sandwich picks for these arguments.
const char *sandwich_kernel_name(const SandwichArgs &a, const SwForce *force = nullptr);

// dst[p * dbs + k] = (float) src[p * sbs + k] for k < count, p < batch.
hipError_t launch_cast_f32(const double *src, int64_t sbs, float *dst, int64_t dbs, int64_t count, int batch,
                           hipStream_t s);
// Reversal of a train of at most kRevMaxCores cores (per core: element
// offsets and r0, n, r1 of the source core; the destination core d-1-k sits
// at doff[k]); dst(b, i, a) = src(a, i, b).
constexpr int kRevMaxCores = 96;
struct RevArgs {
  const double *src;
  double *dst;
  int64_t sstride, dstride;
  int d;
  int64_t soff[kRevMaxCores], doff[kRevMaxCores];
  int r0[kRevMaxCores], n[kRevMaxCores], r1[kRevMaxCores];
};
// max_tiles: the largest ceil(r0/32) ceil(r1/32) n over the cores.
hipError_t launch_tt_reverse(const RevArgs &a, int64_t max_tiles, int batch, hipStream_t s);
// dst[p][k] = src[p][d - k] for the kept-rank arrays ([batch][d+1], int64).
hipError_t launch_rank_reverse(const int64_t *src, int64_t *dst, int d, int batch, hipStream_t s);
// flag[p] (int, device) = 1 when the first `count` doubles of train p
// (pair stride `stride`) are all finite, else 0.
hipError_t launch_finite_check(const double *data, int64_t count, int64_t stride, int batch, int *flag,
                               hipStream_t s);
// dst = (double)src, count elements per pair (pair strides sbs, dbs).
hipError_t launch_cast_f64(const float *src, int64_t sbs, double *dst, int64_t dbs, int64_t count, int batch,
                           hipStream_t s);
// Per pair, scale w[p * bs .. + count) by the power of two that puts its
// largest magnitude in [1, 2).
hipError_t launch_rescale_pow2(float *w, int64_t count, int64_t bs, int batch, hipStream_t s);
// x[p * bs + k] *= alpha[p] (or /= with invert), k < count; alpha on the device.
hipError_t launch_scale_by(double *x, int64_t count, int64_t bs, const double *alpha, int invert, int batch,
                           hipStream_t s);
// Batched strided copy: dst(r, c) = src(r, c) for an M x N block.
hipError_t launch_copy(CMat src, Mat dst, int64_t M, int64_t N, int batch, hipStream_t s);
hipError_t launch_fill(double *p, int64_t count, double v, hipStream_t s);
// Batched strided accumulate: dst(r, c) += src(r, c).
hipError_t launch_add(CMat src, Mat dst, int64_t M, int64_t N, int batch, hipStream_t s);
hipError_t launch_fill_i64(int64_t *p, int64_t count, int64_t v, hipStream_t s);
// dst[p * len + k] = pattern[k] for p < batch, k < len (len <= kMaxRankPattern).
constexpr int kMaxRankPattern = 256;
hipError_t launch_rank_pattern(int64_t *dst, int batch, int len, const int64_t *host_pattern, hipStream_t s);

// ---- GEMM (k_gemm.hip) -----------------------------------------------------
// C = alpha A B + beta C, A is M x K, B is K x N, batched.  With ksplit > 1
// the K range is cut in ksplit chunks whose partial products go to `part`
// (batch * ksplit * M * N doubles) and are summed in a fixed order.
struct GemmArgs {
  CMat A, B;
  Mat C;
  int64_t M, N, K;
  double alpha, beta;
  int batch;
  int ksplit;
  double *part;
  int no_reduce;        // split-K: leave the partial products in `part` (the caller reduces them)
  int prec;             // 0: FP64 matrix cores; 1: FP32 matrix cores; 2: BF16 matrix cores with
                        // FP32 accumulation (split-K partials are FP64 in every case)
  int a_f32, b_f32, c_f32;  // storage of A, B, C is FP32 (pointers reinterpreted), else FP64
  const int *run_flag;  // optional: pair p is computed only when run_flag[p * run_flag_stride] == run_when
  int64_t run_flag_stride;
  int run_when;
  int part_t;           // split-K partials of the launch are written transposed (set by the launcher)
};
hipError_t launch_gemm(const GemmArgs &g, hipStream_t s);
int gemm_pick_ksplit(int64_t M, int64_t N, int64_t K, int batch);
// Sum of the split-K partials of a launch made with no_reduce set, into C.
hipError_t launch_splitk_reduce(const GemmArgs &g, hipStream_t s);
// Output tile (BM x BN) and wave layout (0: 2 x 2, 1: waves along M, 2: along
// N) the launcher uses for an M x N product.
void gemm_tile(int64_t M, int64_t N, int *bm, int *bn, int *wl);
// Name of the kernel launch_gemm runs for g, as a kernel trace lists it.
void gemm_kernel_name(const GemmArgs &g, char *buf, size_t n);
// Layout of the split-K partials: pair p, chunk t at part + (p * ksplit + t) * M * N.

// ---- TSQR (k_qr.hip) -------------------------------------------------------
// Economy Householder QR of an m x n matrix per pair, by a tree of block
// QRs (n <= kQrMaxCols).  k = min(m, n) columns: Q (m x k) is written to `q`
// and R (k x n, upper trapezoidal, diag >= 0) to `r` when r.ptr != nullptr.
constexpr int kQrMaxLevels = 64;
struct QrPlan {
  int64_t m, n, k;
  int levels;
  int64_t rows[kQrMaxLevels];    // rows of the matrix factored at each level
  int64_t blocks[kQrMaxLevels];  // row blocks per level
  int64_t off_v[kQrMaxLevels], off_tau[kQrMaxLevels], off_stack[kQrMaxLevels];
  int64_t off_rtop;
  int64_t ws_doubles;            // per pair
};
bool qr_make_plan(int64_t m, int64_t n, QrPlan *p);
// skip_flag (optional): pairs with skip_flag[p * skip_stride] == 1 are left untouched.
hipError_t launch_tsqr(const QrPlan &p, CMat a, Mat q, Mat r, double *ws, int64_t ws_pair_stride,
                       int batch, hipStream_t s, const int *skip_flag = nullptr, int64_t skip_stride = 0);

// Cholesky factor of a Gram matrix G (n x n, n <= 64, row-major): R (upper,
// diag > 0) and R^{-1}, both n x n row-major with pair stride rbs.  G of pair
// p is the sum over t < ks of g[p * gbs + t * kstride + (i n + j)] (split-K
// partials summed in order; ks = 1 for a plain G).  flag[p * fstride] is set to
// ok when first != 0, else and-ed with ok; ok means every pivot exceeded
// thr_rel times the largest diagonal entry of G.
constexpr int kCholMaxN = 64;
hipError_t launch_chol(const double *g, int64_t gbs, int ks, int64_t kstride, double *r, double *rinv,
                       int64_t rbs, int n, int *flag, int64_t fstride, int first, double thr_rel, int batch,
                       hipStream_t s);
// The same factorisation with the Gram matrix A^T A formed in the kernel from
// A (m x n per pair, any strides; one block per pair streams all of A).
hipError_t launch_gram_chol(CMat A, int64_t m, int n, double *r, double *rinv, int64_t rbs, int *flag,
                            int64_t fstride, int first, double thr_rel, int batch, hipStream_t s);

// ---- Householder QR of short matrices, triangular inverse, Cholesky of
// larger Gram matrices, row sketch (k_hh.hip) --------------------------------
// Householder QR of A (m x n per pair, n <= 128, n <= m <= 384 for n <= 64,
// else <= 256), one workgroup per pair: Q (m x n, explicit, when Q.ptr) and
// R (n x n upper, when R.ptr), diag(R) >= 0.  A may be the same buffer as Q.
// Pairs with skip_flag[p * skip_stride] == 1 are left untouched.
struct HhArgs {
  CMat A;
  Mat Q, R;
  int64_t m, n;
  const int *skip_flag;
  int64_t skip_stride;
};
bool hh_qr_supported(int64_t m, int64_t n);
hipError_t launch_hh_qr(const HhArgs &a, int batch, hipStream_t s);
const char *hh_qr_kernel_name(int64_t m, int64_t n);
// X = R^{-1} of upper triangular R (n x n row-major, n <= 128); flag as in
// launch_chol (cleared by a zero or non-finite diagonal entry; may be null).
// With mask (int [n] per pair, stride mbs): columns whose diagonal entry is
// at most 1e-12 of the column's norm (dep_abs <= 0), or at most dep_abs
// (dep_abs > 0), are replaced by a unit column (scaled to the largest
// diagonal entry) before inversion and marked 1.
hipError_t launch_trinv(const double *r, int64_t rbs, double *x, int64_t xbs, int n, int *flag, int64_t fstride,
                        int first, int *mask, int64_t mbs, double dep_abs, int batch, hipStream_t s);
// Replace the masked columns of A (m x n row-major, pair stride abs) by
// unit-norm random sign vectors.
hipError_t launch_complete_cols(double *a, int64_t m, int n, int64_t abs_, const int *mask, int64_t mbs,
                                uint32_t key, int batch, hipStream_t s);
// Cholesky factor and its inverse of G (n x n row-major, n <= 128, pair
// stride gbs), R and R^{-1} with pair stride rbs; flag as in launch_chol.
hipError_t launch_chol1k(const double *g, int64_t gbs, double *r, double *rinv, int64_t rbs, int n, int *flag,
                         int64_t fstride, int first, double thr_rel, int batch, hipStream_t s);
// B = Omega A (k x n row-major per pair, pair stride bbs): row r of B is the
// signed sum of the rows pi(r), pi(r + k), pi(r + 2k), ... of A (m < 2^31
// rows), pi a pseudo-random permutation and the signs hashed from the row
// index, both keyed by key.
hipError_t launch_sketch_rows(CMat A, int64_t m, int n, int k, double *b, int64_t bbs, uint32_t key, int batch,
                              hipStream_t s);

// Block Gram-Schmidt: mark the columns of a projected panel W (m x cw, cw <=
// 128) whose residual is at most rel of the column's norm before projection
// (||S1_j||^2 + ||W_j||^2), and replace them by random unit vectors.
hipError_t launch_panel_dep(Mat W, CMat S1, int64_t m, int64_t c0, int cw, int *mask, int64_t mbs, double rel,
                            uint32_t key, int batch, hipStream_t s);
// Zero the masked columns of R (rows x cw).
hipError_t launch_zero_masked_cols(Mat R, int rows, int cw, const int *mask, int64_t mbs, int batch, hipStream_t s);

// ---- Jacobi SVD + rank choice (k_svd.hip) ----------------------------------
// For each pair: R (kr x nc, row-major, kr <= nc <= kSvdMaxN) = U S V^T by
// one-sided Jacobi.  Chooses rho (tail rule, cap, and rho <= kmax with
// kmax = min(prev_rank * n_mode, nc) when prev_rank != nullptr, else
// min(kr, nc)), then writes U (kr x ucap, row-major, columns >= rho zero) and
// SVt = S V^T (ucap x nc, rows >= rho zero).  delta2[p] holds
// tol^2 ||A||^2 / (d-1); the first bond computes it from ||R||_F.
struct SvdArgs {
  const double *r;
  int64_t rbs;
  int kr, nc, ucap;
  double *u;
  int64_t ubs;
  double *svt;
  int64_t sbs;
  int batch;
  double *delta2;        // [batch]
  int first_bond;
  double tol2_over_dm1;  // tol^2 / (d-1), 0 for no tolerance
  int64_t cap;           // max_rank, <= 0 for none
  const int64_t *prev_rank;  // device, element p * rank_bs (may be null)
  int64_t n_mode;
  int64_t *rank_out;     // device, element p * rank_bs
  int64_t rank_bs;
  double rel_keep;       // > 0: keep sigma_j > rel_keep * sigma_1 instead (HaTT-2 split)
};
hipError_t launch_svd_trunc(const SvdArgs &a, hipStream_t s);

// Block one-sided Jacobi for matrices too large for one workgroup's LDS:
// A (kr x nc per pair, column-major in `acol`, pair stride acs) is rotated in
// place, one launch per round of disjoint block pairs; flags[2p] collects
// "rotated this sweep", flags[2p+1] is set once a full sweep rotated nothing.
int svd_big_block_width(int kr);
hipError_t launch_svd_big_prepare(const double *r, int64_t rbs, int kr, int nc, double *acol, int64_t acs,
                                  int *flags, int batch, hipStream_t s);
hipError_t launch_svd_big_round(double *acol, int64_t acs, int kr, int nc, int bw, int nb, int t, int *flags,
                                int batch, hipStream_t s);
hipError_t launch_svd_big_sweep_end(int *flags, int batch, hipStream_t s);
// sigma, order, rank choice and U from the rotated columns (S V^T = U^T R is
// the caller's GEMM).
hipError_t launch_svd_big_finish(const SvdArgs &a, const double *acol, int64_t acs, hipStream_t s);

// Frobenius norm of a batch of contiguous blocks: out[p] = ||x_p||.
hipError_t launch_block_norm(const double *x, int64_t count, int64_t bs, double *out, int batch,
                             hipStream_t s);

// Width predictor (k_rankpred.hip): 21 features per bond, a 21-128-128-2
// tanh MLP in FP32.
constexpr int kRpIn = 21, kRpH = 128, kRpOut = 2;
constexpr int kRpTheta = kRpH * kRpIn + kRpH + kRpH * kRpH + kRpH + kRpOut * kRpH + kRpOut;  // 19586
constexpr int kRpStats = 2 * kRpIn + 2 * kRpOut;                                            // 46
constexpr int kRpRowsPerBlock = 64;  // rows per gradient block
constexpr int kRpMaxBonds = 32;      // bonds per feature launch
constexpr int kRpMaxRank = 2048;     // largest bond rank the statistics kernel sorts
struct RpFeatArgs {
  const double *cx[kRpMaxBonds], *cy[kRpMaxBonds];  // core k of x and y (train 0)
  int rxp[kRpMaxBonds], rxn[kRpMaxBonds], ryp[kRpMaxBonds], ryn[kRpMaxBonds], n[kRpMaxBonds];
  int k0;      // 1-based bond index of the first bond of this launch
  int d;       // order of the pair
  float *out;  // feature row of bond k0
};
struct RpAdam {
  float *theta, *m, *v;  // theta == nullptr: no update
  float lr, b1, b2, eps, c1, c2;
};
hipError_t launch_rp_features(const RpFeatArgs &a, int bonds, hipStream_t s);
hipError_t launch_rp_forward(const float *theta, const float *stats, const float *feat, int64_t rows, float *pred,
                             hipStream_t s);
hipError_t launch_rp_grad(const float *theta, const float *stats, const float *feat, const float *label,
                          const int32_t *idx, int64_t batch, float *part, float *loss_part, float *grad,
                          float *loss, const RpAdam &ad, hipStream_t s);
hipError_t launch_rp_stats(const float *feat, const float *label, int64_t rows, float *stats, hipStream_t s);

}  // namespace hatt
