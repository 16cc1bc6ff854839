/*
 * hatt.h -- C ABI of the MI355X (gfx950) library for recompressing the
 * Hadamard product of two tensor trains without forming its partial
 * Kronecker product (PKP) cores ("HaTT", Sun, Huang, Xiao and Yang).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All floating point data is IEEE double, on the device, owned by the
 *   caller.  The library never allocates device memory: scratch space is a
 *   caller-provided workspace whose size the *_plan calls report.
 * - A TT view (hatt_tt) describes `batch` tensor trains of identical shape
 *   stored back to back.  Core k of train b starts at element
 *       data + b * batch_stride + sum_{j<k} rank[j] * n[j] * rank[j+1]
 *   and is row-major [rank[k]][n[k]][rank[k+1]] (last index fastest, the
 *   multi-index convention of Sec. 2.1; H(T) and V(T) are then plain
 *   row-major reshapes).  rank[0] = rank[d] = 1.
 * - Outputs of recompression/rounding are written at "capacity" shape: core
 *   k occupies cap[k] * n[k] * cap[k+1] elements (cap from the plan call),
 *   and when a bond's kept rank rho[k] is smaller than cap[k] the extra
 *   rows/columns are zero.  The kept ranks are written, per train, to a
 *   device int64 array out_rank[batch][d+1].  Zero padding does not change
 *   the represented tensor, so a caller may use the padded cores directly or
 *   slice core k to [rho[k]][n[k]][rho[k+1]].
 * - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *   enqueues work on it (no host synchronisation) unless stated otherwise.
 * - Arguments are validated before anything is enqueued; on an error nothing
 *   is launched and hatt_last_error() returns a message (thread-local).
 *   Device/launch failures return HATT_EDEVICE.  No C++ exception crosses
 *   the ABI.  Calls are re-entrant when they use distinct workspaces.
 */
#ifndef HATT_H_
#define HATT_H_

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define HATT_API __attribute__((visibility("default")))
#else
#define HATT_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HATT_OK = 0,
  HATT_EINVAL = -1,      /* a NULL pointer, a non-positive size or an option out of range */
  HATT_ESHAPE = -2,      /* inconsistent mode sizes or ranks (rank[0] or rank[d] != 1, ...) */
  HATT_EWORKSPACE = -3,  /* workspace smaller than the plan call reported */
  HATT_EDEVICE = -4,     /* a HIP call or kernel launch failed */
  HATT_ENOTCONV = -5,    /* the tolerance-driven width growth did not converge (hatt_recompress_adaptive) */
  HATT_ENONFINITE = -6,  /* non-finite input (hatt_recompress_adaptive, hatt_rankpred_widths) */
  HATT_EUNSUPPORTED = -7 /* a shape the library does not handle (see message) */
} hatt_status;

typedef struct {
  int32_t d;              /* order, >= 1 */
  int32_t batch;          /* number of trains of identical shape, >= 1 */
  const int64_t *n;       /* host [d]: mode sizes, >= 1 */
  const int64_t *rank;    /* host [d+1]: bond ranks, rank[0] = rank[d] = 1 */
  double *data;           /* device: cores (layout above) */
  int64_t batch_stride;   /* elements between trains; 0 means packed */
} hatt_tt;

typedef struct {
  int32_t variant;        /* 1: HaTT-1, sketch split W = W I (eq. HPCRL--1);
                             2: HaTT-2, truncated SVD split (eq. HPCRL--2) */
  double ep;              /* HaTT-2: keep rank-1 terms with sigma > ep * ||W||_2 */
  int64_t ell;            /* requested sketch width l_k for every interior bond */
  const int64_t *ell_bond;/* optional host [d+1] per-bond request (overrides ell) */
  int64_t max_rank;       /* truncation cap on every bond after the sweep; <= 0: none */
  double tol;             /* relative Frobenius tolerance of that truncation; <= 0: none */
  uint64_t seed;          /* key of the Philox4x32-10 sketch (used when no sketch is passed) */
  int32_t precision;      /* 0: FP64 throughout; 1: FP32 range finding -- the HPCRL sketches
                             W^{(k)} (W_L build and W_L W_R^T, Alg. 3) run on the FP32
                             matrix cores with FP32 accumulation and storage; 2: BF16
                             range finding -- the same products with their operands
                             rounded to BF16 on the BF16 matrix cores (FP32 accumulation,
                             FP32 storage).  In both the sweep (Alg. 4: the frame
                             X^{(k)} W^{(k)} with W^{(k)} widened to FP64, its QR, the
                             projection Q^T X, the core update) and the truncation run in
                             FP64, so every frame spans a subspace of range(X^{(k)}) to
                             FP64 accuracy; what the sketch's rounding costs is range
                             capture (HaTT-1 only) */
  const int64_t *max_rank_bond; /* optional host [d+1]: entry k caps the kept rank of bond k
                             (entries <= 0: max_rank applies there); not for the uneven batch */
} hatt_opts;

/*
 * hatt_plan -- sketch widths and workspace size of hatt_recompress.
 * The requested widths are clamped (Sec. 2.2 rank bound and the economy-QR
 * shape condition of Sec. 4): l_0 = l_d = 1; l_k <= r_k s_k;
 * l_k <= l_{k-1} n_k (left to right); l_{k-1} <= n_k l_k (right to left).
 * ell_out: host [d+1] clamped widths, which are also the output capacities.
 * ws_bytes: device workspace bytes for a call with x->batch trains.
 * out_elems: elements of one output train at capacity shape.
 */
HATT_API hatt_status hatt_plan(const hatt_tt *x, const hatt_tt *y, const hatt_opts *opts,
                      int64_t *ell_out, size_t *ws_bytes, int64_t *out_elems);

/*
 * hatt_recompress -- Alg. 4 (HaTT): recompress x (.) y (elementwise product,
 * Sec. 2.2) for every train of the batch, then optionally truncate the
 * result to max_rank and/or tol with Alg. 1's truncation loop run from the
 * right: every output core but the last is the Q of a QR, so the result is
 * already left-orthogonal and Alg. 1's orthogonalisation pass is skipped
 * (the bond rule is tt_round's, with ||z|| read off the last core).
 *   - Sketch: `sketch` may hold an explicit Gaussian TT with ranks
 *     ell_out of hatt_plan (batch 1: shared by all trains, or batch equal to
 *     x->batch: one per train); if NULL the library draws the random
 *     Gaussian TT of Def. 2.1 from Philox4x32-10 keyed by opts->seed
 *     (the same sketch for every train of the batch).
 *   - HPCRL (Alg. 3) builds the sketches W^{(k)} right to left from the cores
 *     of x and y (eqs. 3.3, WLWR, LISRmatrix); the left-to-right sweep
 *     (eqs. updatcores1/2, M*core0) never forms a PKP core.
 *   - out: device, x->batch trains at capacity shape (ell_out), batch stride
 *     out_stride elements (0 = packed, i.e. out_elems).  Without truncation
 *     the output cores 1..d-1 are left-orthogonal (V(X_k)^T V(X_k) = I).
 *   - out_rank: device int64 [batch][d+1], the kept ranks.
 * x and y must have the same d, batch and mode sizes.
 */
HATT_API hatt_status hatt_recompress(const hatt_tt *x, const hatt_tt *y, const hatt_tt *sketch,
                            const hatt_opts *opts, double *out, int64_t out_stride,
                            int64_t *out_rank, void *ws, size_t ws_bytes, void *stream);

/*
 * hatt_recompress_noalloc -- hatt_recompress for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same computation and
 * arguments without the workspace, which is a library-owned static device
 * array of 128 MiB (one per device, held until the process ends; nothing is
 * allocated by the call).  A problem whose hatt_plan workspace exceeds
 * 128 MiB returns HATT_EWORKSPACE before anything is enqueued.  Every call on
 * a device uses that device's one array: calls that overlap on one device
 * (other streams, other host threads) race and must be serialised by the
 * caller; the array keeps the last call's contents, which no call relies on.
 */
HATT_API hatt_status hatt_recompress_noalloc(const hatt_tt *x, const hatt_tt *y, const hatt_tt *sketch,
                                             const hatt_opts *opts, double *out, int64_t out_stride,
                                             int64_t *out_rank, void *stream);

/*
 * Uneven batches: npairs independent recompressions x[p] (.) y[p] whose
 * shapes (order, mode sizes, ranks, batch) differ from pair to pair; each
 * pair is the hatt_recompress problem above.  opts applies to every pair
 * (opts->ell_bond must be NULL): widths are clamped per pair; opts->ell <= 0
 * asks for l_k = max(r_k, s_k) + 8 per bond; pair p draws its Philox sketch
 * with key opts->seed + p.  Outputs go to one flat device buffer: pair p's
 * trains at element offset out_offset[p] (packed, capacity shape as
 * hatt_plan would report), its kept ranks ([batch_p][d_p + 1] int64) at
 * element offset rank_offset[p] of out_rank.
 * hatt_batched_plan: out_offset and rank_offset (host [npairs + 1], the last
 * entry is the total), ell_out (host, may be NULL: the clamped widths of
 * every pair, d_p + 1 entries per pair, concatenated in pair order) and
 * ws_bytes.  The pairs are enqueued, largest first, on up to 32
 * library-owned streams forked from `stream` and joined back to it (so the
 * call composes with stream order and graph capture); concurrent pairs use
 * separate workspace slots.  How many streams run concurrently is bounded by
 * the process's hardware queues (HIP's GPU_MAX_HW_QUEUES).  Each stream's
 * pairs are enqueued by a short-lived host thread of its own (on the caller's
 * device; one thread does it all under graph capture, with the profiler on
 * or while the autotuner records), so a pair with many launches does not
 * hold back the other streams.  No host synchronisation.  Errors of any pair are reported before anything is
 * enqueued.  While `stream` is being captured into a HIP graph at most 12
 * pairs are accepted (HATT_EUNSUPPORTED above that: a capture of 512 pairs,
 * some 10^5 kernel nodes, ended the host process).  Concurrent calls from
 * several host threads are serialised inside the library (the forked
 * streams are shared per device).
 */
HATT_API hatt_status hatt_batched_plan(int32_t npairs, const hatt_tt *x, const hatt_tt *y,
                                       const hatt_opts *opts, int64_t *out_offset,
                                       int64_t *rank_offset, int64_t *ell_out, size_t *ws_bytes);
HATT_API hatt_status hatt_recompress_batched(int32_t npairs, const hatt_tt *x, const hatt_tt *y,
                                             const hatt_opts *opts, double *out, int64_t *out_rank,
                                             void *ws, size_t ws_bytes, void *stream);

/*
 * Tolerance-driven recompression.  The paper fixes target ranks and leaves
 * tolerance control open (Sec. 6); it suggests enlarging l when a sketch's
 * smallest singular value is not small enough (Sec. 5.1.1).  Rule:
 *   start l_k = max(r_k, s_k) + p (clamped as in hatt_plan); run HaTT with
 *   the Philox sketch keyed by seed + attempt, then TT-Rounding at
 *   tol sqrt(3) / 2; accept when every bond keeps rho_k <= l_k - p or l_k is
 *   at its largest feasible value, and the sketch captured the product's
 *   range to within tol / 2: the untruncated HaTT result X is an orthogonal
 *   projection of z = x (.) y, so ||z - X||^2 = ||z||^2 - ||X||^2 (||z|| by
 *   hatt_hadamard_norm2, once per call), and the truncation error is
 *   orthogonal to z - X, so the result is within tol of z (the check cannot
 *   resolve ||z - X||^2 below 256 eps ||z||^2).  Else l_k = min(cap_k,
 *   ceil(1.5 l_k) + p) on each bond failing the slack test (for any train of
 *   the batch), or on every bond below its cap when only the capture test
 *   failed, and retry.  With FP32 or BF16 range finding (opts->precision),
 *   a capture failure with every bond at its cap (where the sketch spans the
 *   product's range up to its own rounding) switches the following attempts
 *   to FP64 range finding instead; the plan's workspace covers both.
 * Widths never grow beyond 3072 (the truncation's SVD limit): a bond that
 * would need more returns HATT_ENOTCONV.
 * hatt_adaptive_plan: cap_out (host [d+1]) = largest widths the growth may
 * reach (the feasible widths, clamped to 3072), ws_bytes = workspace for any
 * attempt, out_elems = elements of one output train at those widths (the
 * per-train slot size).
 * hatt_recompress_adaptive: first checks that x and y hold only finite
 * values (HATT_ENONFINITE otherwise, nothing written but out_rank), then
 * synchronises `stream` once per attempt (the decision needs the kept ranks
 * on the host).  The result of the last
 * attempt is written per train at the widths returned in ell_out (host
 * [d+1]; packed inside each train's slot of out_stride elements, 0 = the
 * planned slot size), kept ranks in out_rank (device [batch][d+1]), the
 * number of attempts in *attempts_out.  Returns HATT_ENOTCONV (with the last
 * attempt's result in place) if max_attempts did not suffice.
 */
typedef struct {
  double tol;             /* relative Frobenius tolerance, > 0 */
  uint64_t seed;          /* attempt a uses the sketch keyed by seed + a */
  int32_t oversample;     /* p; <= 0 means 8 */
  int32_t max_attempts;   /* <= 0 means 8 */
  int32_t variant;        /* 1 or 2 as in hatt_opts */
  double ep;              /* HaTT-2 threshold */
  const int64_t *ell_init;/* optional host [d+1]: start widths instead of max(r_k, s_k) + p
                             (e.g. hatt_rankpred_widths); clamped like any request */
  int32_t precision;      /* as in hatt_opts: 0 FP64, 1 FP32, 2 BF16 range finding */
} hatt_adapt_opts;

HATT_API hatt_status hatt_adaptive_plan(const hatt_tt *x, const hatt_tt *y, const hatt_adapt_opts *opts,
                                        int64_t *cap_out, size_t *ws_bytes, int64_t *out_elems);
HATT_API hatt_status hatt_recompress_adaptive(const hatt_tt *x, const hatt_tt *y, const hatt_adapt_opts *opts,
                                              double *out, int64_t out_stride, int64_t *out_rank,
                                              int64_t *ell_out, int32_t *attempts_out, void *ws,
                                              size_t ws_bytes, void *stream);

/*
 * Tolerance mode over an uneven batch (npairs pairs of any shapes, two
 * factors each): pair p follows the rule of hatt_recompress_adaptive with
 * seed opts->seed + p and its own widths, so its widths, attempts and result
 * are those of the single-pair call with that seed.  Attempts run in rounds:
 * round a runs attempt a of every pair not yet accepted, concurrently on the
 * library streams (forked from `stream` and joined back), then synchronises
 * `stream` once and takes every pair's decision from its kept ranks and
 * ||X||.  Before the first round the same streams check x and y for
 * non-finite values (HATT_ENONFINITE, naming the pair) and form ||x (.) y||
 * of every train.  opts->ell_init, if not NULL, holds the start widths of
 * every pair (d_p + 1 entries per pair, concatenated in pair order).
 * hatt_batched_adaptive_plan: out_offset / rank_offset (host [npairs + 1]):
 * pair p's trains at element offset out_offset[p] of `out`, one slot per
 * train at the widths in cap_out (host, may be NULL; d_p + 1 entries per
 * pair, concatenated: the widths the growth may reach), its kept ranks
 * ([batch_p][d_p + 1]) at rank_offset[p] of out_rank.  ws_min: the smallest
 * workspace that runs every round (one pair at a time when a round's pairs
 * do not fit side by side); ws_full: enough for the largest pairs to run on
 * all streams at once.  Between the two, each round runs as many pairs side
 * by side as the workspace holds.
 * hatt_recompress_batched_adaptive: writes pair p's result packed inside its
 * slots at the widths of its last attempt, those widths in ell_out (host,
 * d_p + 1 per pair, concatenated) and its attempt count in attempts_out
 * (host [npairs]).  A pair that cannot converge (a failing bond at its
 * limit, or max_attempts used) keeps its last result; the other pairs
 * finish, and the call returns HATT_ENOTCONV naming the first such pair.
 * Not capturable (HATT_EUNSUPPORTED under HIP graph capture); concurrent
 * calls are serialised with hatt_recompress_batched.
 */
HATT_API hatt_status hatt_batched_adaptive_plan(int32_t npairs, const hatt_tt *x, const hatt_tt *y,
                                                const hatt_adapt_opts *opts, int64_t *out_offset,
                                                int64_t *rank_offset, int64_t *cap_out, size_t *ws_min,
                                                size_t *ws_full);
HATT_API hatt_status hatt_recompress_batched_adaptive(int32_t npairs, const hatt_tt *x, const hatt_tt *y,
                                                      const hatt_adapt_opts *opts, double *out,
                                                      int64_t *out_rank, int64_t *ell_out,
                                                      int32_t *attempts_out, void *ws, size_t ws_bytes,
                                                      void *stream);

/*
 * Three factors: recompress x (.) y (.) w in one pass, without forming the
 * three-way PKP cores (rank r_k s_k t_k).  The identity that turns the PKP
 * products into two-sided products (eq. kronecker_product_times_vec, used by
 * eqs. WLWR and M*core0) is taken over three factors, so HPCRL (Alg. 3,
 * HaTT-1 split) and the sweep (Alg. 4) apply X_k(i), Y_k(i) and W_k(i) as a
 * three-mode product; the result equals RandOrth (Alg. 2) on the explicit
 * three-way PKP train with the same sketch.  The paper forms its cubic
 * nonlinearity as successive products (Sec. 5, Example 4); this form skips
 * the intermediate recompression.  Output, ranks and truncation are those of
 * hatt_recompress (three-way PKP index order: x's index slowest, w's fastest).
 * Limits: one triple per call (every batch 1), opts->variant 1,
 * opts->precision 0 (HATT_EUNSUPPORTED otherwise).  Widths are clamped with
 * r_k s_k t_k in place of r_k s_k.  x, y and w must have the same d and mode
 * sizes.
 * hatt_plan3 / hatt_recompress3: as hatt_plan / hatt_recompress.
 * hatt_adaptive_plan3 / hatt_recompress3_adaptive: the tolerance-driven rule
 * above with start widths max(r_k, s_k, t_k) + p but the slack test alone
 * (truncation at tol, no capture test); the finiteness check covers all three
 * factors.
 */
HATT_API hatt_status hatt_plan3(const hatt_tt *x, const hatt_tt *y, const hatt_tt *w, const hatt_opts *opts,
                                int64_t *ell_out, size_t *ws_bytes, int64_t *out_elems);
HATT_API hatt_status hatt_recompress3(const hatt_tt *x, const hatt_tt *y, const hatt_tt *w, const hatt_tt *sketch,
                                      const hatt_opts *opts, double *out, int64_t out_stride, int64_t *out_rank,
                                      void *ws, size_t ws_bytes, void *stream);
HATT_API hatt_status hatt_adaptive_plan3(const hatt_tt *x, const hatt_tt *y, const hatt_tt *w,
                                         const hatt_adapt_opts *opts, int64_t *cap_out, size_t *ws_bytes,
                                         int64_t *out_elems);
HATT_API hatt_status hatt_recompress3_adaptive(const hatt_tt *x, const hatt_tt *y, const hatt_tt *w,
                                               const hatt_adapt_opts *opts, double *out, int64_t out_stride,
                                               int64_t *out_rank, int64_t *ell_out, int32_t *attempts_out,
                                               void *ws, size_t ws_bytes, void *stream);

/*
 * tt_hadamard_explicit -- the PKP cores of x (.) y (Sec. 2.2):
 * A_k(a s + b, i, a' s' + b') = X_k(a, i, a') Y_k(b, i, b'), ranks r_k s_k.
 * out: device, batch trains with ranks r_k s_k, stride out_stride
 * (0 = packed).  HBM-write bound; no workspace.
 */
HATT_API hatt_status tt_hadamard_explicit(const hatt_tt *x, const hatt_tt *y, double *out,
                                 int64_t out_stride, void *stream);

/*
 * tt_randorth_plan / tt_randorth -- RandOrth (Alg. 2) of an explicit TT a:
 * the sketch W^{(k)} = (A_{k+1..d} contracted with R_{k+1..d}) right to
 * left (eq. rtlpc), then for k = 1..d-1: Q = QR(V(B_k) W^{(k)}) becomes
 * V(B_k), M = Q^T V(B_k) (the core before the QR), H(B_{k+1}) = M H(A_{k+1}); optionally
 * the rank-l result (left-orthogonal) is truncated to max_rank and/or tol as
 * in hatt_recompress.  On the
 * PKP cores of x (.) y (tt_hadamard_explicit) it is the paper's RandOrth
 * comparator, and with the same sketch it represents the same tensor as
 * hatt_recompress (HaTT reorganises exactly these products).  Widths are
 * clamped as in hatt_plan with the ranks of a in place of r_k s_k; the
 * sketch is `sketch` (ranks ell_out, batch 1 or a->batch) or, if NULL, the
 * Philox sketch keyed by seed (the same one hatt_recompress draws for that
 * seed and those widths).  Output at
 * capacity shape ell_out, kept ranks in out_rank (device [batch][d+1]).
 * tt_randorth_plan reports the workspace for a call with truncation.
 */
HATT_API hatt_status tt_randorth_plan(const hatt_tt *a, int64_t ell, const int64_t *ell_bond, int64_t *ell_out,
                                      size_t *ws_bytes, int64_t *out_elems);
HATT_API hatt_status tt_randorth(const hatt_tt *a, const hatt_tt *sketch, int64_t ell, const int64_t *ell_bond,
                                 uint64_t seed, int64_t max_rank, double tol, double *out, int64_t out_stride,
                                 int64_t *out_rank, void *ws, size_t ws_bytes, void *stream);

/*
 * tt_round_plan / tt_round -- TT-Rounding (Alg. 1): right-to-left QR
 * orthogonalisation, then left-to-right economy QR + SVD truncation.
 * Bond rule: delta = tol ||a||_F / sqrt(d-1); keep the smallest rho >= 1
 * whose discarded tail sum_{j>rho} sigma_j^2 <= delta^2 (all of them when
 * tol <= 0), then rho = min(rho, max_rank) when max_rank > 0.
 * Output at capacity shape cap (written by tt_round_plan to cap_out
 * [d+1]: the input ranks, clamped to the economy-QR shapes), zero padded,
 * kept ranks in out_rank (device int64 [batch][d+1]).
 */
HATT_API hatt_status tt_round_plan(const hatt_tt *a, int64_t *cap_out, size_t *ws_bytes, int64_t *out_elems);
HATT_API hatt_status tt_round(const hatt_tt *a, int64_t max_rank, double tol, double *out,
                     int64_t out_stride, int64_t *out_rank, void *ws, size_t ws_bytes,
                     void *stream);

/*
 * tt_norm -- Frobenius norm (Sec. 2.1) of every train, computed as
 * ||B_1||_F after right-to-left QR orthogonalisation (the identity used by
 * Alg. 1).  out: device double [batch].  Workspace from tt_norm_plan.
 */
HATT_API hatt_status tt_norm_plan(const hatt_tt *a, size_t *ws_bytes);
HATT_API hatt_status tt_norm(const hatt_tt *a, double *out, void *ws, size_t ws_bytes, void *stream);

/*
 * tt_check_finite -- flag[b] (device int32 [batch]) = 1 when every entry of
 * train b's cores is finite, else 0; enqueue only.  The other enqueue-only
 * entry points do not inspect their inputs: a non-finite input yields
 * non-finite output and meaningless kept ranks, so a caller that cannot
 * trust its data runs this first (the tolerance mode does).
 */
HATT_API hatt_status tt_check_finite(const hatt_tt *a, int32_t *flag, void *stream);

/*
 * hatt_hadamard_norm2 -- ||x (.) y||_F^2 of every train (device out [batch]),
 * without the PKP cores: the Gram recursion of the TT inner product (Sec.
 * 2.1), G_0 = 1, G_k = sum_i Z_k(i)^T G_{k-1} Z_k(i) with Z_k(i) =
 * X_k(i) kron Y_k(i) (Sec. 2.2), each step as two sandwich contractions and
 * a fixed-order sum over i, ||z||^2 = G_d.  x and y must have the same d,
 * mode sizes and batch.  Work on the stream, no synchronisation;
 * hatt_hadamard_norm2_plan gives the workspace (r_k s_k r_{k+1} s_{k+1} n_k
 * doubles twice, plus one Gram matrix).
 */
HATT_API hatt_status hatt_hadamard_norm2_plan(const hatt_tt *x, const hatt_tt *y, size_t *ws_bytes);
HATT_API hatt_status hatt_hadamard_norm2(const hatt_tt *x, const hatt_tt *y, double *out, void *ws,
                                         size_t ws_bytes, void *stream);

/*
 * tt_scale -- multiply (invert = 0) or divide (invert = 1) train b of `a` by
 * alpha[b] (device double [batch], e.g. the output of tt_norm), through its
 * first core, in place; enqueue only.  Lets an iteration that repeats
 * Hadamard products (the power iteration of Sec. 5, Example 3) keep its
 * iterate normalised without a host round trip.
 */
HATT_API hatt_status tt_scale(const hatt_tt *a, const double *alpha, int32_t invert, void *stream);

/*
 * hatt_sketch_fill -- materialise the seeded random Gaussian TT (Def. 2.1)
 * with ranks ell[0..d] (ell[0] = ell[d] = 1) and mode sizes n[0..d-1]:
 * entries N(0, 1/(ell_{k-1} n_k ell_k)) from Philox4x32-10 (key = seed,
 * counter = (pair index low, pair index high, k, 0x5A7C), two 53-bit
 * uniforms per pair of entries, Box-Muller).  out: device, packed cores.
 */
HATT_API hatt_status hatt_sketch_fill(uint64_t seed, int32_t d, const int64_t *n, const int64_t *ell,
                             double *out, void *stream);

/*
 * QR method used by every entry point for the QR factorisations of the
 * HaTT sweep (Alg. 4) and of TT-Rounding (Alg. 1), process-wide:
 *   0 (default): CholeskyQR2 on the matrix cores for matrices of at most 64
 *      columns (and at least as many rows), Householder TSQR otherwise; a
 *      pair whose Gram matrix is too ill-conditioned for CholeskyQR2
 *      (condition number beyond about 1e6, rank deficiency included) is
 *      recomputed by Householder TSQR inside the same call;
 *   1: Householder TSQR (and panelled block Gram-Schmidt above 128 columns)
 *      everywhere.
 * Workspace sizes depend on the method: plan again after changing it.  Not
 * thread-safe with concurrent plan or compute calls.  HATT_EINVAL for other
 * values.
 */
HATT_API hatt_status hatt_set_qr_method(int32_t method);

/*
 * Autotuner (shape buckets to kernel choices; not in the paper).  Mode 0
 * (default): the fixed tile and kernel rules.  Mode 1 (record): the first
 * launch of each shape bucket times its candidates on the caller's stream
 * (a host wait per candidate, so a recording call is slow and synchronises)
 * and keeps the fastest for that bucket; later launches reuse it.  Mode 2
 * (use): recorded choices only, no timing; unseen buckets take the fixed
 * rules.  Buckets: a GEMM by (M, N, K, batch, compute type, operand
 * layouts), its candidate K splits 1, 2, 4 .. 64; a sandwich contraction by
 * its shapes, output layout and type, its candidates the matrix-core plan
 * with and without the register-blocked and slice-major kernels, smaller
 * sketch-column chunks, and (FP64) the vector-ALU kernels.  Choices change
 * only the summation order of split-K products (results agree to rounding).
 * Nothing is timed while the stream is captured into a graph, nor a GEMM
 * that accumulates into its output.  The table is per process, shared by all
 * devices and threads (it is guarded by a mutex).
 * hatt_tune_mode: sets the mode (HATT_EINVAL outside 0..2).
 * hatt_tune_clear: empties the table.
 * hatt_tune_table: writes the table as text, one bucket per line
 * ("<bucket> -> <choice>  <us> us (fixed rules <us> us)"), NUL-terminated and
 * cut to cap bytes, into buf (may be NULL); returns the bytes the whole table
 * needs, terminator included.
 */
HATT_API hatt_status hatt_tune_mode(int32_t mode);
HATT_API hatt_status hatt_tune_clear(void);
HATT_API int64_t hatt_tune_table(char *buf, int64_t cap);

/*
 * Instrumentation (not thread-safe; for benchmarks).  Between
 * hatt_profile_start() and hatt_profile_stop() every kernel launch the
 * library enqueues is bracketed by two HIP events on the launching stream
 * and attributed to one of HATT_PROFILE_CLASSES kernel classes (names from
 * hatt_profile_class_name).  hatt_profile_stop() waits for those events and
 * writes, per class, the summed event-to-event milliseconds to ms_out and
 * the number of launcher calls to calls_out (both host arrays of length
 * HATT_PROFILE_CLASSES).  A launcher call may enqueue more than one kernel
 * (a split-K GEMM adds its reduction, a QR one kernel per tree level).
 */
#define HATT_PROFILE_CLASSES 8
HATT_API hatt_status hatt_profile_start(void);
HATT_API hatt_status hatt_profile_stop(double *ms_out, int64_t *calls_out);
HATT_API const char *hatt_profile_class_name(int32_t cls);
/* Text table written by the last hatt_profile_stop(): one line per launch
 * site ("class: label", GEMMs labelled with M x N x K and split), with its
 * summed milliseconds and calls, largest first.  Valid until the next stop. */
HATT_API const char *hatt_profile_report(void);

/*
 * Learned start widths (a per-bond predictor; not part of the paper, which
 * picks l by hand and only suggests enlarging a sketch that is too narrow,
 * Sec. 5.1.1).  For every bond k = 1..d-1 of a pair (x, y) a small network
 * predicts the rank the truncation at the requested tolerance keeps (rho_k)
 * and the narrowest width the adaptive rule of hatt_recompress_adaptive
 * accepts (min(cap_k, rho_k + p)); hatt_recompress_adaptive started at
 * those widths (ell_init) then falls back to growing them when the
 * prediction was short, and its acceptance rule judges the result.
 *
 * Rows: the bonds of pair 0 (k = 1..d_0-1), then those of pair 1, ...
 * (sum over pairs of d_p - 1 rows); statistics come from train 0 of a pair.
 * Feature row (FP32, 21 values): ln r_k(x), ln r_k(y), ln n_k, k/d, ln d,
 * then the quantiles at q = j/7 (j = 0..7, linear interpolation between
 * order statistics) of ln max(c_a, 1e-300) over the r_k columns a of V(x_k)
 * (c_a = squared column norm, the diagonal of V(x_k)^T V(x_k)), then the
 * same 8 for y.  Bond ranks up to 2048.
 * Network (FP32): x^ = (f - mu_x) / sd_x; h1 = tanh(W1 x^ + b1);
 * h2 = tanh(W2 h1 + b2); o = W3 h2 + b3; prediction = o * sd_y + mu_y
 * (in ln units: ln rho_k, ln l*_k).
 * theta (HATT_RANKPRED_NTHETA floats): W1[128][21] b1[128] W2[128][128]
 * b2[128] W3[2][128] b3[2], row-major; stats (HATT_RANKPRED_NSTATS floats):
 * mu_x[21] sd_x[21] mu_y[2] sd_y[2].  All buffers are device FP32 and owned
 * by the caller; every call only enqueues work on `stream`.
 */
#define HATT_RANKPRED_NIN 21
#define HATT_RANKPRED_NTHETA 19586
#define HATT_RANKPRED_NSTATS 46

/* feat: device float [rows][21], rows as above. */
HATT_API hatt_status hatt_rankpred_features(int32_t npairs, const hatt_tt *x, const hatt_tt *y, float *feat,
                                           void *stream);
/* stats = column means and population standard deviations of feat [rows][21]
 * and label [rows][2] (a deviation below 1e-8 is stored as 1). */
HATT_API hatt_status hatt_rankpred_fit_stats(const float *feat, const float *label, int64_t rows, float *stats,
                                            void *stream);
/* pred: device float [rows][2], the network's predictions (ln rho, ln l*). */
HATT_API hatt_status hatt_rankpred_forward(const float *theta, const float *stats, const float *feat,
                                          int64_t rows, float *pred, void *stream);
/* Workspace bytes of hatt_rankpred_grad / hatt_rankpred_train_step for a
 * minibatch of `batch` rows. */
HATT_API size_t hatt_rankpred_ws_bytes(int64_t batch);
/* Gradient (grad: device float [NTHETA]) and value (loss: device float [1])
 * of L = 1/(2B) sum over the B = batch rows idx[0..B) (device int32 row
 * numbers into feat/label) of |o - (label - mu_y) / sd_y|^2. */
HATT_API hatt_status hatt_rankpred_grad(const float *theta, const float *stats, const float *feat,
                                       const float *label, const int32_t *idx, int64_t batch, float *grad,
                                       float *loss, void *ws, size_t ws_bytes, void *stream);
typedef struct {
  double lr, beta1, beta2, eps;  /* Kingma and Ba's Adam; <= 0 picks 1e-3, 0.9, 0.999, 1e-8 */
} hatt_adam_opts;
/* One Adam step (Kingma and Ba, ICLR 2015, Alg. 1) on the same loss: theta,
 * m and v (device float [NTHETA]) are updated in place; step counts from 1;
 * loss (device float [1], may be NULL) receives the minibatch loss before
 * the update. */
HATT_API hatt_status hatt_rankpred_train_step(float *theta, float *adam_m, float *adam_v, int64_t step,
                                             const hatt_adam_opts *opts, const float *stats, const float *feat,
                                             const float *label, const int32_t *idx, int64_t batch, float *loss,
                                             void *ws, size_t ws_bytes, void *stream);
/* Host only: training targets of one accepted tolerance-mode
 * recompression of order d: for bond k = 1..d-1, row k-1 of out (host float
 * [d-1][2]) is (ln rho_k, ln min(cap_k, rho_k + p)), from the kept ranks
 * (host [d+1], each >= 1) and the widths the growth may reach (host [d+1],
 * e.g. cap_out of hatt_adaptive_plan); p = oversample (<= 0 means 8). */
HATT_API hatt_status hatt_rankpred_labels(int32_t d, const int64_t *kept, const int64_t *cap, int32_t oversample,
                                         float *out);
/* Host only: widths and predicted kept ranks from predictions (host float
 * [rows][2], e.g. copied back from hatt_rankpred_forward).  Per bond
 * l_k = ceil((1 + margin) max(e^{pred_1}, e^{pred_0} + p)) and
 * rho_k = ceil(e^{pred_0}), both >= 1; l is then clamped as in hatt_plan.
 * ell_out / rho_out: host, d_p + 1 entries per pair, concatenated in pair
 * order (entries 0 and d_p are 1). */
HATT_API hatt_status hatt_rankpred_widths(int32_t npairs, const hatt_tt *x, const hatt_tt *y, const float *pred,
                                         double margin, int32_t oversample, int64_t *ell_out, int64_t *rho_out);

/* Message describing the last error of the calling thread ("" if none). */
HATT_API const char *hatt_last_error(void);

/* Library version string. */
HATT_API const char *hatt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HATT_H_ */
