// Host side of libhatt: validation, planning, workspace carving and the
// kernel sequences of HaTT (Alg. 3 + Alg. 4), TT-Rounding (Alg. 1), the
// explicit PKP Hadamard product and the TT norm.  Everything here runs on the
// host and only enqueues kernels; no device memory is allocated.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>

#include <algorithm>
#include <memory>
#include <functional>
#include <mutex>
#include <thread>
#include <string>
#include <map>
#include <vector>

#include "common.h"
#include "hatt.h"

using namespace hatt;

// Scratch of hatt_recompress_noalloc: a library-owned device array used in
// place of a caller workspace, for callers that cannot allocate device
// memory.  In host code `hatt_scratch` names a host-side stand-in; its
// device address comes from hipGetSymbolAddress, resolved once per device
// (each device holds its own copy, kept until the process ends) and used
// wherever host code needs the array.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) char hatt_scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

hatt_status fail(hatt_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

struct Shape {
  int d = 0;
  int batch = 0;
  std::vector<int64_t> n, r, off;
  int64_t total = 0;
  int64_t stride = 0;
  double *data = nullptr;
};

void make_offsets(const std::vector<int64_t> &n, const std::vector<int64_t> &r,
                  std::vector<int64_t> *off, int64_t *total) {
  const int d = (int)n.size();
  off->assign(d, 0);
  int64_t acc = 0;
  for (int k = 0; k < d; ++k) {
    (*off)[k] = acc;
    acc += r[k] * n[k] * r[k + 1];
  }
  *total = acc;
}

hatt_status read_tt(const hatt_tt *t, const char *name, Shape *s, bool need_data) {
  if (t == nullptr) return fail(HATT_EINVAL, std::string(name) + ": NULL tensor view");
  if (t->d < 1) return fail(HATT_EINVAL, std::string(name) + ": d must be >= 1");
  if (t->batch < 1) return fail(HATT_EINVAL, std::string(name) + ": batch must be >= 1");
  if (t->n == nullptr || t->rank == nullptr)
    return fail(HATT_EINVAL, std::string(name) + ": NULL n or rank array");
  s->d = t->d;
  s->batch = t->batch;
  s->n.assign(t->n, t->n + t->d);
  s->r.assign(t->rank, t->rank + t->d + 1);
  for (int k = 0; k < t->d; ++k)
    if (s->n[k] < 1) return fail(HATT_ESHAPE, std::string(name) + ": mode size < 1");
  for (int k = 0; k <= t->d; ++k)
    if (s->r[k] < 1) return fail(HATT_ESHAPE, std::string(name) + ": rank < 1");
  if (s->r[0] != 1 || s->r[t->d] != 1)
    return fail(HATT_ESHAPE, std::string(name) + ": rank[0] and rank[d] must be 1");
  make_offsets(s->n, s->r, &s->off, &s->total);
  if (t->batch_stride != 0 && t->batch_stride < s->total)
    return fail(HATT_EINVAL, std::string(name) + ": batch_stride smaller than one train");
  s->stride = t->batch_stride ? t->batch_stride : s->total;
  s->data = t->data;
  if (need_data && s->data == nullptr) return fail(HATT_EINVAL, std::string(name) + ": NULL data");
  return HATT_OK;
}

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;

hatt_status scratch_address(void **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(HATT_EDEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return HATT_OK;
  }
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(hatt_scratch));
  if (e != hipSuccess || p == nullptr)
    return fail(HATT_EDEVICE, std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e));
  g_scratch_ptr[dev] = p;
  *out = p;
  return HATT_OK;
}

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures.
struct Ws {
  char *base;
  size_t off = 0;
  explicit Ws(void *b) : base((char *)b) {}
  double *d(int64_t count) {
    size_t bytes = ((size_t)std::max<int64_t>(count, 1) * 8 + 255) & ~(size_t)255;
    double *p = base ? (double *)(base + off) : nullptr;
    off += bytes;
    return p;
  }
  int64_t *i64(int64_t count) { return (int64_t *)d(count); }
};

// Optional per-launch timing: when enabled, every launcher call below is
// bracketed by two HIP events on its stream and attributed to a kernel class.
// Every launch made inside a QR (CholeskyQR2 GEMMs and Cholesky factors,
// Householder TSQR, panel projections) is attributed to the class "qr".
enum { P_SKETCH, P_PKP, P_LAST, P_SANDWICH, P_GEMM, P_QR, P_SVD, P_OTHER, P_NCLASS };
const char *kClassNames[P_NCLASS] = {"sketch_fill", "pkp_expand", "hpcrl_last", "sandwich",
                                     "gemm_f64",    "qr",         "svd_trunc",  "copy_fill_norm"};
int g_class_override = -1;
struct ClassScope {
  int prev;
  explicit ClassScope(int c) : prev(g_class_override) { g_class_override = c; }
  ~ClassScope() { g_class_override = prev; }
};
// QR method: 0 = CholeskyQR2 where it applies (<= 64 columns) with per-pair
// Householder fallback, 1 = Householder TSQR only.
bool g_use_chol = true;
struct ProfRec {
  int cls;
  hipEvent_t a, b;
  std::string site;
};
// Label of the next launch for the per-site report (set by helpers that
// know the shape, e.g. the GEMM dispatcher); empty: the launcher's name.
std::string g_site;
std::string g_prof_report;
struct Profiler {
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};
Profiler g_prof;

int class_of(const char *expr) {
  if (g_class_override >= 0) return g_class_override;
  if (strstr(expr, "launch_gemm") || strstr(expr, "launch_splitk")) return P_GEMM;
  if (strstr(expr, "launch_tsqr")) return P_QR;
  if (strstr(expr, "launch_sandwich")) return P_SANDWICH;
  if (strstr(expr, "launch_svd")) return P_SVD;
  if (strstr(expr, "launch_pkp")) return P_PKP;
  if (strstr(expr, "launch_sketch")) return P_SKETCH;
  return P_OTHER;
}

void site(const char *fmt, ...) {
  if (!g_prof.on) return;
  char b[160];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(b, sizeof b, fmt, ap);
  va_end(ap);
  g_site = b;
}

std::string site_of(const char *expr) {
  std::string lab = g_site;
  if (lab.empty()) {
    const char *e = strchr(expr, '(');
    lab.assign(expr, e ? (size_t)(e - expr) : strlen(expr));
  }
  const char *cls = kClassNames[class_of(expr)];
  return std::string(cls) + ": " + lab;
}

#define LAUNCH(expr)                                                            \
  do {                                                                          \
    if (run) {                                                                  \
      hipEvent_t pa_ = nullptr, pb_ = nullptr;                                  \
      if (g_prof.on) {                                                          \
        pa_ = g_prof.get();                                                     \
        pb_ = g_prof.get();                                                     \
        if (pa_) (void)hipEventRecord(pa_, st);                                       \
      }                                                                         \
      (void)hipGetLastError(); /* report only this launch's own error */        \
      hipError_t e_ = (expr);                                                   \
      if (g_prof.on && pa_ && pb_) {                                            \
        (void)hipEventRecord(pb_, st);                                          \
        g_prof.recs.push_back(ProfRec{class_of(#expr), pa_, pb_, site_of(#expr)}); \
      }                                                                         \
      if (g_prof.on) g_site.clear();                                            \
      if (e_ != hipSuccess)                                                     \
        return fail(HATT_EDEVICE, std::string("HIP error in ") + #expr + ": " + \
                                      hipGetErrorString(e_));                   \
    }                                                                           \
  } while (0)

std::vector<int64_t> clamp_ell(const std::vector<int64_t> &n, const std::vector<int64_t> &rx,
                               const std::vector<int64_t> &ry, const std::vector<int64_t> &req) {
  const int d = (int)n.size();
  std::vector<int64_t> l(d + 1, 1);
  for (int k = 1; k < d; ++k) l[k] = std::max<int64_t>(1, std::min(req[k], rx[k] * ry[k]));
  for (int k = 1; k < d; ++k) l[k] = std::min(l[k], l[k - 1] * n[k - 1]);
  for (int k = d - 1; k >= 1; --k) l[k] = std::min(l[k], n[k] * l[k + 1]);
  return l;
}

// GEMM helper: picks the split and checks the partial buffer.
struct GemmCtx {
  double *part;
  int64_t part_cap;   // doubles available
  int64_t part_need;  // max requested (measuring)
};

// Storage / compute types of one product: prec = 1 (2) runs it on the FP32 (BF16) matrix
// cores (no K split); a32 / b32 / c32 mark FP32 storage of A / B / C.
struct GemmTypes {
  int prec = 0, a32 = 0, b32 = 0, c32 = 0;
};

// ---------------------------------------------------------------------------
// Autotuner.  In record mode the first launch of a shape bucket times its
// candidate configurations on the caller's stream (one untimed and three
// timed launches each, HIP events, a host wait) and keeps the fastest; use
// mode takes the recorded choices and leaves unseen buckets to the fixed
// rules.  Buckets: a GEMM by (M, N, K, batch, compute type, operand layouts),
// its candidates the K splits 1..64; a sandwich by (its shapes, output
// layout, type), its candidates the kernel and chunk choices of SwForce.
// Tuning is skipped while the stream is being captured into a graph and for
// a GEMM that accumulates into C (its repeated launches would not be
// idempotent).
struct TuneEntry {
  int ks = 1;
  SwForce f{};
  double us = 0.0, us_default = 0.0;
  std::string choice;
};
std::mutex g_tune_mu;
int g_tune_mode = 0;
std::map<std::string, TuneEntry> g_tune;

bool stream_capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

bool tune_get(const std::string &key, TuneEntry *e) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *e = it->second;
  return true;
}

void tune_put(const std::string &key, const TuneEntry &e) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[key] = e;
}

// Microseconds per launch of fn on st (one untimed launch first); < 0 when a
// launch fails.
template <class F>
double time_launches(hipStream_t st, F fn) {
  constexpr int reps = 3;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
  double us = -1.0;
  bool ok = fn() == hipSuccess && hipEventRecord(e0, st) == hipSuccess;
  for (int r = 0; ok && r < reps; ++r) ok = fn() == hipSuccess;
  float ms = 0.0f;
  if (ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
      hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
    us = 1000.0 * ms / reps;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return us;
}

std::string sandwich_tune_key(const SandwichArgs &a) {
  char b[160];
  // the unit-stride flags tell the W_L build from the core update of equal shapes
  snprintf(b, sizeof b, "sandwich RA=%d RI=%d SI=%d SO=%d n=%lld G=%lld batch=%d og1=%d cg1=%d ylr1=%d prec=%d", a.RA,
           a.RI, a.SI, a.SO, (long long)a.n, (long long)a.G, a.batch, a.og == 1 ? 1 : 0, a.cg == 1 ? 1 : 0,
           a.ylr == 1 ? 1 : 0, a.prec);
  return b;
}

// The sandwich override for this launch (false: the fixed rules); in record
// mode an unseen bucket is tuned here first.
bool sandwich_tune(bool run, const SandwichArgs &a, hipStream_t st, SwForce *out) {
  if (g_tune_mode == 0) return false;
  const std::string key = sandwich_tune_key(a);
  TuneEntry e;
  if (tune_get(key, &e)) {
    *out = e.f;
    return true;
  }
  if (g_tune_mode != 1 || !run || stream_capturing(st)) return false;
  std::vector<SwForce> cands(1);  // the fixed rules first
  SwForce f;
  f.no_ks = 1;
  cands.push_back(f);
  f = SwForce{};
  f.no_slice = 1;
  cands.push_back(f);
  for (int div : {2, 4}) {
    f = SwForce{};
    f.gc_div = div;
    cands.push_back(f);
  }
  if (a.prec == 0) {
    f = SwForce{};
    f.valu = 1;
    cands.push_back(f);
  }
  // distinct launches only: candidates that resolve to the same kernel and plan are timed once
  std::vector<std::string> seen;
  double best = -1.0, def = -1.0;
  SwForce bf{};
  std::string bname;
  for (size_t c = 0; c < cands.size(); ++c) {
    const SwForce &fc = cands[c];
    SwPlan pl{};
    std::string sig = sandwich_kernel_name(a, &fc);
    if (!fc.valu && sandwich_mfma_plan(a, kSandwichLdsDoubles, &pl, &fc))
      sig += " GC=" + std::to_string(pl.GC) + " ks=" + std::to_string(pl.ks) + " slice=" + std::to_string(pl.slice);
    if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;
    seen.push_back(sig);
    const double us = time_launches(st, [&]() { return launch_sandwich(a, st, &fc); });
    if (us < 0.0) {
      (void)hipGetLastError();
      continue;
    }
    if (c == 0) def = us;
    if (best < 0.0 || us < best) {
      best = us;
      bf = fc;
      bname = sig;
    }
  }
  if (best < 0.0) return false;
  e.f = bf;
  e.us = best;
  e.us_default = def;
  e.choice = bname;
  tune_put(key, e);
  *out = bf;
  return true;
}

hatt_status gemm(bool run, GemmCtx &gc, CMat A, CMat B, Mat C, int64_t M, int64_t N, int64_t K,
                 double alpha, double beta, int batch, hipStream_t st, bool allow_split,
                 const int *run_flag = nullptr, int64_t run_flag_stride = 0, int *ks_out = nullptr,
                 GemmTypes ty = GemmTypes{}, int run_when = 1) {
  GemmArgs g{};
  g.prec = ty.prec;
  g.a_f32 = ty.a32;
  g.b_f32 = ty.b32;
  g.c_f32 = ty.c32;
  g.no_reduce = 1;  // the reduction, when needed, is its own launch below
  g.run_flag = run_flag;
  g.run_flag_stride = run_flag_stride;
  g.run_when = run_when;
  g.A = A;
  g.B = B;
  g.C = C;
  g.M = M;
  g.N = N;
  g.K = K;
  g.alpha = alpha;
  g.beta = beta;
  g.batch = batch;
  g.ksplit = allow_split ? gemm_pick_ksplit(M, N, K, batch) : 1;
  // autotuner: the K split of this product's bucket
  std::vector<int> cands;
  std::string tkey;
  if (g_tune_mode != 0 && allow_split && beta == 0.0 && ks_out == nullptr && run_flag == nullptr &&
      !(run && (C.ptr == A.ptr || C.ptr == B.ptr))) {
    char kb[200];
    snprintf(kb, sizeof kb, "gemm %lldx%lldx%lld batch=%d prec=%d a32=%d b32=%d c32=%d A=%d%d B=%d%d C=%d%d",
             (long long)M, (long long)N, (long long)K, batch, ty.prec, ty.a32, ty.b32, ty.c32, A.rs == 1, A.cs == 1,
             B.rs == 1, B.cs == 1, C.rs == 1, C.cs == 1);
    tkey = kb;
    TuneEntry te;
    if (tune_get(tkey, &te)) {
      g.ksplit = te.ks;
    } else if (g_tune_mode == 1) {
      for (int ks = 1; ks <= 64; ks *= 2)
        if (ks == 1 || K >= (int64_t)ks * 64) cands.push_back(ks);
    }
  }
  auto need_of = [&](int ks) { return ks > 1 ? (int64_t)batch * ks * M * N : (int64_t)0; };
  int64_t need = need_of(g.ksplit);
  for (int ks : cands) need = std::max(need, need_of(ks));
  gc.part_need = std::max(gc.part_need, need);
  if (g.ksplit > 1 && need_of(g.ksplit) > gc.part_cap) g.ksplit = 1;
  g.part = gc.part;
  if (run && !cands.empty() && !stream_capturing(st)) {
    const int ks_default = g.ksplit;
    double best = -1.0, def = -1.0;
    int bks = ks_default;
    for (int ks : cands) {
      if (need_of(ks) > gc.part_cap) continue;
      GemmArgs t = g;
      t.ksplit = ks;
      const double us = time_launches(st, [&]() {
        hipError_t e = launch_gemm(t, st);
        if (e == hipSuccess && ks > 1) e = launch_splitk_reduce(t, st);
        return e;
      });
      if (us < 0.0) {
        (void)hipGetLastError();
        continue;
      }
      if (ks == ks_default) def = us;
      if (best < 0.0 || us < best) {
        best = us;
        bks = ks;
      }
    }
    if (best >= 0.0) {
      TuneEntry te;
      te.ks = bks;
      te.us = best;
      te.us_default = def;
      te.choice = "ks=" + std::to_string(bks);
      tune_put(tkey, te);
      g.ksplit = bks;
    }
  }
  if (ks_out != nullptr) *ks_out = g.ksplit;
  if (g_prof.on) {
    char b[200], kn[96];
    gemm_kernel_name(g, kn, sizeof kn);
    snprintf(b, sizeof b, "gemm %lldx%lldx%lld ks=%d%s [%s]", (long long)M, (long long)N, (long long)K,
             g.ksplit, run_flag ? " flagged" : "", kn);
    g_site = b;
  }
  LAUNCH(launch_gemm(g, st));
  g_site.clear();
  if (g.ksplit > 1 && ks_out == nullptr) {
    site("splitk_reduce %lldx%lld ks=%d", (long long)M, (long long)N, g.ksplit);
    LAUNCH(launch_splitk_reduce(g, st));
  }
  return HATT_OK;
}

// ---------------------------------------------------------------------------
// QR dispatch.  Up to kQrMaxCols columns: one TSQR.  Wider (m >= n): block
// classical Gram-Schmidt with re-orthogonalisation of each panel's Q factor
// (BCGS2 of Barlow and Smoktunowicz), panels of kPanel columns:
//   S1 = Q_prev^T A_p;  W = A_p - Q_prev S1;  W = Q1 R1 (TSQR)
//   S2 = Q_prev^T Q1;   W2 = Q1 - Q_prev S2;  W2 = Q2 R2 (TSQR)
//   R(prev, p) = S1 + S2 R1,  R(p, p) = R2 R1.
// The second pass is what keeps Q orthonormal when a panel is (numerically)
// rank deficient: the first TSQR then completes the panel with normalised
// rounding noise that still has O(1) components along Q_prev.
constexpr int64_t kPanel = 128;  // <= 128 columns: one preconditioned CholeskyQR2 or TSQR per panel

// Sketch-preconditioned CholeskyQR2 (tall frames up to kPcholMaxN columns):
// B = Omega A (k = 256 signed row sums), [~, R0] = Householder QR of B,
// A' = A R0^{-1}, then CholeskyQR2 of A' and R = R2 R1 R0.  R0 equalises the
// column space so that A' is well conditioned even when A is numerically
// rank deficient (a sketched frame wider than the rank it sees); a pair whose
// Cholesky factors still fail the pivot tests is recomputed by Householder
// TSQR, as for plain CholeskyQR2.
constexpr int64_t kPcholMaxN = 128;
constexpr int64_t kPcholSketchRows = 256;  // rows of B (>= 2n for every n <= kPcholMaxN)

struct QrOp {
  int64_t m = 0, n = 0, k = 0;
  bool hh = false;                   // one-workgroup Householder QR (short frames)
  bool pchol = false;                // sketch-preconditioned CholeskyQR2 with TSQR fallback
  int64_t sk_rows = 0;               // pchol: rows of the sketch B
  bool has_direct = false;           // `direct` holds a TSQR plan (the fallback)
  bool chol = false;                 // CholeskyQR2 with per-pair TSQR fallback
  bool big = false;
  bool wide = false;                 // m < n, n > kQrMaxCols: QR of the first m columns, then R2 = Q^T A2
  std::shared_ptr<QrOp> sub;
  QrPlan direct{};
  std::vector<QrOp> panels;          // big: one QR per panel (CholeskyQR2 or TSQR)
  std::vector<QrOp> panels2;         // big: second-pass QR per panel (projected preconditioned CholeskyQR2)
  int64_t panel = 0;                 // big: panel width
  int64_t ws_doubles = 0;  // per pair
  int64_t ws_tree = 0;     // big: TSQR tree part at the front; chol: fallback TSQR tree
};

// CholeskyQR2 (n <= kCholMaxN, m >= n): G = A^T A, R1 = chol(G), Q1 = A R1^{-1},
// then the same on Q1 giving R2; Q = Q1 R2^{-1}, R = R2 R1.  All products run
// on the MFMA GEMM.  A pair whose first Gram matrix has a pivot below 1e-12 of
// its largest diagonal entry (condition number beyond ~1e6, which includes
// rank-deficient inputs), or whose second Gram matrix is not close to the
// identity, is recomputed by Householder TSQR instead; the decision is taken
// on the device, per pair, so no host synchronisation is needed.
constexpr double kCholThr1 = 1e-12;
constexpr double kCholThr2 = 0.5;

int64_t chol_ws_doubles(int64_t m, int64_t n) { return m * n + 5 * n * n + 1; }
// pchol scratch after the CholeskyQR2 block: A' (m n), B (k n), R0, R0^{-1},
// T (n n each), the dependent-column mask (n ints)
int64_t pchol_ws_doubles(int64_t m, int64_t n, int64_t k) { return m * n + k * n + 3 * n * n + n; }

// Sketch-preconditioned CholeskyQR2 for the second pass of a panel (any
// m >= n, n <= kPcholMaxN): the sketch keeps min(m, kPcholSketchRows) rows
// (for m at most that, a signed row permutation), the TSQR plan, where one
// exists, is the fallback.
bool qr_prepare_pass2(int64_t m, int64_t n, QrOp *op) {
  *op = QrOp{};
  op->m = m;
  op->n = n;
  op->k = std::min(m, n);
  op->sk_rows = std::min<int64_t>(m, kPcholSketchRows);
  if (m < n || n > kPcholMaxN || !hh_qr_supported(op->sk_rows, n)) return false;
  op->pchol = true;
  op->has_direct = qr_make_plan(m, n, &op->direct);
  op->ws_tree = op->has_direct ? op->direct.ws_doubles : 0;
  op->ws_doubles = op->ws_tree + chol_ws_doubles(m, n) + pchol_ws_doubles(m, n, op->sk_rows);
  return true;
}

bool qr_prepare(int64_t m, int64_t n, QrOp *op) {
  op->m = m;
  op->n = n;
  op->k = std::min(m, n);
  op->big = op->wide = op->chol = op->hh = op->pchol = false;
  op->ws_doubles = 0;
  op->ws_tree = 0;
  // short frames: one workgroup runs the Householder QR in registers
  if (g_use_chol && m >= n && hh_qr_supported(m, n)) {
    op->hh = true;
    return true;
  }
  // wide frames: QR of the first m columns, then R2 = Q^T A2 (qr_exec)
  if (g_use_chol && m < n && hh_qr_supported(m, m)) {
    op->wide = true;
    op->sub = std::make_shared<QrOp>();
    if (!qr_prepare(m, m, op->sub.get())) return false;
    op->ws_doubles = op->sub->ws_doubles;
    return true;
  }
  // tall frames up to kPcholMaxN columns: CholeskyQR2 (many pairs of at
  // most 64 columns) or its sketch-preconditioned form, with the Householder
  // TSQR fallback where a TSQR plan exists
  if (g_use_chol && m >= n && n <= kPcholMaxN) {
    op->has_direct = qr_make_plan(m, n, &op->direct);
    op->chol = op->has_direct && n <= kCholMaxN;
    op->sk_rows = kPcholSketchRows;
    op->pchol = m >= kPcholSketchRows && hh_qr_supported(kPcholSketchRows, n);
    if (op->chol || op->pchol) {
      op->ws_tree = op->has_direct ? op->direct.ws_doubles : 0;
      op->ws_doubles = op->ws_tree + chol_ws_doubles(m, n) + (op->pchol ? pchol_ws_doubles(m, n, op->sk_rows) : 0);
      return true;
    }
  }
  // tall frames wider than one panel go to BCGS2 over panels: the one-shot
  // tree for them has blocks of barely n rows, so it needs many levels and
  // forms Q a few columns at a time
  const bool panelled = g_use_chol && m >= n && n > kPcholMaxN;
  if (n <= kQrMaxCols && !panelled && qr_make_plan(m, n, &op->direct)) {
    op->has_direct = true;
    op->ws_doubles = op->direct.ws_doubles;
    return true;
  }
  if (m < n) {
    // Householder reflectors of a wide matrix depend only on its first m columns
    if (n <= kQrMaxCols) return false;
    op->wide = true;
    op->sub = std::make_shared<QrOp>();
    if (!qr_prepare(m, m, op->sub.get())) return false;
    op->ws_doubles = op->sub->ws_doubles;
    return true;
  }
  op->big = true;
  op->panels.clear();
  op->panels2.clear();
  // panels: preconditioned CholeskyQR2 takes 128 columns; a Householder TSQR
  // panel (method 1) at most 64, where a tree of >= 2n-row blocks exists
  const int64_t panel = g_use_chol ? kPanel : 64;
  if (n <= panel) return false;  // a single panel would recurse into this same shape
  int64_t w = 0;
  for (int64_t c0 = 0; c0 < n; c0 += panel) {
    const int64_t cw = std::min(panel, n - c0);
    QrOp pl, pl2;
    if (!qr_prepare(m, cw, &pl) || pl.big || pl.wide) return false;
    op->panels.push_back(pl);
    w = std::max(w, pl.ws_doubles);
    if (c0 > 0) {
      if (!qr_prepare_pass2(m, cw, &pl2)) return false;
      w = std::max(w, pl2.ws_doubles);
    }
    op->panels2.push_back(pl2);
  }
  op->ws_tree = w;
  op->panel = panel;
  // panel QR scratch + S1, S2 (n x panel each) + R1, R2 (panel x panel each) + dependence mask
  op->ws_doubles = w + 2 * n * panel + 2 * panel * panel + panel;
  return true;
}

constexpr int kCholFuseMinPairs = 32;
// Second-pass dependence threshold of a panel (its columns are projections
// of orthonormal vectors): a direction within 1e-7 of the earlier panels
// carries at most ~1e-14 of the input (the projection's rounding noise).
constexpr double kPass2DepAbs = 1e-7;

// CholeskyQR2 that leaves Q = Q1 R2^{-1} unformed for the pairs it keeps:
// the caller applies Q1 and R2^{-1} itself (Q holds the fallback's Q for the
// flagged pairs, flag 0).
// With q1_in_q set (by the caller), Q1 itself is written where Q goes (the
// fallback's Q then replaces it for the flagged pairs), so Q = Q1 R2^{-1}
// there for the kept pairs and Q for the others.
struct QrDeferred {
  bool q1_in_q = false;
  const double *q1 = nullptr, *r2i = nullptr;  // m x n and n x n row-major, pair stride wsp
  const int *flag = nullptr;                   // 1: CholeskyQR2 kept the pair
  int64_t wsp = 0, fst = 0;
  bool used = false;
};

// Optional projection (second pass of a panel): prev holds the c0
// orthonormal columns of the earlier panels and A is already projected
// against them.  Then a sketch pivot at most dep_abs marks its column as
// dependent (A's columns are projections of orthonormal vectors, so such a
// direction lies within that angle of the earlier panels and carries
// nothing of the input), and A' (completion vectors included) is projected
// twice against prev before its CholeskyQR2, so that Q is orthogonal to the
// earlier panels to working precision.  pscr: c0 x n doubles per pair.
struct PcholProj {
  CMat prev{};
  int64_t c0 = 0;
  double *pscr = nullptr;
  double dep_abs = 0.0;
};

hatt_status pchol_exec(bool run, const QrOp &op, CMat A, Mat Q, Mat R, double *ws, int64_t wsp, int P,
                       GemmCtx &gc, hipStream_t st, QrDeferred *def, uint32_t salt,
                       const PcholProj *proj = nullptr) {
  const int64_t m = op.m, n = op.n, k = op.sk_rows;
  double *q1 = ws + op.ws_tree;  // m x n row-major
  double *g = q1 + m * n;
  double *r1 = g + n * n, *r1i = r1 + n * n, *r2 = r1i + n * n, *r2i = r2 + n * n;
  int *flag = reinterpret_cast<int *>(r2i + n * n);
  double *ap = r2i + n * n + 1;
  double *B = ap + m * n, *R0 = B + k * n, *R0i = R0 + n * n, *T = R0i + n * n;
  int *mask = reinterpret_cast<int *>(T + n * n);
  const int64_t fst = 2 * wsp, mbs = 2 * wsp;
  const bool inq = def != nullptr && def->q1_in_q;
  const Mat q1m = inq ? Q : Mat{q1, n, 1, wsp};
  CMat q1c{q1m.ptr, q1m.rs, q1m.cs, q1m.bs}, q1t{q1m.ptr, q1m.cs, q1m.rs, q1m.bs};
  CMat apc{ap, n, 1, wsp}, apt{ap, 1, n, wsp};
  hatt_status sg;
  // preconditioner: R0 of the Householder QR of the row sketch B = Omega A
  site("pchol sketch %lldx%lld k=%lld", (long long)m, (long long)n, (long long)k);
  LAUNCH(launch_sketch_rows(A, m, (int)n, (int)k, B, wsp, 0x9E3779B9u, P, st));
  {
    HhArgs h{};
    h.A = CMat{B, n, 1, wsp};
    h.Q = Mat{nullptr, 0, 0, 0};
    h.R = Mat{R0, n, 1, wsp};
    h.m = k;
    h.n = n;
    site("pchol hh %lldx%lld [%s]", (long long)k, (long long)n, hh_qr_kernel_name(k, n));
    LAUNCH(launch_hh_qr(h, P, st));
  }
  // R0^{-1}; sketch columns that depend on the ones before them (pivot at
  // most 1e-13 of the largest) are marked and their columns of A' replaced
  // by random unit vectors: Q then spans range(A) plus those directions
  site("pchol trinv %lld", (long long)n);
  LAUNCH(launch_trinv(R0, wsp, R0i, wsp, (int)n, flag, fst, 1, mask, mbs, proj ? proj->dep_abs : 0.0, P, st));
  sg = gemm(run, gc, A, CMat{R0i, n, 1, wsp}, Mat{ap, n, 1, wsp}, m, n, n, 1.0, 0.0, P, st, false);
  if (sg != HATT_OK) return sg;
  site("pchol complete %lldx%lld", (long long)m, (long long)n);
  LAUNCH(launch_complete_cols(ap, m, (int)n, wsp, mask, mbs, 0x7F4A7C15u ^ (salt * 0x9E3779B9u), P, st));
  if (proj != nullptr && proj->c0 > 0) {
    const CMat pv = proj->prev, pvt{pv.ptr, pv.cs, pv.rs, pv.bs};
    for (int pass = 0; pass < 2; ++pass) {
      sg = gemm(run, gc, pvt, apc, Mat{proj->pscr, n, 1, wsp}, proj->c0, n, m, 1.0, 0.0, P, st, true);
      if (sg != HATT_OK) return sg;
      sg = gemm(run, gc, pv, CMat{proj->pscr, n, 1, wsp}, Mat{ap, n, 1, wsp}, m, n, proj->c0, -1.0, 1.0, P, st,
                false);
      if (sg != HATT_OK) return sg;
    }
  }
  // CholeskyQR2 of A'
  sg = gemm(run, gc, apt, apc, Mat{g, n, 1, wsp}, n, n, m, 1.0, 0.0, P, st, true);
  if (sg != HATT_OK) return sg;
  site("pchol chol1k %lld", (long long)n);
  LAUNCH(launch_chol1k(g, wsp, r1, r1i, wsp, (int)n, flag, fst, 0, kCholThr1, P, st));
  sg = gemm(run, gc, apc, CMat{r1i, n, 1, wsp}, q1m, m, n, n, 1.0, 0.0, P, st, false);
  if (sg != HATT_OK) return sg;
  sg = gemm(run, gc, q1t, q1c, Mat{g, n, 1, wsp}, n, n, m, 1.0, 0.0, P, st, true);
  if (sg != HATT_OK) return sg;
  site("pchol chol1k %lld", (long long)n);
  LAUNCH(launch_chol1k(g, wsp, r2, r2i, wsp, (int)n, flag, fst, 0, kCholThr2, P, st));
  if (R.ptr) {
    // R = Q^T A = R2^{-T} (Q1^T A), exact because range(Q) contains range(A);
    // formed before Q is written (Q may share A's buffer)
    sg = gemm(run, gc, q1t, A, Mat{T, n, 1, wsp}, n, n, m, 1.0, 0.0, P, st, true);
    if (sg != HATT_OK) return sg;
    sg = gemm(run, gc, CMat{r2i, 1, n, wsp}, CMat{T, n, 1, wsp}, R, n, n, n, 1.0, 0.0, P, st, false, flag, fst);
    if (sg != HATT_OK) return sg;
  }
  if (def != nullptr) {
    def->q1 = q1m.ptr;
    def->r2i = r2i;
    def->flag = flag;
    def->wsp = wsp;
    def->fst = fst;
    def->used = true;
  } else {
    sg = gemm(run, gc, q1c, CMat{r2i, n, 1, wsp}, Q, m, n, n, 1.0, 0.0, P, st, false, flag, fst);
    if (sg != HATT_OK) return sg;
  }
  if (op.has_direct) {
    site("tsqr fallback %lldx%lld", (long long)m, (long long)n);
    LAUNCH(launch_tsqr(op.direct, A, Q, R, ws, wsp, P, st, flag, fst));
  }
  return HATT_OK;
}

hatt_status cholqr2_exec(bool run, const QrOp &op, CMat A, Mat Q, Mat R, double *ws, int64_t wsp, int P,
                         GemmCtx &gc, hipStream_t st, QrDeferred *def = nullptr) {
  const int64_t m = op.m, n = op.n;
  double *q1 = ws + op.ws_tree;  // m x n row-major
  double *g = q1 + m * n;
  double *r1 = g + n * n, *r1i = r1 + n * n, *r2 = r1i + n * n, *r2i = r2 + n * n;
  int *flag = reinterpret_cast<int *>(r2i + n * n);
  const int64_t fst = 2 * wsp;  // flag stride in ints
  CMat At{A.ptr, A.cs, A.rs, A.bs};
  const bool inq = def != nullptr && def->q1_in_q;
  const Mat q1m = inq ? Q : Mat{q1, n, 1, wsp};
  CMat q1c{q1m.ptr, q1m.rs, q1m.cs, q1m.bs}, q1t{q1m.ptr, q1m.cs, q1m.rs, q1m.bs};
  hatt_status sg;
  if (P >= kCholFuseMinPairs) {
    // many pairs fill the GPU with one block per pair: each block forms its
    // pair's Gram matrix on the matrix cores and factors it in place
    site("gram+chol %lldx%lld", (long long)m, (long long)n);
    LAUNCH(launch_gram_chol(A, m, (int)n, r1, r1i, wsp, flag, fst, 1, kCholThr1, P, st));
    sg = gemm(run, gc, A, CMat{r1i, n, 1, wsp}, q1m, m, n, n, 1.0, 0.0, P, st, false);
    if (sg != HATT_OK) return sg;
    site("gram+chol %lldx%lld", (long long)m, (long long)n);
    LAUNCH(launch_gram_chol(q1c, m, (int)n, r2, r2i, wsp, flag, fst, 0, kCholThr2, P, st));
  } else {
    // few pairs: a split-K Gram GEMM (with its parallel reduction) spreads the
    // long K over the GPU, then one block per pair factors G
    sg = gemm(run, gc, At, A, Mat{g, n, 1, wsp}, n, n, m, 1.0, 0.0, P, st, true);
    if (sg != HATT_OK) return sg;
    site("chol %lld", (long long)n);
    LAUNCH(launch_chol(g, wsp, 1, 0, r1, r1i, wsp, (int)n, flag, fst, 1, kCholThr1, P, st));
    sg = gemm(run, gc, A, CMat{r1i, n, 1, wsp}, q1m, m, n, n, 1.0, 0.0, P, st, false);
    if (sg != HATT_OK) return sg;
    sg = gemm(run, gc, q1t, q1c, Mat{g, n, 1, wsp}, n, n, m, 1.0, 0.0, P, st, true);
    if (sg != HATT_OK) return sg;
    site("chol %lld", (long long)n);
    LAUNCH(launch_chol(g, wsp, 1, 0, r2, r2i, wsp, (int)n, flag, fst, 0, kCholThr2, P, st));
  }
  if (def != nullptr) {
    def->q1 = q1m.ptr;
    def->r2i = r2i;
    def->flag = flag;
    def->wsp = wsp;
    def->fst = fst;
    def->used = true;
  } else {
    sg = gemm(run, gc, q1c, CMat{r2i, n, 1, wsp}, Q, m, n, n, 1.0, 0.0, P, st, false, flag, fst);
    if (sg != HATT_OK) return sg;
  }
  if (R.ptr) {
    sg = gemm(run, gc, CMat{r2, n, 1, wsp}, CMat{r1, n, 1, wsp}, R, n, n, n, 1.0, 0.0, P, st, false, flag, fst);
    if (sg != HATT_OK) return sg;
  }
  site("tsqr fallback %lldx%lld", (long long)m, (long long)n);
  LAUNCH(launch_tsqr(op.direct, A, Q, R, ws, wsp, P, st, flag, fst));
  return HATT_OK;
}

// A (m x n), Q (m x k), R (k x n row-major with row stride r.rs, or null).
// R, when given, must be a contiguous per-pair block of rbuf doubles.
// salt: distinguishes the random completion vectors of the QRs of one block
// Gram-Schmidt (its panels and passes share one column space).
hatt_status qr_exec(bool run, const QrOp &op, CMat A, Mat Q, Mat R, int64_t rbuf, double *ws, int64_t wsp,
                    int P, GemmCtx &gc, hipStream_t st, QrDeferred *def = nullptr, uint32_t salt = 0) {
  ClassScope cls(P_QR);
  if (op.wide) {
    hatt_status s0 = qr_exec(run, *op.sub, A, Q, R, rbuf, ws, wsp, P, gc, st);
    if (s0 != HATT_OK) return s0;
    if (R.ptr) {
      const int64_t m = op.m;
      return gemm(run, gc, CMat{Q.ptr, Q.cs, Q.rs, Q.bs}, CMat{A.ptr + m * A.cs, A.rs, A.cs, A.bs},
                  Mat{R.ptr + m * R.cs, R.rs, R.cs, R.bs}, m, op.n - m, m, 1.0, 0.0, P, st, true);
    }
    return HATT_OK;
  }
  if (op.hh) {
    HhArgs h{};
    h.A = A;
    h.Q = Q;
    h.R = R.ptr ? R : Mat{nullptr, 0, 0, 0};
    h.m = op.m;
    h.n = op.n;
    site("hh %lldx%lld [%s]", (long long)op.m, (long long)op.n, hh_qr_kernel_name(op.m, op.n));
    LAUNCH(launch_hh_qr(h, P, st));
    return HATT_OK;
  }
  // many pairs of at most 64 columns: the fused Gram + Cholesky blocks
  if (op.pchol && !(op.chol && P >= kCholFuseMinPairs))
    return pchol_exec(run, op, A, Q, R, ws, wsp, P, gc, st, def, salt);
  if (op.chol) return cholqr2_exec(run, op, A, Q, R, ws, wsp, P, gc, st, def);
  if (!op.big) {
    site("tsqr %lldx%lld", (long long)op.m, (long long)op.n);
    LAUNCH(launch_tsqr(op.direct, A, Q, R, ws, wsp, P, st));
    return HATT_OK;
  }
  const int64_t m = op.m, n = op.n;
  double *s1buf = ws + op.ws_tree;
  double *s2buf = s1buf + n * op.panel;
  double *r1buf = s2buf + n * op.panel;
  double *r2buf = r1buf + op.panel * op.panel;
  int *pmask = reinterpret_cast<int *>(r2buf + op.panel * op.panel);
  LAUNCH(launch_copy(A, Q, m, n, P, st));
  if (R.ptr) LAUNCH(launch_fill(R.ptr, (int64_t)P * rbuf, 0.0, st));
  int pi = 0;
  for (int64_t c0 = 0; c0 < n; c0 += op.panel, ++pi) {
    const int64_t cw = std::min(op.panel, n - c0);
    CMat Qprev{Q.ptr, Q.rs, Q.cs, Q.bs};
    CMat QprevT{Q.ptr, Q.cs, Q.rs, Q.bs};
    Mat Qpan{Q.ptr + c0 * Q.cs, Q.rs, Q.cs, Q.bs};
    CMat Qpanc{Qpan.ptr, Qpan.rs, Qpan.cs, Qpan.bs};
    Mat rdiag = R.ptr ? Mat{R.ptr + c0 * R.rs + c0 * R.cs, R.rs, R.cs, R.bs} : Mat{nullptr, 0, 0, 0};
    if (c0 == 0) {
      hatt_status sp0 = qr_exec(run, op.panels[pi], Qpanc, Qpan, rdiag, rbuf, ws, wsp, P, gc, st, nullptr, 1u);
      if (sp0 != HATT_OK) return sp0;
      continue;
    }
    // first pass: S1 goes straight into R's block above the diagonal
    Mat s1 = R.ptr ? Mat{R.ptr + c0 * R.cs, R.rs, R.cs, R.bs} : Mat{s1buf, cw, 1, wsp};
    CMat s1c{s1.ptr, s1.rs, s1.cs, s1.bs};
    hatt_status sg = gemm(run, gc, QprevT, Qpanc, s1, c0, cw, m, 1.0, 0.0, P, st, true);
    if (sg != HATT_OK) return sg;
    sg = gemm(run, gc, Qprev, s1c, Qpan, m, cw, c0, -1.0, 1.0, P, st, false);
    if (sg != HATT_OK) return sg;
    // columns already in the span of the previous panels (residual at most
    // 1e-12 of the column) become random vectors for the panel QR, and their
    // R1 columns zero: A_p = Q_prev S1 + Q1 R1 then still holds to that level,
    // and both passes work on a well-conditioned panel
    site("panel dependence %lldx%lld", (long long)m, (long long)cw);
    LAUNCH(launch_panel_dep(Qpan, s1c, m, c0, (int)cw, pmask, 2 * wsp, 1e-12, 0x51ED270Bu ^ (uint32_t)pi, P, st));
    Mat r1 = R.ptr ? Mat{r1buf, cw, 1, wsp} : Mat{nullptr, 0, 0, 0};
    sg = qr_exec(run, op.panels[pi], Qpanc, Qpan, r1, rbuf, ws, wsp, P, gc, st, nullptr, 2u * (uint32_t)pi + 2u);
    if (sg != HATT_OK) return sg;
    if (R.ptr) LAUNCH(launch_zero_masked_cols(r1, (int)cw, (int)cw, pmask, 2 * wsp, P, st));
    // second pass on the orthonormalised panel
    sg = gemm(run, gc, QprevT, Qpanc, Mat{s2buf, cw, 1, wsp}, c0, cw, m, 1.0, 0.0, P, st, true);
    if (sg != HATT_OK) return sg;
    sg = gemm(run, gc, Qprev, CMat{s2buf, cw, 1, wsp}, Qpan, m, cw, c0, -1.0, 1.0, P, st, false);
    if (sg != HATT_OK) return sg;
    // the panel now spans what the input adds to the earlier panels, plus
    // directions that the first pass took from rounding noise; those lie
    // within a small angle of the earlier panels, so this pass replaces
    // them (sketch pivots below 1e-7) by random directions orthogonal to
    // the earlier panels
    Mat r2 = R.ptr ? Mat{r2buf, cw, 1, wsp} : Mat{nullptr, 0, 0, 0};
    PcholProj pj;
    pj.prev = Qprev;
    pj.c0 = c0;
    pj.pscr = s1buf;
    pj.dep_abs = kPass2DepAbs;
    sg = pchol_exec(run, op.panels2[pi], Qpanc, Qpan, r2, ws, wsp, P, gc, st, nullptr, 2u * (uint32_t)pi + 3u, &pj);
    if (sg != HATT_OK) return sg;
    if (R.ptr) {
      // R(prev, p) += S2 R1;  R(p, p) = R2 R1
      sg = gemm(run, gc, CMat{s2buf, cw, 1, wsp}, CMat{r1buf, cw, 1, wsp}, s1, c0, cw, cw, 1.0, 1.0, P, st,
                false);
      if (sg != HATT_OK) return sg;
      sg = gemm(run, gc, CMat{r2buf, cw, 1, wsp}, CMat{r1buf, cw, 1, wsp}, rdiag, cw, cw, cw, 1.0, 0.0, P, st,
                false);
      if (sg != HATT_OK) return sg;
    }
  }
  return HATT_OK;
}

// SVD + rank choice dispatch: one-workgroup Jacobi when the matrix fits in
// LDS, else block Jacobi over global memory (scratch `big` of kr*nc doubles
// per pair plus 2 ints).
// Sweeps enqueued for the block Jacobi (a sweep after convergence returns at
// once on the device flags, so spare sweeps cost only their launches): 24
// covers dense random 1296-column matrices, which 14 did not.
constexpr int kBigSweeps = 24;

int64_t svd_ws_doubles(int kr, int nc) {
  if (nc <= kSvdMaxN && (int64_t)kr * nc <= kQrLdsDoubles) return 0;
  return (int64_t)kr * nc + 1;
}

hatt_status svd_exec(bool run, const SvdArgs &sa, double *big, int64_t bigp, int *flags, GemmCtx &gc,
                     hipStream_t st) {
  if (sa.nc <= kSvdMaxN && (int64_t)sa.kr * sa.nc <= kQrLdsDoubles) {
    site("svd %dx%d", sa.kr, sa.nc);
    LAUNCH(launch_svd_trunc(sa, st));
    if (sa.nc <= 64) return HATT_OK;
    // the one-workgroup Jacobi above 64 columns leaves S V^T = U^T R to a GEMM
    return gemm(run, gc, CMat{sa.u, 1, sa.ucap, sa.ubs}, CMat{sa.r, sa.nc, 1, sa.rbs}, Mat{sa.svt, sa.nc, 1, sa.sbs},
                sa.ucap, sa.nc, sa.kr, 1.0, 0.0, sa.batch, st, true);
  }
  if (sa.nc > kSvdBigMaxN)
    return fail(HATT_EUNSUPPORTED, "SVD of more than " + std::to_string(kSvdBigMaxN) + " columns is not built");
  const int bw = svd_big_block_width(sa.kr);
  if (bw < 1) return fail(HATT_EUNSUPPORTED, "SVD column too long for the block Jacobi");
  int nb = (sa.nc + bw - 1) / bw;
  nb += nb & 1;
  LAUNCH(launch_svd_big_prepare(sa.r, sa.rbs, sa.kr, sa.nc, big, bigp, flags, sa.batch, st));
  for (int sw = 0; sw < kBigSweeps; ++sw) {
    for (int t = 0; t < nb - 1; ++t)
      LAUNCH(launch_svd_big_round(big, bigp, sa.kr, sa.nc, bw, nb, t, flags, sa.batch, st));
    LAUNCH(launch_svd_big_sweep_end(flags, sa.batch, st));
  }
  LAUNCH(launch_svd_big_finish(sa, big, bigp, st));
  // S V^T = U^T R (rows beyond the kept rank are zero because U's columns are)
  return gemm(run, gc, CMat{sa.u, 1, sa.ucap, sa.ubs}, CMat{sa.r, sa.nc, 1, sa.rbs}, Mat{sa.svt, sa.nc, 1, sa.sbs},
              sa.ucap, sa.nc, sa.kr, 1.0, 0.0, sa.batch, st, true);
}

// ---------------------------------------------------------------------------
// TT-Rounding (Alg. 1) of `batch` trains.
//   src: cores with ranks rin (layout from rin), pair stride sstride.
//   If in_place, the work is done directly on src (then rin must already
//   satisfy the economy-QR shape clamps and the output capacities equal rin);
//   else src is copied to a work buffer first.
//   out: capacity layout `cap`, pair stride ostride; orank: [batch][d+1].
struct RoundSpec {
  std::vector<int64_t> n, rin, cap;
  double *src;
  int64_t sstride;
  bool in_place;
  double *out;
  int64_t ostride;
  int64_t *orank;
  int64_t max_rank;
  std::vector<int64_t> bond_cap;  // optional [d+1]: per-bond cap (replaces max_rank)
  double tol;
  int batch;
  bool right_orth = false;  // cores 1..d-1 already have orthonormal rows: no right-to-left pass
  bool norm_only;     // stop after the right-to-left sweep and write ||B_1||
  double *norm_out;   // [batch] (norm_only)
};

std::vector<int64_t> round_caps(const std::vector<int64_t> &n, const std::vector<int64_t> &r) {
  const int d = (int)n.size();
  std::vector<int64_t> b(r);
  b[d] = 1;
  for (int k = d - 1; k >= 1; --k) b[k] = std::min(r[k], n[k] * b[k + 1]);
  std::vector<int64_t> c(b);
  c[0] = 1;
  for (int k = 1; k < d; ++k) c[k] = std::min(c[k], c[k - 1] * n[k - 1]);
  return c;
}

hatt_status round_body(bool run, const RoundSpec &sp, Ws &ws, GemmCtx &gc, hipStream_t st) {
  const int d = (int)sp.n.size();
  const int P = sp.batch;
  const auto &n = sp.n;
  std::vector<int64_t> soff;
  int64_t stot;
  make_offsets(n, sp.rin, &soff, &stot);
  // right-to-left ranks
  std::vector<int64_t> rb(sp.rin);
  if (!sp.right_orth)
    for (int c = d - 1; c >= 1; --c) rb[c] = std::min(sp.rin[c], n[c] * rb[c + 1]);
  const auto &cap = sp.cap;
  // --- sizes
  int64_t qr_ws = 1, qbuf = 1, rbuf = 1, ubuf = 1, sbuf = 1, tbuf = 1, tmp = 1, svd_ws = 1;
  int64_t lq_q = 1, lq_r = 1, lq_s = 1;
  std::vector<QrOp> op_rl(d), op_lr(d), op_lq(d);
  if (sp.right_orth) tmp = std::max(tmp, n[0] * rb[1]);  // the first core, copied for the left-to-right pass
  for (int c = d - 1; c >= 1 && !sp.right_orth; --c) {
    const int64_t m = n[c] * rb[c + 1], nc = sp.rin[c];
    if (!qr_prepare(m, nc, &op_rl[c]))
      return fail(HATT_EUNSUPPORTED, "TT-Rounding: a right-to-left QR of " + std::to_string(m) + " x " +
                                         std::to_string(nc) + " exceeds the library's QR limits");
    qr_ws = std::max(qr_ws, op_rl[c].ws_doubles);
    rbuf = std::max(rbuf, op_rl[c].k * nc);
    tmp = std::max(tmp, sp.rin[c - 1] * n[c - 1] * op_rl[c].k);
  }
  if (!sp.norm_only) {
    for (int c = 0; c < d - 1; ++c) {
      const int64_t m = cap[c] * n[c], nc = rb[c + 1];
      if (!qr_prepare(m, nc, &op_lr[c]))
        return fail(HATT_EUNSUPPORTED, "TT-Rounding: a left-to-right QR of " + std::to_string(m) + " x " +
                                           std::to_string(nc) + " exceeds the library's QR limits");
      const int64_t k = op_lr[c].k;
      if (k < nc) {
        // wide R (k x nc): its SVD through R^T = Q' R', the k x k factor R'^T
        if (!qr_prepare(nc, k, &op_lq[c]))
          return fail(HATT_EUNSUPPORTED, "TT-Rounding: the QR of a " + std::to_string(nc) + " x " +
                                             std::to_string(k) + " transposed R factor is not supported");
        qr_ws = std::max(qr_ws, op_lq[c].ws_doubles);
        lq_q = std::max(lq_q, nc * k);
        lq_r = std::max(lq_r, k * k);
        lq_s = std::max(lq_s, cap[c + 1] * k);
      }
      if (std::min(k, nc) > kSvdBigMaxN)
        return fail(HATT_EUNSUPPORTED, "TT-Rounding: bond rank " + std::to_string(nc) +
                                           " exceeds the library's SVD limit (" + std::to_string(kSvdBigMaxN) + ")");
      qr_ws = std::max(qr_ws, op_lr[c].ws_doubles);
      qbuf = std::max(qbuf, m * k);
      rbuf = std::max(rbuf, k * nc);
      ubuf = std::max(ubuf, k * cap[c + 1]);
      sbuf = std::max(sbuf, cap[c + 1] * nc);
      tbuf = std::max(tbuf, cap[c + 1] * n[c + 1] * rb[c + 2]);
      tmp = std::max(tmp, k * cap[c + 1]);  // R2^{-1} U of a deferred CholeskyQR2
      tmp = std::max(tmp, cap[c + 1] * nc);  // S V^T R2^{-T} of a deferred right-to-left QR
      svd_ws = std::max(svd_ws, svd_ws_doubles((int)k, (int)std::min(k, nc)));
    }
  }
  double *work = sp.in_place ? sp.src : ws.d((int64_t)P * stot);
  const int64_t wstride = sp.in_place ? sp.sstride : stot;
  double *wqr = ws.d((int64_t)P * qr_ws);
  double *Qb = ws.d((int64_t)P * qbuf);
  double *Rb = ws.d((int64_t)P * rbuf);
  double *Ub = ws.d((int64_t)P * ubuf);
  double *Sb = ws.d((int64_t)P * sbuf);
  double *T0 = ws.d((int64_t)P * tbuf);
  double *T1 = ws.d((int64_t)P * tbuf);
  double *Tm = ws.d((int64_t)P * tmp);
  // right-to-left cores 1..d-2 whose CholeskyQR2 left Q as Q1 (kept pairs):
  // their R2^{-1} (rin x rin) and the keep flag, per pair
  std::vector<int64_t> keep_off(d + 1, 0);
  int64_t keep_tot = 1;
  for (int c = 1; c <= d - 2; ++c) {
    keep_off[c] = keep_tot;
    keep_tot += sp.rin[c] * sp.rin[c] + 1;
  }
  double *keep = ws.d((int64_t)P * keep_tot);
  double *LqQ = ws.d((int64_t)P * lq_q);
  double *LqR = ws.d((int64_t)P * lq_r);
  double *LqL = ws.d((int64_t)P * lq_r);
  double *LqS = ws.d((int64_t)P * lq_s);
  std::vector<char> deferred(d + 1, 0);
  double *dl2 = ws.d(P);
  double *svdbig = ws.d((int64_t)P * svd_ws);
  int *flags = (int *)ws.d(P);

  if (!sp.in_place)
    LAUNCH(launch_copy(CMat{sp.src, stot, 1, sp.sstride}, Mat{work, stot, 1, stot}, 1, stot, P, st));
  if (d == 1) {
    if (sp.norm_only) {
      LAUNCH(launch_block_norm(work, stot, wstride, sp.norm_out, P, st));
    } else {
      LAUNCH(launch_copy(CMat{work, stot, 1, wstride}, Mat{sp.out, stot, 1, sp.ostride}, 1, stot, P, st));
      LAUNCH(launch_fill_i64(sp.orank, (int64_t)P * 2, 1, st));
    }
    return HATT_OK;
  }
  if (sp.right_orth)  // the left-to-right pass reads the first core from Tm
    LAUNCH(launch_copy(CMat{work + soff[0], n[0] * rb[1], 1, wstride}, Mat{Tm, n[0] * rb[1], 1, tmp}, 1,
                       n[0] * rb[1], P, st));
  // --- right-to-left orthogonalisation; core c layout: [*][n_c][rb_{c+1}] compact.
  // V(B_{c-1}) R^T lands in Tm in that same compact layout, and the next QR
  // reads it there (writing its Q into the core's slot), so no copy-back.
  for (int c = d - 1; c >= 1 && !sp.right_orth; --c) {
    const QrOp &op = op_rl[c];
    const int64_t m = n[c] * rb[c + 1], nc = sp.rin[c], k = op.k;
    double *core = work + soff[c];
    // H(B_c)^T is m x nc: element (j, a) = src[a * m + j]
    const CMat src = (c == d - 1) ? CMat{core, 1, m, wstride} : CMat{Tm, 1, m, tmp};
    // below the last core the QR is not in place: CholeskyQR2 may leave Q1 in
    // the core's slot and R2^{-1} aside (the left-to-right pass applies it)
    QrDeferred qd;
    qd.q1_in_q = true;
    hatt_status s = qr_exec(run, op, src, Mat{core, 1, m, wstride}, Mat{Rb, nc, 1, rbuf}, rbuf, wqr, qr_ws, P, gc,
                            st, (c < d - 1 && !sp.norm_only) ? &qd : nullptr);
    if (s != HATT_OK) return s;
    if (qd.used) {
      if (op.k != nc) return fail(HATT_EUNSUPPORTED, "internal: deferred QR with k != n");
      // R2^{-1} and the flag int right after it, as nc * nc + 1 doubles
      LAUNCH(launch_copy(CMat{qd.r2i, nc * nc + 1, 1, qd.wsp}, Mat{keep + keep_off[c], nc * nc + 1, 1, keep_tot}, 1,
                         nc * nc + 1, P, st));
      deferred[c] = 1;
    }
    // V(B_{c-1}) R^T, V(B_{c-1}) is (rin_{c-1} n_{c-1}) x nc with row stride nc
    const double *prev = work + soff[c - 1];
    const int64_t mp = sp.rin[c - 1] * n[c - 1];
    s = gemm(run, gc, CMat{prev, nc, 1, wstride}, CMat{Rb, 1, nc, rbuf}, Mat{Tm, k, 1, tmp}, mp, k, nc, 1.0,
             0.0, P, st, true);
    if (s != HATT_OK) return s;
  }
  // the orthogonalised first core lives in Tm (rin_0 = 1 row of n_0 rb_1 entries)
  if (sp.norm_only) {
    LAUNCH(launch_block_norm(Tm, n[0] * rb[1], tmp, sp.norm_out, P, st));
    return HATT_OK;
  }
  // --- left-to-right truncation
  LAUNCH(launch_fill_i64(sp.orank, (int64_t)P * (d + 1), 1, st));
  std::vector<int64_t> ooff;
  int64_t otot;
  make_offsets(n, cap, &ooff, &otot);
  const double tol2 = (sp.tol > 0.0) ? sp.tol * sp.tol / (double)(d - 1) : 0.0;
  double *Tcur = nullptr, *Tnext = T0;
  for (int c = 0; c < d - 1; ++c) {
    const QrOp &op = op_lr[c];
    const int64_t m = cap[c] * n[c], nc = rb[c + 1], k = op.k;
    CMat V = (c == 0) ? CMat{Tm, nc, 1, tmp} : CMat{Tcur, nc, 1, tbuf};
    // the output core needs Q only through Q U: CholeskyQR2 may leave it as Q1 R2^{-1}
    QrDeferred qd;
    hatt_status s =
        qr_exec(run, op, V, Mat{Qb, k, 1, qbuf}, Mat{Rb, nc, 1, rbuf}, rbuf, wqr, qr_ws, P, gc, st, &qd);
    if (s != HATT_OK) return s;
    SvdArgs sa{};
    sa.r = Rb;
    sa.rbs = rbuf;
    sa.kr = (int)k;
    sa.nc = (int)nc;
    sa.ucap = (int)cap[c + 1];
    sa.u = Ub;
    sa.ubs = ubuf;
    sa.svt = Sb;
    sa.sbs = sbuf;
    sa.batch = P;
    sa.delta2 = dl2;
    sa.first_bond = (c == 0);
    sa.tol2_over_dm1 = tol2;
    sa.cap = sp.bond_cap.empty() ? sp.max_rank : sp.bond_cap[c + 1];
    sa.prev_rank = (c == 0) ? nullptr : sp.orank + c;
    sa.n_mode = n[c];
    sa.rank_out = sp.orank + c + 1;
    sa.rank_bs = d + 1;
    if (k > nc) return fail(HATT_EUNSUPPORTED, "internal: QR rank exceeds columns");
    if (k < nc) {
      // R^T = Q' R' (nc x k); the singular values and left vectors of R are
      // those of L = R'^T (k x k); S V^T = U^T R
      s = qr_exec(run, op_lq[c], CMat{Rb, 1, nc, rbuf}, Mat{LqQ, k, 1, lq_q}, Mat{LqR, k, 1, lq_r}, lq_r, wqr, qr_ws,
                  P, gc, st);
      if (s != HATT_OK) return s;
      LAUNCH(launch_copy(CMat{LqR, 1, k, lq_r}, Mat{LqL, k, 1, lq_r}, k, k, P, st));
      SvdArgs sl = sa;
      sl.r = LqL;
      sl.rbs = lq_r;
      sl.nc = (int)k;
      sl.svt = LqS;
      sl.sbs = lq_s;
      s = svd_exec(run, sl, svdbig, svd_ws, flags, gc, st);
      if (s != HATT_OK) return s;
      s = gemm(run, gc, CMat{Ub, 1, cap[c + 1], ubuf}, CMat{Rb, nc, 1, rbuf}, Mat{Sb, nc, 1, sbuf}, cap[c + 1], nc, k,
               1.0, 0.0, P, st, true);
    } else {
      s = svd_exec(run, sa, svdbig, svd_ws, flags, gc, st);
    }
    if (s != HATT_OK) return s;
    // out core c = Q U  (m x cap_{c+1})
    const Mat oc{sp.out + ooff[c], cap[c + 1], 1, sp.ostride};
    if (qd.used) {
      // kept pairs: Q1 (R2^{-1} U); pairs the fallback recomputed: Q U
      s = gemm(run, gc, CMat{qd.r2i, k, 1, qd.wsp}, CMat{Ub, cap[c + 1], 1, ubuf}, Mat{Tm, cap[c + 1], 1, tmp},
               k, cap[c + 1], k, 1.0, 0.0, P, st, false, qd.flag, qd.fst, nullptr, GemmTypes{}, 1);
      if (s != HATT_OK) return s;
      s = gemm(run, gc, CMat{qd.q1, k, 1, qd.wsp}, CMat{Tm, cap[c + 1], 1, tmp}, oc, m, cap[c + 1], k, 1.0, 0.0,
               P, st, true, qd.flag, qd.fst, nullptr, GemmTypes{}, 1);
      if (s != HATT_OK) return s;
      s = gemm(run, gc, CMat{Qb, k, 1, qbuf}, CMat{Ub, cap[c + 1], 1, ubuf}, oc, m, cap[c + 1], k, 1.0, 0.0, P,
               st, true, qd.flag, qd.fst, nullptr, GemmTypes{}, 0);
    } else {
      s = gemm(run, gc, CMat{Qb, k, 1, qbuf}, CMat{Ub, cap[c + 1], 1, ubuf}, oc, m, cap[c + 1], k, 1.0, 0.0, P,
               st, true);
    }
    if (s != HATT_OK) return s;
    // next core = SVt H(B_{c+1}):  (cap_{c+1} x nc) (nc x n_{c+1} rb_{c+2})
    const int64_t ncol = n[c + 1] * rb[c + 2];
    const CMat hnext{work + soff[c + 1], ncol, 1, wstride};
    const Mat tn{Tnext, ncol, 1, tbuf};
    if (deferred[c + 1]) {
      // the slot holds Q1^T for the kept pairs (H = R2^{-T} Q1^T): (SVt R2^{-T}) Q1^T
      const double *r2k = keep + keep_off[c + 1];
      const int *kf = reinterpret_cast<const int *>(r2k + nc * nc);
      const int64_t kfs = 2 * keep_tot;
      s = gemm(run, gc, CMat{Sb, nc, 1, sbuf}, CMat{r2k, 1, nc, keep_tot}, Mat{Tm, nc, 1, tmp}, cap[c + 1], nc, nc,
               1.0, 0.0, P, st, false, kf, kfs, nullptr, GemmTypes{}, 1);
      if (s != HATT_OK) return s;
      s = gemm(run, gc, CMat{Tm, nc, 1, tmp}, hnext, tn, cap[c + 1], ncol, nc, 1.0, 0.0, P, st, true, kf, kfs,
               nullptr, GemmTypes{}, 1);
      if (s != HATT_OK) return s;
      s = gemm(run, gc, CMat{Sb, nc, 1, sbuf}, hnext, tn, cap[c + 1], ncol, nc, 1.0, 0.0, P, st, true, kf, kfs,
               nullptr, GemmTypes{}, 0);
    } else {
      s = gemm(run, gc, CMat{Sb, nc, 1, sbuf}, hnext, tn, cap[c + 1], ncol, nc, 1.0, 0.0, P, st, true);
    }
    if (s != HATT_OK) return s;
    Tcur = Tnext;
    Tnext = (Tnext == T0) ? T1 : T0;
  }
  // last core
  LAUNCH(launch_copy(CMat{Tcur, 1, 1, tbuf}, Mat{sp.out + ooff[d - 1], 1, 1, sp.ostride}, 1,
                     cap[d - 1] * n[d - 1], P, st));
  return HATT_OK;
}

// Measures the split-K partial buffer with a dry pass, reserves it at the
// front of this call's workspace share, then runs (or measures) the body.
hatt_status round_run(bool run, const RoundSpec &sp, Ws &ws, GemmCtx &, hipStream_t st) {
  Ws probe(nullptr);
  GemmCtx g0{nullptr, 0, 0};
  hatt_status s = round_body(false, sp, probe, g0, st);
  if (s != HATT_OK) return s;
  GemmCtx g1{nullptr, 0, 0};
  g1.part = ws.d(std::max<int64_t>(g0.part_need, 1));
  g1.part_cap = g0.part_need;
  return round_body(run, sp, ws, g1, st);
}

// Truncation of a left-orthogonal train (cores 0..d-2 with orthonormal
// columns in V(.), as Alg. 4 and Alg. 2 leave them) in place at capacity
// ranks l: Alg. 1's truncation loop run from the right.  The train is
// reversed into scratch (a reversed left-orthogonal train is right-orthogonal,
// which is what Alg. 1's first pass would produce), truncated left to right
// there without that pass, and reversed back with its kept ranks.
hatt_status truncate_left_orth(bool run, const std::vector<int64_t> &n, const std::vector<int64_t> &l,
                               double *out, int64_t ostride, int64_t *orank, const std::vector<int64_t> &bond_cap,
                               double tol, int P, Ws &ws, hipStream_t st) {
  const int d = (int)n.size();
  if (d > kRevMaxCores)
    return fail(HATT_EUNSUPPORTED, "truncation: order above " + std::to_string(kRevMaxCores) + " is not built");
  std::vector<int64_t> ooff, roff, nr(d), lr(d + 1), cr(d + 1, 0);
  int64_t otot, rtot;
  make_offsets(n, l, &ooff, &otot);
  for (int k = 0; k < d; ++k) nr[k] = n[d - 1 - k];
  for (int k = 0; k <= d; ++k) {
    lr[k] = l[d - k];
    if (!bond_cap.empty()) cr[k] = bond_cap[d - k];
  }
  make_offsets(nr, lr, &roff, &rtot);
  double *rev = ws.d((int64_t)P * rtot);
  int64_t *rrank = ws.i64((int64_t)P * (d + 1));
  RevArgs fwd{}, bwd{};
  fwd.src = out;
  fwd.dst = rev;
  fwd.sstride = ostride;
  fwd.dstride = rtot;
  fwd.d = d;
  bwd.src = rev;
  bwd.dst = out;
  bwd.sstride = rtot;
  bwd.dstride = ostride;
  bwd.d = d;
  int64_t mx = 1;
  for (int k = 0; k < d; ++k) {
    fwd.soff[k] = ooff[k];
    fwd.doff[k] = roff[d - 1 - k];
    fwd.r0[k] = (int)l[k];
    fwd.n[k] = (int)n[k];
    fwd.r1[k] = (int)l[k + 1];
    bwd.soff[k] = roff[k];
    bwd.doff[k] = ooff[d - 1 - k];
    bwd.r0[k] = (int)lr[k];
    bwd.n[k] = (int)nr[k];
    bwd.r1[k] = (int)lr[k + 1];
    mx = std::max(mx, ((l[k] + 31) / 32) * ((l[k + 1] + 31) / 32) * n[k]);
  }
  LAUNCH(launch_tt_reverse(fwd, mx, P, st));
  RoundSpec rs{};
  rs.n = nr;
  rs.rin = lr;
  rs.cap = lr;
  rs.src = rev;
  rs.sstride = rtot;
  rs.in_place = true;
  rs.out = rev;
  rs.ostride = rtot;
  rs.orank = rrank;
  rs.max_rank = 0;
  rs.bond_cap = cr;
  rs.tol = tol;
  rs.batch = P;
  rs.right_orth = true;
  GemmCtx gr{nullptr, 0, 0};
  hatt_status s = round_run(run, rs, ws, gr, st);
  if (s != HATT_OK) return s;
  LAUNCH(launch_tt_reverse(bwd, mx, P, st));
  LAUNCH(launch_rank_reverse(rrank, orank, d, P, st));
  return HATT_OK;
}

// ---------------------------------------------------------------------------
struct HattSpec {
  Shape X, Y;
  Shape W;                        // third factor (three = true)
  bool three = false;
  std::vector<int64_t> ryw;       // rank of the trailing factors per bond: s_k, or s_k t_k
  std::vector<int64_t> ell;
  std::vector<int64_t> bond_cap;  // [d+1] truncation cap per bond (0: none)
  const double *sketch;  // explicit sketch data or nullptr
  int64_t sketch_stride;
  hatt_opts o;
  double *out;
  int64_t ostride;
  int64_t *orank;
  double *xnorm = nullptr;  // optional device [batch]: ||X|| of the untruncated HaTT output
};

hatt_status hatt3_body(bool run, const HattSpec &sp, Ws &ws, GemmCtx &gc, hipStream_t st);

hatt_status hatt_body(bool run, const HattSpec &sp, Ws &ws, GemmCtx &gc, hipStream_t st) {
  if (sp.three) return hatt3_body(run, sp, ws, gc, st);
  const int d = sp.X.d, P = sp.X.batch;
  const auto &n = sp.X.n, &r = sp.X.r, &s = sp.Y.r, &l = sp.ell;
  std::vector<int64_t> ooff, skoff;
  int64_t otot, sktot;
  make_offsets(n, l, &ooff, &otot);
  make_offsets(n, l, &skoff, &sktot);
  const double *xd = sp.X.data, *yd = sp.Y.data;
  const int64_t xs = sp.X.stride, ys = sp.Y.stride;

  // ---- sizes
  std::vector<int64_t> woff(d + 1, 0);
  int64_t wtot = 0;
  for (int b = 1; b < d; ++b) {
    woff[b] = wtot;
    wtot += r[b] * s[b] * l[b];
  }
  int64_t wlsz = 1, xsz = 1, ysz = 1, msz = 1, qrws = 1;
  std::vector<QrOp> qp(d);
  for (int c = 1; c <= d - 2; ++c) wlsz = std::max(wlsz, r[c] * s[c] * n[c] * l[c + 1]);
  for (int c = 0; c < d; ++c) xsz = std::max(xsz, l[c] * n[c] * r[c + 1] * s[c + 1]);
  for (int c = 0; c < d - 1; ++c) {
    ysz = std::max(ysz, l[c] * n[c] * l[c + 1]);
    msz = std::max(msz, l[c + 1] * r[c + 1] * s[c + 1]);
    if (!qr_prepare(l[c] * n[c], l[c + 1], &qp[c]))
      return fail(HATT_EUNSUPPORTED, "HaTT: the QR of a " + std::to_string(l[c] * n[c]) + " x " +
                                         std::to_string(l[c + 1]) + " sketched frame is not supported");
    qrws = std::max(qrws, qp[c].ws_doubles);
  }
  // HaTT-2: per HPCRL bond, QR + SVD of W^{(k)} (r s x l), U (r s x l), W_R (l' n x l)
  const bool v2 = (sp.o.variant == 2);
  std::vector<QrOp> qw(d);
  int64_t h2_q = 1, h2_r = 1, h2_wr = 1, h2_svd = 1;
  if (v2) {
    for (int c = d - 2; c >= 1; --c) {
      const int64_t rs1 = r[c + 1] * s[c + 1], l1 = l[c + 1];
      if (!qr_prepare(rs1, l1, &qw[c]))
        return fail(HATT_EUNSUPPORTED, "HaTT-2: QR of a sketch matrix is not supported at this size");
      qrws = std::max(qrws, qw[c].ws_doubles);
      h2_q = std::max(h2_q, rs1 * l1);
      h2_r = std::max(h2_r, l1 * l1);
      h2_wr = std::max(h2_wr, l[c] * n[c] * l1);
      h2_svd = std::max(h2_svd, svd_ws_doubles((int)l1, (int)l1));
    }
  }
  double *sk = nullptr;
  int64_t sks = 0;
  if (sp.sketch) {
    sk = (double *)sp.sketch;
    sks = sp.sketch_stride;
  } else {
    sk = ws.d(sktot);
    sks = 0;
  }
  // FP32 range finding keeps W^{(k)} and W_L as FP32 inside the same buffers
  // (BF16 range finding keeps the same FP32 storage; only the sandwich and
  // W_L W_R^T products round their operands to BF16 on the matrix cores)
  const bool f32 = (sp.o.precision != 0);
  double *W = ws.d((int64_t)P * std::max<int64_t>(wtot, 1));
  double *WL = ws.d((int64_t)P * wlsz);
  float *Wf = reinterpret_cast<float *>(W), *WLf = reinterpret_cast<float *>(WL);
  auto as_d = [](float *p) { return reinterpret_cast<double *>(static_cast<void *>(p)); };
  const int64_t lastsz = (d >= 2) ? std::max<int64_t>(r[d - 1] * s[d - 1] * l[d - 1], 1) : 1;
  double *Wlast = (f32 && d >= 2) ? ws.d((int64_t)P * lastsz) : nullptr;
  // FP32 range finding: each W^{(k)} is widened to FP64 for the sketched
  // frame X^{(k)} W^{(k)}, which then lies in range(X^{(k)}) to FP64 accuracy
  int64_t wdsz = 1;
  for (int b = 1; b < d; ++b) wdsz = std::max(wdsz, r[b] * s[b] * l[b]);
  double *Wd = f32 ? ws.d((int64_t)P * wdsz) : nullptr;
  double *Hlast = (d >= 2) ? ws.d((int64_t)P * r[d - 1] * s[d - 1] * n[d - 1]) : nullptr;
  double *Xc = ws.d((int64_t)P * xsz);
  double *Yb = ws.d((int64_t)P * ysz);
  double *Mb = ws.d((int64_t)P * msz);
  double *wqr = ws.d((int64_t)P * qrws);
  double *h2Q = v2 ? ws.d((int64_t)P * h2_q) : nullptr;   // Q of W, then U = Q U_R
  double *h2U = v2 ? ws.d((int64_t)P * h2_q) : nullptr;
  double *h2R = v2 ? ws.d((int64_t)P * h2_r) : nullptr;   // R of W
  double *h2Ur = v2 ? ws.d((int64_t)P * h2_r) : nullptr;  // U of R (zero beyond the kept terms)
  double *h2S = v2 ? ws.d((int64_t)P * h2_r) : nullptr;   // S V^T rows
  double *h2WR = v2 ? ws.d((int64_t)P * h2_wr) : nullptr;
  double *h2big = v2 ? ws.d((int64_t)P * h2_svd) : nullptr;
  double *h2misc = v2 ? ws.d((int64_t)P * 3) : nullptr;    // [delta2 | SVD flags | kept terms] x P
  if (d == 1) {
    LAUNCH(launch_fill_i64(sp.orank, (int64_t)P * 2, 1, st));
    PkpArgs pa{xd, yd, sp.out, 1, 1, 1, 1, n[0], xs, ys, sp.ostride, P};
    LAUNCH(launch_pkp(pa, st));
    return HATT_OK;
  }
  if (!sp.sketch) {
    for (int k = 0; k < d; ++k) {
      const int64_t cnt = l[k] * n[k] * l[k + 1];
      LAUNCH(launch_sketch_fill(sp.o.seed, k, cnt, 1.0 / sqrt((double)cnt), sk + skoff[k], st));
    }
  }
  // ---- HPCRL (Alg. 3), HaTT-1 split
  {
    // W^{(d-1)} = H(Y_d (x)^1 Z_d) H(R_d)^T: the product's last-core rows
    // (rank r s, one mode index each: the PKP of two rank-1-on-the-right
    // cores, r s n entries) times the sketch's last core on the matrix cores
    ClassScope cs(P_LAST);
    const int64_t rs = r[d - 1] * s[d - 1];
    PkpArgs pl{xd + sp.X.off[d - 1], yd + sp.Y.off[d - 1], Hlast, r[d - 1], 1, s[d - 1], 1, n[d - 1], xs, ys,
               rs * n[d - 1], P};
    LAUNCH(launch_pkp(pl, st));
    hatt_status sl = gemm(run, gc, CMat{Hlast, n[d - 1], 1, rs * n[d - 1]}, CMat{sk + skoff[d - 1], 1, n[d - 1], sks},
                          Mat{f32 ? Wlast : W + woff[d - 1], l[d - 1], 1, f32 ? lastsz : wtot}, rs, l[d - 1],
                          n[d - 1], 1.0, 0.0, P, st, true);
    if (sl != HATT_OK) return sl;
    if (f32) {
      // FP32 keeps 8 exponent bits: each W^{(k)} is brought back to unit scale
      // by a power of two (range(X W) is unchanged by any rescaling of W)
      const int64_t cnt = r[d - 1] * s[d - 1] * l[d - 1];
      LAUNCH(launch_cast_f32(Wlast, lastsz, Wf + woff[d - 1], wtot, cnt, P, st));
      LAUNCH(launch_rescale_pow2(Wf + woff[d - 1], cnt, wtot, P, st));
    }
  }
  for (int c = d - 2; c >= 1; --c) {
    const int64_t rs1 = r[c + 1] * s[c + 1], l1 = l[c + 1];
    const double *ucol = W + woff[c + 1];  // U operand: W itself (HaTT-1) or U_R (HaTT-2)
    int64_t ucb = wtot;
    if (v2) {
      // eq. HPCRL--2: W = Q R, R = U_R S V^T, keep sigma > ep sigma_1
      hatt_status s2 = qr_exec(run, qw[c], CMat{W + woff[c + 1], l1, 1, wtot}, Mat{h2Q, l1, 1, h2_q},
                               Mat{h2R, l1, 1, h2_r}, h2_r, wqr, qrws, P, gc, st);
      if (s2 != HATT_OK) return s2;
      SvdArgs sa{};
      sa.r = h2R;
      sa.rbs = h2_r;
      sa.kr = (int)l1;
      sa.nc = (int)l1;
      sa.ucap = (int)l1;
      sa.u = h2Ur;
      sa.ubs = h2_r;
      sa.svt = h2S;
      sa.sbs = h2_r;
      sa.batch = P;
      sa.delta2 = h2misc;
      sa.first_bond = 0;
      sa.tol2_over_dm1 = 0.0;
      sa.cap = 0;
      sa.prev_rank = nullptr;
      sa.n_mode = 1;
      sa.rank_out = (int64_t *)(h2misc + 2 * P);
      sa.rank_bs = 1;
      sa.rel_keep = std::max(sp.o.ep, 1e-300);
      s2 = svd_exec(run, sa, h2big, h2_svd, (int *)(h2misc + P), gc, st);
      if (s2 != HATT_OK) return s2;
      s2 = gemm(run, gc, CMat{h2Q, l1, 1, h2_q}, CMat{h2Ur, l1, 1, h2_r}, Mat{h2U, l1, 1, h2_q}, rs1, l1, l1,
                1.0, 0.0, P, st, true);
      if (s2 != HATT_OK) return s2;
      // W_R(g', (i, gamma)) = R_k(i) (sigma V)(:, gamma): V(R_k) (S V^T)^T
      s2 = gemm(run, gc, CMat{sk + skoff[c], l1, 1, sks}, CMat{h2S, 1, l1, h2_r}, Mat{h2WR, l1, 1, h2_wr},
                l[c] * n[c], l1, l1, 1.0, 0.0, P, st, true);
      if (s2 != HATT_OK) return s2;
      ucol = h2U;
      ucb = h2_q;
    }
    SandwichArgs a{};
    a.prec = sp.o.precision;
    a.yl = xd + sp.X.off[c];
    a.ylb = xs;
    a.yli = r[c + 1];
    a.ylr = n[c] * r[c + 1];
    a.ylc = 1;
    a.zr = yd + sp.Y.off[c];
    a.zrb = ys;
    a.zri = s[c + 1];
    a.zrr = 1;
    a.zrc = n[c] * s[c + 1];
    a.c = f32 ? as_d(Wf + woff[c + 1]) : ucol;
    a.cb = ucb;
    a.cg = 1;
    a.ca = s[c + 1] * l1;
    a.cbb = l1;
    // W_L column-major (rows (a', b') fastest): each (i, gamma) column is one
    // contiguous block of r s entries, so the sandwich writes whole blocks
    a.o = f32 ? as_d(WLf) : WL;
    a.ob = wlsz;
    a.oi = l1 * r[c] * s[c];
    a.og = r[c] * s[c];
    a.oa = s[c];
    a.obb = 1;
    a.RA = (int)r[c];
    a.RI = (int)r[c + 1];
    a.SI = (int)s[c + 1];
    a.SO = (int)s[c];
    a.n = n[c];
    a.G = l1;
    a.batch = P;
    if (f32) {
      SwPlan swp;
      if (!sandwich_mfma_plan(a, kSandwichLdsDoubles, &swp))
        return fail(HATT_EUNSUPPORTED, "low-precision range finding: no matrix-core sandwich plan for these ranks "
                                       "(use FP64)");
    }
    if (!sandwich_supported(a))
      return fail(HATT_EUNSUPPORTED, "HaTT: no sandwich kernel for the W_L build at core " + std::to_string(c) +
                                         " (ranks " + std::to_string(a.RA) + ", " + std::to_string(a.RI) + " of x, " +
                                         std::to_string(a.SO) + ", " + std::to_string(a.SI) + " of y)");
    SwForce sf;
    const bool tuned = sandwich_tune(run, a, st, &sf);
    site("sandwich W_L n=%lld G=%lld RA=%d RI=%d SI=%d SO=%d [%s]", (long long)n[c], (long long)l1, a.RA, a.RI,
         a.SI, a.SO, sandwich_kernel_name(a, tuned ? &sf : nullptr));
    LAUNCH(launch_sandwich(a, st, tuned ? &sf : nullptr));
    const int64_t K = n[c] * l1;
    const CMat wr = v2 ? CMat{h2WR, 1, K, h2_wr} : CMat{sk + skoff[c], 1, K, sks};
    hatt_status stt;
    if (f32) {
      GemmTypes ty;
      ty.prec = sp.o.precision;
      ty.a32 = 1;
      ty.c32 = 1;
      stt = gemm(run, gc, CMat{as_d(WLf), 1, r[c] * s[c], wlsz}, wr, Mat{as_d(Wf + woff[c]), l[c], 1, wtot}, r[c] * s[c],
                 l[c], K, 1.0, 0.0, P, st, true, nullptr, 0, nullptr, ty);
      if (stt == HATT_OK) LAUNCH(launch_rescale_pow2(Wf + woff[c], r[c] * s[c] * l[c], wtot, P, st));
    } else {
      stt = gemm(run, gc, CMat{WL, 1, r[c] * s[c], wlsz}, wr, Mat{W + woff[c], l[c], 1, wtot}, r[c] * s[c], l[c], K, 1.0,
                 0.0, P, st, true);
    }
    if (stt != HATT_OK) return stt;
  }
  // ---- sweep (Alg. 4)
  {
    PkpArgs pa{xd, yd, Xc, 1, r[1], 1, s[1], n[0], xs, ys, xsz, P};
    LAUNCH(launch_pkp(pa, st));
  }
  for (int c = 0; c < d - 1; ++c) {
    const int64_t m = l[c] * n[c], rs1 = r[c + 1] * s[c + 1];
    hatt_status stt;
    if (f32) {
      // the sketch found in FP32 is just another sketch: the frame product
      // itself runs in FP64, so the frame's range stays inside range(X^{(k)})
      LAUNCH(launch_cast_f64(Wf + woff[c + 1], wtot, Wd, wdsz, rs1 * l[c + 1], P, st));
      stt = gemm(run, gc, CMat{Xc, rs1, 1, xsz}, CMat{Wd, l[c + 1], 1, wdsz}, Mat{Yb, l[c + 1], 1, ysz}, m,
                 l[c + 1], rs1, 1.0, 0.0, P, st, true);
    } else {
      stt = gemm(run, gc, CMat{Xc, rs1, 1, xsz}, CMat{W + woff[c + 1], l[c + 1], 1, wtot},
                 Mat{Yb, l[c + 1], 1, ysz}, m, l[c + 1], rs1, 1.0, 0.0, P, st, true);
    }
    if (stt != HATT_OK) return stt;
    double *qcore = sp.out + ooff[c];
    stt = qr_exec(run, qp[c], CMat{Yb, l[c + 1], 1, ysz}, Mat{qcore, l[c + 1], 1, sp.ostride},
                  Mat{nullptr, 0, 0, 0}, 0, wqr, qrws, P, gc, st);
    if (stt != HATT_OK) return stt;
    stt = gemm(run, gc, CMat{qcore, 1, l[c + 1], sp.ostride}, CMat{Xc, rs1, 1, xsz}, Mat{Mb, rs1, 1, msz},
               l[c + 1], rs1, m, 1.0, 0.0, P, st, true);
    if (stt != HATT_OK) return stt;
    const int cn = c + 1;
    if (cn == d - 1) {
      // last core (right ranks 1): X_d(g, i) = sum_{a,b} M(g, a s + b) Y_d(a, i) Z_d(b, i)
      // = (M H)(g, i) with H the last-core PKP rows HPCRL formed
      hatt_status sg = gemm(run, gc, CMat{Mb, rs1, 1, msz}, CMat{Hlast, n[cn], 1, rs1 * n[cn]},
                            Mat{sp.out + ooff[cn], n[cn], 1, sp.ostride}, l[cn], n[cn], rs1, 1.0, 0.0, P, st, true);
      if (sg != HATT_OK) return sg;
      continue;
    }
    SandwichArgs a{};
    a.yl = xd + sp.X.off[cn];
    a.ylb = xs;
    a.yli = r[cn + 1];
    a.ylr = 1;
    a.ylc = n[cn] * r[cn + 1];
    a.zr = yd + sp.Y.off[cn];
    a.zrb = ys;
    a.zri = s[cn + 1];
    a.zrr = n[cn] * s[cn + 1];
    a.zrc = 1;
    a.c = Mb;
    a.cb = msz;
    a.cg = rs1;
    a.ca = s[cn];
    a.cbb = 1;
    if (cn < d - 1) {
      a.o = Xc;
      a.ob = xsz;
      a.oi = r[cn + 1] * s[cn + 1];
      a.og = n[cn] * r[cn + 1] * s[cn + 1];
      a.oa = s[cn + 1];
      a.obb = 1;
    } else {
      a.o = sp.out + ooff[cn];
      a.ob = sp.ostride;
      a.oi = 1;
      a.og = n[cn];
      a.oa = 1;
      a.obb = 1;
    }
    a.RA = (int)r[cn + 1];
    a.RI = (int)r[cn];
    a.SI = (int)s[cn];
    a.SO = (int)s[cn + 1];
    a.n = n[cn];
    a.G = l[cn];
    a.batch = P;
    if (!sandwich_supported(a))
      return fail(HATT_EUNSUPPORTED, "HaTT: no sandwich kernel for the core update at core " + std::to_string(cn) +
                                         " (ranks " + std::to_string(a.RI) + ", " + std::to_string(a.RA) + " of x, " +
                                         std::to_string(a.SI) + ", " + std::to_string(a.SO) + " of y)");
    SwForce sf;
    const bool tuned = sandwich_tune(run, a, st, &sf);
    site("sandwich update n=%lld G=%lld RA=%d RI=%d SI=%d SO=%d [%s]", (long long)n[cn], (long long)l[cn], a.RA,
         a.RI, a.SI, a.SO, sandwich_kernel_name(a, tuned ? &sf : nullptr));
    LAUNCH(launch_sandwich(a, st, tuned ? &sf : nullptr));
  }
  // ranks before truncation: the sketch widths
  if ((int)l.size() > kMaxRankPattern) return fail(HATT_EUNSUPPORTED, "order too large for the library (rank pattern buffer)");
  LAUNCH(launch_rank_pattern(sp.orank, P, d + 1, l.data(), st));
  // ||X|| of the untruncated result: every core but the last is orthonormal
  if (sp.xnorm != nullptr && d >= 2)
    LAUNCH(launch_block_norm(sp.out + ooff[d - 1], l[d - 1] * n[d - 1], sp.ostride, sp.xnorm, P, st));
  // ---- truncation (Alg. 1 on the rank-l result)
  bool capped = false;
  for (int64_t c : sp.bond_cap) capped = capped || c > 0;
  const bool trunc = capped || (sp.o.tol > 0.0);
  if (trunc && d >= 2) {
    // every output core but the last is the Q of a QR: left-orthogonal
    hatt_status s1 = truncate_left_orth(run, n, l, sp.out, sp.ostride, sp.orank, sp.bond_cap, sp.o.tol, P, ws, st);
    if (s1 != HATT_OK) return s1;
  }
  return HATT_OK;
}

// ---------------------------------------------------------------------------
// Three factors, z = x (.) y (.) w: one triple per call, FP64, HaTT-1.  The
// Kronecker-times-vector identity behind eq. WLWR and eq. M*core0, taken
// over three factors, turns HPCRL's recursion and the sweep's core update
// into three-mode products.  Each mode product is one GEMM batched over the
// mode index i that contracts the tensor's leading rank index and appends
// the new index last (a cyclic rotation of the index order), so the
// products chain without a permutation pass:
//   HPCRL, bond k+1 -> k:  V_i = W^{(k+1)} R_k(i)^T, then
//     V[i][a'][b'][c'][g] -> T1[i][b'][c'][g][a] -> T2[i][c'][g][a][b]
//     -> W^{(k)}[g][a][b][c]  (the last product also sums over i: K = (i, c'))
//   core update, M = Q^T X^{(k)} stored as [a][b][c][g]:
//     M -> U1[i][b][c][g][a'] -> U2[i][c][g][a'][b'] -> X^{(k+1)}[i][g][a'][b'][c']
// W^{(k)} is column-major (rows (a, b, c), a slowest).  The sketched frame
// X^{(k)} W^{(k)} is a GEMM per i whose rows g land on rows (g, i) of the
// frame (the output core's order), and M = sum_i Q_i^T X_i reduces per-i
// products in a fixed order.
hatt_status hatt3_body(bool run, const HattSpec &sp, Ws &ws, GemmCtx &gc, hipStream_t st) {
  const int d = sp.X.d;
  const auto &n = sp.X.n, &r = sp.X.r, &s = sp.Y.r, &t = sp.W.r, &l = sp.ell;
  std::vector<int64_t> ooff, skoff;
  int64_t otot, sktot;
  make_offsets(n, l, &ooff, &otot);
  make_offsets(n, l, &skoff, &sktot);
  const double *xd = sp.X.data, *yd = sp.Y.data, *wd = sp.W.data;
  std::vector<int64_t> rst(d + 1);
  for (int b = 0; b <= d; ++b) rst[b] = r[b] * s[b] * t[b];
  std::vector<int64_t> woff(d + 1, 0);
  int64_t wtot = 0;
  for (int b = 1; b < d; ++b) {
    woff[b] = wtot;
    wtot += rst[b] * l[b];
  }
  int64_t vsz = 1, t1sz = 1, t2sz = 1, u1sz = 1, u2sz = 1;
  for (int c = 1; c <= d - 2; ++c) {
    vsz = std::max(vsz, n[c] * rst[c + 1] * l[c]);
    t1sz = std::max(t1sz, n[c] * s[c + 1] * t[c + 1] * l[c] * r[c]);
    t2sz = std::max(t2sz, n[c] * t[c + 1] * l[c] * r[c] * s[c]);
    u1sz = std::max(u1sz, n[c] * s[c] * t[c] * l[c] * r[c + 1]);
    u2sz = std::max(u2sz, n[c] * t[c] * l[c] * r[c + 1] * s[c + 1]);
  }
  int64_t xsz = 1, ysz = 1, msz = 1, mpsz = 1, qrws = 1;
  std::vector<QrOp> qp(d);
  for (int c = 0; c < d - 1; ++c) {
    xsz = std::max(xsz, n[c] * l[c] * rst[c + 1]);
    ysz = std::max(ysz, l[c] * n[c] * l[c + 1]);
    msz = std::max(msz, l[c + 1] * rst[c + 1]);
    if (n[c] > 1) mpsz = std::max(mpsz, n[c] * l[c + 1] * rst[c + 1]);
    if (!qr_prepare(l[c] * n[c], l[c + 1], &qp[c]))
      return fail(HATT_EUNSUPPORTED, "HaTT (three factors): the QR of a " + std::to_string(l[c] * n[c]) + " x " +
                                         std::to_string(l[c + 1]) + " sketched frame is not supported");
    qrws = std::max(qrws, qp[c].ws_doubles);
  }
  const int64_t ptsz = std::max<int64_t>(r[d - 1] * s[d - 1] * n[d - 1], r[1] * s[1] * n[0]);
  double *sk = nullptr;
  if (sp.sketch) {
    sk = (double *)sp.sketch;
  } else {
    sk = ws.d(sktot);
  }
  double *W = ws.d(std::max<int64_t>(wtot, 1));
  double *Vb = ws.d(vsz), *T1b = ws.d(t1sz), *T2b = ws.d(t2sz);
  double *U1 = ws.d(u1sz), *U2 = ws.d(u2sz);
  double *Hlast = ws.d(rst[d - 1] * n[d - 1]);
  double *ptmp = ws.d(ptsz);
  double *Xc = ws.d(xsz), *Yb = ws.d(ysz), *Mb = ws.d(msz), *Mp = ws.d(mpsz);
  double *wqr = ws.d(qrws);
  if (d == 1) {
    LAUNCH(launch_fill_i64(sp.orank, 2, 1, st));
    PkpArgs p1{xd, yd, ptmp, 1, 1, 1, 1, n[0], 0, 0, 0, 1};
    LAUNCH(launch_pkp(p1, st));
    PkpArgs p2{ptmp, wd, sp.out, 1, 1, 1, 1, n[0], 0, 0, 0, 1};
    LAUNCH(launch_pkp(p2, st));
    return HATT_OK;
  }
  if (!sp.sketch) {
    for (int k = 0; k < d; ++k) {
      const int64_t cnt = l[k] * n[k] * l[k + 1];
      LAUNCH(launch_sketch_fill(sp.o.seed, k, cnt, 1.0 / sqrt((double)cnt), sk + skoff[k], st));
    }
  }
  hatt_status stt;
  // ---- HPCRL (Alg. 3), HaTT-1 split
  {
    // W^{(d-1)}: rows (a, b, c) of the right-rank-1 last cores times the
    // sketch's last core
    ClassScope cs(P_LAST);
    const int c = d - 1;
    PkpArgs p1{xd + sp.X.off[c], yd + sp.Y.off[c], ptmp, r[c], 1, s[c], 1, n[c], 0, 0, 0, 1};
    LAUNCH(launch_pkp(p1, st));
    PkpArgs p2{ptmp, wd + sp.W.off[c], Hlast, r[c] * s[c], 1, t[c], 1, n[c], 0, 0, 0, 1};
    LAUNCH(launch_pkp(p2, st));
    stt = gemm(run, gc, CMat{Hlast, n[c], 1, 0}, CMat{sk + skoff[c], 1, n[c], 0}, Mat{W + woff[c], 1, rst[c], 0},
               rst[c], l[c], n[c], 1.0, 0.0, 1, st, true);
    if (stt != HATT_OK) return stt;
  }
  for (int c = d - 2; c >= 1; --c) {
    const int64_t nn = n[c], l0 = l[c], l1 = l[c + 1];
    const int64_t r0 = r[c], s0 = s[c], t0 = t[c], r1 = r[c + 1], s1 = s[c + 1], t1 = t[c + 1];
    const int64_t K1 = rst[c + 1];
    // V_i = W^{(k+1)} R_k(i)^T
    stt = gemm(run, gc, CMat{W + woff[c + 1], 1, K1, 0}, CMat{sk + skoff[c], 1, nn * l1, l1},
               Mat{Vb, l0, 1, K1 * l0}, K1, l0, l1, 1.0, 0.0, (int)nn, st, true);
    if (stt != HATT_OK) return stt;
    // T1_i[(b' c' g), a] = sum_a' V_i[a', (b' c' g)] X_k(a, i, a')
    stt = gemm(run, gc, CMat{Vb, 1, s1 * t1 * l0, K1 * l0}, CMat{xd + sp.X.off[c], 1, nn * r1, r1},
               Mat{T1b, r0, 1, s1 * t1 * l0 * r0}, s1 * t1 * l0, r0, r1, 1.0, 0.0, (int)nn, st, true);
    if (stt != HATT_OK) return stt;
    // T2_i[(c' g a), b] = sum_b' T1_i[b', (c' g a)] Y_k(b, i, b')
    stt = gemm(run, gc, CMat{T1b, 1, t1 * l0 * r0, s1 * t1 * l0 * r0}, CMat{yd + sp.Y.off[c], 1, nn * s1, s1},
               Mat{T2b, s0, 1, t1 * l0 * r0 * s0}, t1 * l0 * r0, s0, s1, 1.0, 0.0, (int)nn, st, true);
    if (stt != HATT_OK) return stt;
    // W^{(k)}[(g a b), c] = sum_{(i, c')} T2[(i, c'), (g a b)] W_k(c, i, c')
    stt = gemm(run, gc, CMat{T2b, 1, l0 * r0 * s0, 0}, CMat{wd + sp.W.off[c], 1, nn * t1, 0},
               Mat{W + woff[c], t0, 1, 0}, l0 * r0 * s0, t0, nn * t1, 1.0, 0.0, 1, st, true);
    if (stt != HATT_OK) return stt;
  }
  // ---- sweep (Alg. 4)
  {
    // X^{(1)}: row i, columns (a, b, c) of the first cores
    PkpArgs p1{xd, yd, ptmp, 1, r[1], 1, s[1], n[0], 0, 0, 0, 1};
    LAUNCH(launch_pkp(p1, st));
    PkpArgs p2{ptmp, wd, Xc, 1, r[1] * s[1], 1, t[1], n[0], 0, 0, 0, 1};
    LAUNCH(launch_pkp(p2, st));
  }
  for (int c = 0; c < d - 1; ++c) {
    const int64_t nn = n[c], lc = l[c], l1 = l[c + 1], K1 = rst[c + 1];
    // sketched frame: slice i of X^{(k)} (rows g) times W^{(k)} -> frame rows (g, i)
    stt = gemm(run, gc, CMat{Xc, K1, 1, lc * K1}, CMat{W + woff[c + 1], 1, K1, 0}, Mat{Yb, nn * l1, 1, l1}, lc, l1,
               K1, 1.0, 0.0, (int)nn, st, true);
    if (stt != HATT_OK) return stt;
    double *qcore = sp.out + ooff[c];
    stt = qr_exec(run, qp[c], CMat{Yb, l1, 1, ysz}, Mat{qcore, l1, 1, sp.ostride}, Mat{nullptr, 0, 0, 0}, 0, wqr,
                  qrws, 1, gc, st);
    if (stt != HATT_OK) return stt;
    // M = Q^T X^{(k)} = sum_i Q_i^T X_i, stored column-major (rows g')
    if (nn == 1) {
      stt = gemm(run, gc, CMat{qcore, 1, l1, 0}, CMat{Xc, K1, 1, 0}, Mat{Mb, 1, l1, 0}, l1, K1, lc, 1.0, 0.0, 1, st,
                 true);
      if (stt != HATT_OK) return stt;
    } else {
      stt = gemm(run, gc, CMat{qcore, 1, nn * l1, l1}, CMat{Xc, K1, 1, lc * K1}, Mat{Mp, K1, 1, l1 * K1}, l1, K1,
                 lc, 1.0, 0.0, (int)nn, st, false);
      if (stt != HATT_OK) return stt;
      GemmArgs ra{};
      ra.M = l1;
      ra.N = K1;
      ra.batch = 1;
      ra.ksplit = (int)nn;
      ra.part = Mp;
      ra.C = Mat{Mb, 1, l1, 0};
      ra.alpha = 1.0;
      ra.beta = 0.0;
      site("reduce M over %lld slices", (long long)nn);
      LAUNCH(launch_splitk_reduce(ra, st));
    }
    const int cn = c + 1;
    if (cn == d - 1) {
      // last core: X_d(g, i) = sum_{(a, b, c)} M(g, (a, b, c)) X_d(a, i) Y_d(b, i) W_d(c, i)
      stt = gemm(run, gc, CMat{Mb, 1, l1, 0}, CMat{Hlast, n[cn], 1, 0}, Mat{sp.out + ooff[cn], n[cn], 1, 0}, l1,
                 n[cn], K1, 1.0, 0.0, 1, st, true);
      if (stt != HATT_OK) return stt;
      continue;
    }
    const int64_t n1 = n[cn], ra_ = r[cn], sa = s[cn], ta = t[cn], r2 = r[cn + 1], s2 = s[cn + 1], t2 = t[cn + 1];
    // U1_i[(b c g), a'] = sum_a M[a, (b c g)] X(a, i, a')
    stt = gemm(run, gc, CMat{Mb, 1, sa * ta * l1, 0}, CMat{xd + sp.X.off[cn], n1 * r2, 1, r2},
               Mat{U1, r2, 1, sa * ta * l1 * r2}, sa * ta * l1, r2, ra_, 1.0, 0.0, (int)n1, st, true);
    if (stt != HATT_OK) return stt;
    // U2_i[(c g a'), b'] = sum_b U1_i[b, (c g a')] Y(b, i, b')
    stt = gemm(run, gc, CMat{U1, 1, ta * l1 * r2, sa * ta * l1 * r2}, CMat{yd + sp.Y.off[cn], n1 * s2, 1, s2},
               Mat{U2, s2, 1, ta * l1 * r2 * s2}, ta * l1 * r2, s2, sa, 1.0, 0.0, (int)n1, st, true);
    if (stt != HATT_OK) return stt;
    // X^{(k+1)}_i[(g a' b'), c'] = sum_c U2_i[c, (g a' b')] W(c, i, c')
    stt = gemm(run, gc, CMat{U2, 1, l1 * r2 * s2, ta * l1 * r2 * s2}, CMat{wd + sp.W.off[cn], n1 * t2, 1, t2},
               Mat{Xc, t2, 1, l1 * rst[cn + 1]}, l1 * r2 * s2, t2, ta, 1.0, 0.0, (int)n1, st, true);
    if (stt != HATT_OK) return stt;
  }
  if ((int)l.size() > kMaxRankPattern) return fail(HATT_EUNSUPPORTED, "order too large for the library (rank pattern buffer)");
  LAUNCH(launch_rank_pattern(sp.orank, 1, d + 1, l.data(), st));
  bool capped = false;
  for (int64_t cp : sp.bond_cap) capped = capped || cp > 0;
  if ((capped || sp.o.tol > 0.0) && d >= 2) {
    stt = truncate_left_orth(run, n, l, sp.out, sp.ostride, sp.orank, sp.bond_cap, sp.o.tol, 1, ws, st);
    if (stt != HATT_OK) return stt;
  }
  return HATT_OK;
}

// ---------------------------------------------------------------------------
// ||x (.) y||_F^2 per train without the PKP cores (Sec. 2.2: the product's
// cores are Z_k(i) = X_k(i) kron Y_k(i)).  The Gram recursion of the TT inner
// product, G_0 = 1, G_k = sum_i Z_k(i)^T G_{k-1} Z_k(i), ||z||^2 = G_d, with
// each step as two sandwich contractions (the identity of eq.
// kronecker_product_times_vec applied to the rows of G, then to the columns
// of the result) and a fixed-order sum over i:
//   K_i[(a b), (c' d')] = sum_{c, d} G[(a b), (c d)] X(c, i, c') Y(d, i, d')
//   G'[(a' b'), (c' d')] = sum_i sum_{a, b} X(a, i, a') Y(b, i, b') K_i[(a b), (c' d')]
// The second contraction runs one mode index per batch entry (the
// sandwich's batch dimension carries i), so trains are taken one at a time.
hatt_status hadamard_norm2_body(bool run, const Shape &X, const Shape &Y, double *out, Ws &ws, GemmCtx &gc,
                                hipStream_t st) {
  const int d = X.d;
  const auto &n = X.n, &r = X.r, &s = Y.r;
  int64_t gsz = 1, ksz = 1;
  for (int k = 0; k < d; ++k) {
    gsz = std::max(gsz, (r[k + 1] * s[k + 1]) * (r[k + 1] * s[k + 1]));
    ksz = std::max(ksz, n[k] * (r[k] * s[k]) * (r[k + 1] * s[k + 1]));
    ksz = std::max(ksz, n[k] * (r[k + 1] * s[k + 1]) * (r[k + 1] * s[k + 1]));
  }
  double *G = ws.d(gsz), *Kb = ws.d(ksz), *Ob = ws.d(ksz);
  for (int p = 0; p < X.batch; ++p) {
    LAUNCH(launch_fill(G, 1, 1.0, st));
    for (int k = 0; k < d; ++k) {
      const int64_t r0 = r[k], s0 = s[k], r1 = r[k + 1], s1 = s[k + 1], nn = n[k];
      const int64_t q0 = r0 * s0, q1 = r1 * s1;
      const double *xk = X.data + p * X.stride + X.off[k], *yk = Y.data + p * Y.stride + Y.off[k];
      SandwichArgs a{};
      // K_i = G Z_i: row g of G folded to (c, d), X_i^T (.) Y_i
      a.yl = xk;
      a.ylb = 0;
      a.yli = r1;
      a.ylr = 1;
      a.ylc = nn * r1;
      a.zr = yk;
      a.zrb = 0;
      a.zri = s1;
      a.zrr = nn * s1;
      a.zrc = 1;
      a.c = G;
      a.cb = 0;
      a.cg = q0;
      a.ca = s0;
      a.cbb = 1;
      a.o = Kb;
      a.ob = 0;
      a.oi = q0 * q1;
      a.og = q1;
      a.oa = s1;
      a.obb = 1;
      a.RA = (int)r1;
      a.RI = (int)r0;
      a.SI = (int)s0;
      a.SO = (int)s1;
      a.n = nn;
      a.G = q0;
      a.batch = 1;
      if (!sandwich_supported(a)) return fail(HATT_EUNSUPPORTED, "||x (.) y||: no sandwich kernel for these ranks");
      site("norm2 rows n=%lld G=%lld RA=%d RI=%d SI=%d SO=%d", (long long)nn, (long long)q0, a.RA, a.RI, a.SI, a.SO);
      LAUNCH(launch_sandwich(a, st));
      // O_i = Z_i^T K_i: column g of K_i folded to (a, b); the batch entry is i
      SandwichArgs b{};
      b.yl = xk;
      b.ylb = r1;
      b.yli = 0;
      b.ylr = 1;
      b.ylc = nn * r1;
      b.zr = yk;
      b.zrb = s1;
      b.zri = 0;
      b.zrr = nn * s1;
      b.zrc = 1;
      b.c = Kb;
      b.cb = q0 * q1;
      b.cg = 1;
      b.ca = s0 * q1;
      b.cbb = q1;
      b.o = (nn == 1) ? G : Ob;
      b.ob = q1 * q1;
      b.oi = 0;
      b.og = 1;
      b.oa = s1 * q1;
      b.obb = q1;
      b.RA = (int)r1;
      b.RI = (int)r0;
      b.SI = (int)s0;
      b.SO = (int)s1;
      b.n = 1;
      b.G = q1;
      b.batch = (int)nn;
      if (!sandwich_supported(b)) return fail(HATT_EUNSUPPORTED, "||x (.) y||: no sandwich kernel for these ranks");
      site("norm2 columns n=%lld G=%lld RA=%d RI=%d SI=%d SO=%d", (long long)nn, (long long)q1, b.RA, b.RI, b.SI,
           b.SO);
      LAUNCH(launch_sandwich(b, st));
      if (nn > 1) {
        // G = sum_i O_i in the order of i
        GemmArgs ra{};
        ra.M = q1;
        ra.N = q1;
        ra.batch = 1;
        ra.ksplit = (int)nn;
        ra.part = Ob;
        ra.C = Mat{G, q1, 1, 0};
        ra.alpha = 1.0;
        ra.beta = 0.0;
        LAUNCH(launch_splitk_reduce(ra, st));
      }
    }
    LAUNCH(launch_copy(CMat{G, 1, 1, 0}, Mat{out + p, 1, 1, 0}, 1, 1, 1, st));
  }
  (void)gc;
  return HATT_OK;
}

hatt_status hatt_run(bool run, const HattSpec &sp, Ws &ws, hipStream_t st) {
  Ws probe(nullptr);
  GemmCtx g0{nullptr, 0, 0};
  hatt_status s = hatt_body(false, sp, probe, g0, st);
  if (s != HATT_OK) return s;
  GemmCtx g1{nullptr, 0, 0};
  g1.part = ws.d(std::max<int64_t>(g0.part_need, 1));
  g1.part_cap = g0.part_need;
  return hatt_body(run, sp, ws, g1, st);
}

// ---------------------------------------------------------------------------
// RandOrth (Alg. 2) on an explicit TT a (for a Hadamard product: its PKP
// cores), with the sketch right to left (eq. rtlpc) and the orthogonalising
// sweep, then optionally TT-Rounding of the rank-l result.  The paper's
// second comparator (Table 4.1): the same products and QRs as HaTT, but on
// cores of rank R_k = r_k s_k.
struct RoSpec {
  Shape A;
  std::vector<int64_t> ell;
  const double *sketch;
  int64_t sketch_stride;
  uint64_t seed;
  int64_t max_rank;
  double tol;
  double *out;
  int64_t ostride;
  int64_t *orank;
};

hatt_status randorth_body(bool run, const RoSpec &sp, Ws &ws, GemmCtx &gc, hipStream_t st) {
  const int d = sp.A.d, P = sp.A.batch;
  const auto &n = sp.A.n, &R = sp.A.r, &l = sp.ell;
  std::vector<int64_t> ooff, skoff;
  int64_t otot, sktot;
  make_offsets(n, l, &ooff, &otot);
  make_offsets(n, l, &skoff, &sktot);
  const double *ad = sp.A.data;
  const int64_t as = sp.A.stride;
  std::vector<int64_t> woff(d + 1, 0);
  int64_t wtot = 1, tsz = 1, bsz = 1, ysz = 1, msz = 1, qrws = 1;
  for (int b = 1; b < d; ++b) {
    woff[b] = wtot;
    wtot += R[b] * l[b];
  }
  for (int c = 1; c <= d - 2; ++c) tsz = std::max(tsz, R[c] * n[c] * l[c + 1]);
  std::vector<QrOp> qp(d);
  for (int c = 0; c < d - 1; ++c) {
    bsz = std::max(bsz, l[c] * n[c] * R[c + 1]);
    ysz = std::max(ysz, l[c] * n[c] * l[c + 1]);
    msz = std::max(msz, l[c + 1] * R[c + 1]);
    if (!qr_prepare(l[c] * n[c], l[c + 1], &qp[c]))
      return fail(HATT_EUNSUPPORTED, "RandOrth: the QR of a " + std::to_string(l[c] * n[c]) + " x " +
                                         std::to_string(l[c + 1]) + " sketched frame is not supported");
    qrws = std::max(qrws, qp[c].ws_doubles);
  }
  bsz = std::max(bsz, l[d - 1] * n[d - 1]);
  double *sk = sp.sketch ? (double *)sp.sketch : ws.d(sktot);
  const int64_t sks = sp.sketch ? sp.sketch_stride : 0;
  double *W = ws.d((int64_t)P * wtot);
  double *T = ws.d((int64_t)P * tsz);
  double *B0 = ws.d((int64_t)P * bsz);
  double *B1 = ws.d((int64_t)P * bsz);
  double *Yb = ws.d((int64_t)P * ysz);
  double *Mb = ws.d((int64_t)P * msz);
  double *wqr = ws.d((int64_t)P * qrws);
  if (d == 1) {
    LAUNCH(launch_fill_i64(sp.orank, (int64_t)P * 2, 1, st));
    LAUNCH(launch_copy(CMat{ad, n[0], 1, as}, Mat{sp.out, n[0], 1, sp.ostride}, 1, n[0], P, st));
    return HATT_OK;
  }
  if (!sp.sketch) {
    for (int k = 0; k < d; ++k) {
      const int64_t cnt = l[k] * n[k] * l[k + 1];
      LAUNCH(launch_sketch_fill(sp.seed, k, cnt, 1.0 / sqrt((double)cnt), sk + skoff[k], st));
    }
  }
  // W^{(d-1)} = H(A_d) H(R_d)^T
  hatt_status s = gemm(run, gc, CMat{ad + sp.A.off[d - 1], n[d - 1], 1, as}, CMat{sk + skoff[d - 1], 1, n[d - 1], sks},
                       Mat{W + woff[d - 1], l[d - 1], 1, wtot}, R[d - 1], l[d - 1], n[d - 1], 1.0, 0.0, P, st, true);
  if (s != HATT_OK) return s;
  for (int c = d - 2; c >= 1; --c) {
    // V(T) = V(A_c) W^{(c+1)}; W^{(c)} = H(T) H(R_c)^T
    s = gemm(run, gc, CMat{ad + sp.A.off[c], R[c + 1], 1, as}, CMat{W + woff[c + 1], l[c + 1], 1, wtot},
             Mat{T, l[c + 1], 1, tsz}, R[c] * n[c], l[c + 1], R[c + 1], 1.0, 0.0, P, st, true);
    if (s != HATT_OK) return s;
    s = gemm(run, gc, CMat{T, n[c] * l[c + 1], 1, tsz}, CMat{sk + skoff[c], 1, n[c] * l[c + 1], sks},
             Mat{W + woff[c], l[c], 1, wtot}, R[c], l[c], n[c] * l[c + 1], 1.0, 0.0, P, st, true);
    if (s != HATT_OK) return s;
  }
  // sweep: B_1 = A_1; Y = V(B_k) W^{(k)}, Q = qr(Y), M = Q^T V(B_k), H(B_{k+1}) = M H(A_{k+1})
  double *Bc = B0, *Bn = B1;
  LAUNCH(launch_copy(CMat{ad, R[1], 1, as}, Mat{Bc, R[1], 1, bsz}, n[0], R[1], P, st));
  for (int c = 0; c < d - 1; ++c) {
    const int64_t m = l[c] * n[c];
    s = gemm(run, gc, CMat{Bc, R[c + 1], 1, bsz}, CMat{W + woff[c + 1], l[c + 1], 1, wtot}, Mat{Yb, l[c + 1], 1, ysz},
             m, l[c + 1], R[c + 1], 1.0, 0.0, P, st, true);
    if (s != HATT_OK) return s;
    double *qcore = sp.out + ooff[c];
    s = qr_exec(run, qp[c], CMat{Yb, l[c + 1], 1, ysz}, Mat{qcore, l[c + 1], 1, sp.ostride}, Mat{nullptr, 0, 0, 0}, 0,
                wqr, qrws, P, gc, st);
    if (s != HATT_OK) return s;
    s = gemm(run, gc, CMat{qcore, 1, l[c + 1], sp.ostride}, CMat{Bc, R[c + 1], 1, bsz}, Mat{Mb, R[c + 1], 1, msz},
             l[c + 1], R[c + 1], m, 1.0, 0.0, P, st, true);
    if (s != HATT_OK) return s;
    const int cn = c + 1;
    const int64_t ncol = n[cn] * R[cn + 1];
    if (cn < d - 1) {
      s = gemm(run, gc, CMat{Mb, R[cn], 1, msz}, CMat{ad + sp.A.off[cn], ncol, 1, as}, Mat{Bn, ncol, 1, bsz}, l[cn],
               ncol, R[cn], 1.0, 0.0, P, st, true);
    } else {
      s = gemm(run, gc, CMat{Mb, R[cn], 1, msz}, CMat{ad + sp.A.off[cn], ncol, 1, as},
               Mat{sp.out + ooff[cn], ncol, 1, sp.ostride}, l[cn], ncol, R[cn], 1.0, 0.0, P, st, true);
    }
    if (s != HATT_OK) return s;
    std::swap(Bc, Bn);
  }
  if ((int)l.size() > kMaxRankPattern) return fail(HATT_EUNSUPPORTED, "order too large for the library (rank pattern buffer)");
  LAUNCH(launch_rank_pattern(sp.orank, P, d + 1, l.data(), st));
  if ((sp.max_rank > 0 || sp.tol > 0.0) && d >= 2) {
    // RandOrth's cores but the last are the Q factors of its QRs: left-orthogonal
    std::vector<int64_t> caps(d + 1, std::max<int64_t>(sp.max_rank, 0));
    s = truncate_left_orth(run, n, l, sp.out, sp.ostride, sp.orank, caps, sp.tol, P, ws, st);
    if (s != HATT_OK) return s;
  }
  return HATT_OK;
}

hatt_status randorth_run(bool run, const RoSpec &sp, Ws &ws, hipStream_t st) {
  Ws probe(nullptr);
  GemmCtx g0{nullptr, 0, 0};
  hatt_status s = randorth_body(false, sp, probe, g0, st);
  if (s != HATT_OK) return s;
  GemmCtx g1{nullptr, 0, 0};
  g1.part = ws.d(std::max<int64_t>(g0.part_need, 1));
  g1.part_cap = g0.part_need;
  return randorth_body(run, sp, ws, g1, st);
}

hatt_status randorth_prepare(const hatt_tt *a, int64_t ell, const int64_t *ell_bond, int64_t max_rank, double tol,
                             RoSpec *sp, bool need_data) {
  hatt_status st = read_tt(a, "a", &sp->A, need_data);
  if (st != HATT_OK) return st;
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(HATT_EINVAL, "tol must be finite and >= 0");
  const int d = sp->A.d;
  std::vector<int64_t> req(d + 1, 1), ones(d + 1, 1);
  for (int k = 1; k < d; ++k) {
    req[k] = ell_bond ? ell_bond[k] : ell;
    if (req[k] < 1) return fail(HATT_EINVAL, "sketch width must be >= 1");
  }
  sp->ell = clamp_ell(sp->A.n, sp->A.r, ones, req);
  sp->max_rank = max_rank;
  sp->tol = tol;
  sp->sketch = nullptr;
  sp->sketch_stride = 0;
  sp->out = nullptr;
  sp->orank = nullptr;
  return HATT_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

hatt_status tt_randorth_plan(const hatt_tt *a, int64_t ell, const int64_t *ell_bond, int64_t *ell_out,
                             size_t *ws_bytes, int64_t *out_elems) {
  RoSpec sp{};
  hatt_status st = randorth_prepare(a, ell, ell_bond, 0, 0.0, &sp, false);
  if (st != HATT_OK) return st;
  // the truncation's workspace is the larger one: plan with it
  sp.tol = 1.0;
  Ws ws(nullptr);
  st = randorth_run(false, sp, ws, nullptr);
  if (st != HATT_OK) return st;
  if (ell_out)
    for (int k = 0; k <= sp.A.d; ++k) ell_out[k] = sp.ell[k];
  if (ws_bytes) *ws_bytes = ws.off;
  if (out_elems) {
    std::vector<int64_t> off;
    int64_t tot;
    make_offsets(sp.A.n, sp.ell, &off, &tot);
    *out_elems = tot;
  }
  g_err.clear();
  return HATT_OK;
}

hatt_status tt_randorth(const hatt_tt *a, const hatt_tt *sketch, int64_t ell, const int64_t *ell_bond, uint64_t seed,
                        int64_t max_rank, double tol, double *out, int64_t out_stride, int64_t *out_rank, void *ws,
                        size_t ws_bytes, void *stream) {
  RoSpec sp{};
  hatt_status st = randorth_prepare(a, ell, ell_bond, max_rank, tol, &sp, true);
  if (st != HATT_OK) return st;
  if (out == nullptr || out_rank == nullptr) return fail(HATT_EINVAL, "out or out_rank is NULL");
  std::vector<int64_t> off;
  int64_t otot;
  make_offsets(sp.A.n, sp.ell, &off, &otot);
  if (out_stride != 0 && out_stride < otot) return fail(HATT_EINVAL, "out_stride smaller than one output train");
  sp.out = out;
  sp.ostride = out_stride ? out_stride : otot;
  sp.orank = out_rank;
  sp.seed = seed;
  if (sketch != nullptr) {
    Shape sk;
    st = read_tt(sketch, "sketch", &sk, true);
    if (st != HATT_OK) return st;
    if (sk.d != sp.A.d || sk.n != sp.A.n || sk.r != sp.ell)
      return fail(HATT_ESHAPE, "sketch shape differs from the planned sketch widths");
    if (sk.batch != 1 && sk.batch != sp.A.batch)
      return fail(HATT_ESHAPE, "sketch batch must be 1 or equal to the input batch");
    sp.sketch = sk.data;
    sp.sketch_stride = (sk.batch == 1) ? 0 : sk.stride;
  }
  Ws meas(nullptr);
  st = randorth_run(false, sp, meas, nullptr);
  if (st != HATT_OK) return st;
  if (ws == nullptr || ws_bytes < meas.off)
    return fail(HATT_EWORKSPACE, "workspace too small: need " + std::to_string(meas.off) + " bytes");
  Ws w(ws);
  st = randorth_run(true, sp, w, (hipStream_t)stream);
  if (st == HATT_OK) g_err.clear();
  return st;
}

const char *hatt_last_error(void) { return g_err.c_str(); }

hatt_status hatt_profile_start(void) {
  g_prof.recs.clear();
  g_prof.used = 0;
  g_prof.on = true;
  return HATT_OK;
}

hatt_status hatt_profile_stop(double *ms_out, int64_t *calls_out) {
  g_prof.on = false;
  if (ms_out == nullptr || calls_out == nullptr) return fail(HATT_EINVAL, "profile_stop: NULL output");
  for (int c = 0; c < P_NCLASS; ++c) {
    ms_out[c] = 0.0;
    calls_out[c] = 0;
  }
  std::map<std::string, std::pair<double, int64_t>> by_site;
  for (const ProfRec &r : g_prof.recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(HATT_EDEVICE, "profile_stop: event sync failed");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      return fail(HATT_EDEVICE, "profile_stop: elapsed time failed");
    ms_out[r.cls] += ms;
    calls_out[r.cls] += 1;
    auto &acc = by_site[r.site];
    acc.first += ms;
    acc.second += 1;
  }
  std::vector<std::pair<double, std::string>> rows;
  for (auto &kv : by_site) {
    char b[64];
    snprintf(b, sizeof b, "%12.3f ms %8lld calls  ", kv.second.first, (long long)kv.second.second);
    rows.emplace_back(kv.second.first, std::string(b) + kv.first);
  }
  std::sort(rows.begin(), rows.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
  g_prof_report.clear();
  for (auto &rw : rows) g_prof_report += rw.second + "\n";
  g_prof.recs.clear();
  g_prof.used = 0;
  return HATT_OK;
}

const char *hatt_profile_report(void) { return g_prof_report.c_str(); }

hatt_status hatt_set_qr_method(int32_t method) {
  if (method != 0 && method != 1) return fail(HATT_EINVAL, "QR method must be 0 (CholeskyQR2 + fallback) or 1");
  g_use_chol = (method == 0);
  return HATT_OK;
}

hatt_status hatt_tune_mode(int32_t mode) {
  if (mode < 0 || mode > 2) return fail(HATT_EINVAL, "tune mode must be 0 (off), 1 (record) or 2 (use)");
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_mode = mode;
  g_err.clear();
  return HATT_OK;
}

hatt_status hatt_tune_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.clear();
  g_err.clear();
  return HATT_OK;
}

int64_t hatt_tune_table(char *buf, int64_t cap) {
  std::string txt;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    char line[160];
    for (const auto &kv : g_tune) {
      snprintf(line, sizeof line, " -> %s  %.1f us (fixed rules %.1f us)\n", kv.second.choice.c_str(), kv.second.us,
               kv.second.us_default);
      txt += kv.first + line;
    }
  }
  const int64_t len = (int64_t)txt.size();
  if (buf != nullptr && cap > 0) {
    const int64_t n = std::min(len, cap - 1);
    memcpy(buf, txt.data(), (size_t)n);
    buf[n] = '\0';
  }
  return len + 1;
}

const char *hatt_profile_class_name(int32_t cls) {
  if (cls < 0 || cls >= P_NCLASS) return "";
  return kClassNames[cls];
}
const char *hatt_version(void) { return "hatt-mi355x 0.1 (gfx950, fp64)"; }

static hatt_status hatt_prepare(const hatt_tt *x, const hatt_tt *y, const hatt_tt *w, const hatt_opts *o,
                                HattSpec *sp, bool need_data) {
  if (o == nullptr) return fail(HATT_EINVAL, "opts is NULL");
  hatt_status st = read_tt(x, "x", &sp->X, need_data);
  if (st != HATT_OK) return st;
  st = read_tt(y, "y", &sp->Y, need_data);
  if (st != HATT_OK) return st;
  if (sp->X.d != sp->Y.d) return fail(HATT_ESHAPE, "x and y have different orders");
  if (sp->X.batch != sp->Y.batch) return fail(HATT_ESHAPE, "x and y have different batch counts");
  if (sp->X.n != sp->Y.n) return fail(HATT_ESHAPE, "x and y have different mode sizes");
  sp->ryw = sp->Y.r;
  sp->three = (w != nullptr);
  if (sp->three) {
    st = read_tt(w, "w", &sp->W, need_data);
    if (st != HATT_OK) return st;
    if (sp->W.d != sp->X.d) return fail(HATT_ESHAPE, "x and w have different orders");
    if (sp->W.n != sp->X.n) return fail(HATT_ESHAPE, "x and w have different mode sizes");
    if (sp->X.batch != 1 || sp->W.batch != 1)
      return fail(HATT_EUNSUPPORTED, "three factors: one triple per call (batch 1)");
    if (o->variant != 1) return fail(HATT_EUNSUPPORTED, "three factors: HaTT-1 only");
    if (o->precision != 0) return fail(HATT_EUNSUPPORTED, "three factors: FP64 only");
    for (int k = 0; k <= sp->X.d; ++k) sp->ryw[k] = sp->Y.r[k] * sp->W.r[k];
  }
  if (o->variant != 1 && o->variant != 2) return fail(HATT_EINVAL, "variant must be 1 or 2");
  if (o->variant == 2 && !(o->ep >= 0.0 && o->ep < 1.0)) return fail(HATT_EINVAL, "ep must be in [0, 1)");
  if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return fail(HATT_EINVAL, "tol must be finite and >= 0");
  if (o->precision < 0 || o->precision > 2)
    return fail(HATT_EINVAL, "precision must be 0 (FP64), 1 (FP32) or 2 (BF16)");
  if (o->precision != 0 && o->variant != 1)
    return fail(HATT_EUNSUPPORTED, "low-precision range finding is built for HaTT-1 only");
  const int d = sp->X.d;
  std::vector<int64_t> req(d + 1, 1);
  for (int k = 1; k < d; ++k) {
    req[k] = o->ell_bond ? o->ell_bond[k] : o->ell;
    if (req[k] < 1) return fail(HATT_EINVAL, "sketch width must be >= 1");
  }
  sp->ell = clamp_ell(sp->X.n, sp->X.r, sp->ryw, req);
  sp->o = *o;
  sp->o.max_rank_bond = nullptr;  // read here only; the caller's array need not outlive the call
  sp->bond_cap.assign(d + 1, std::max<int64_t>(o->max_rank, 0));
  if (o->max_rank_bond != nullptr)
    for (int k = 1; k < d; ++k)
      if (o->max_rank_bond[k] > 0) sp->bond_cap[k] = o->max_rank_bond[k];
  return HATT_OK;
}

static hatt_status plan_common(const hatt_tt *x, const hatt_tt *y, const hatt_tt *w, const hatt_opts *opts,
                               int64_t *ell_out, size_t *ws_bytes, int64_t *out_elems) {
  HattSpec sp{};
  hatt_status st = hatt_prepare(x, y, w, opts, &sp, false);
  if (st != HATT_OK) return st;
  sp.sketch = nullptr;
  sp.out = nullptr;
  sp.orank = nullptr;
  Ws ws(nullptr);
  st = hatt_run(false, sp, ws, nullptr);
  if (st != HATT_OK) return st;
  if (ell_out)
    for (int k = 0; k <= sp.X.d; ++k) ell_out[k] = sp.ell[k];
  if (ws_bytes) *ws_bytes = ws.off;
  if (out_elems) {
    std::vector<int64_t> off;
    int64_t tot;
    make_offsets(sp.X.n, sp.ell, &off, &tot);
    *out_elems = tot;
  }
  g_err.clear();
  return HATT_OK;
}

static hatt_status recompress_common(const hatt_tt *x, const hatt_tt *y, const hatt_tt *w, const hatt_tt *sketch,
                                     const hatt_opts *opts, double *out, int64_t out_stride, int64_t *out_rank,
                                     void *ws, size_t ws_bytes, void *stream) {
  HattSpec sp{};
  hatt_status st = hatt_prepare(x, y, w, opts, &sp, true);
  if (st != HATT_OK) return st;
  if (out == nullptr || out_rank == nullptr) return fail(HATT_EINVAL, "out or out_rank is NULL");
  std::vector<int64_t> off;
  int64_t otot;
  make_offsets(sp.X.n, sp.ell, &off, &otot);
  if (out_stride != 0 && out_stride < otot) return fail(HATT_EINVAL, "out_stride smaller than one output train");
  sp.out = out;
  sp.ostride = out_stride ? out_stride : otot;
  sp.orank = out_rank;
  sp.sketch = nullptr;
  sp.sketch_stride = 0;
  if (sketch != nullptr) {
    Shape sk;
    st = read_tt(sketch, "sketch", &sk, true);
    if (st != HATT_OK) return st;
    if (sk.d != sp.X.d || sk.n != sp.X.n || sk.r != sp.ell)
      return fail(HATT_ESHAPE, "sketch shape differs from the planned sketch widths");
    if (sk.batch != 1 && sk.batch != sp.X.batch)
      return fail(HATT_ESHAPE, "sketch batch must be 1 or equal to the input batch");
    sp.sketch = sk.data;
    sp.sketch_stride = (sk.batch == 1) ? 0 : sk.stride;
  }
  Ws meas(nullptr);
  st = hatt_run(false, sp, meas, nullptr);
  if (st != HATT_OK) return st;
  if (ws == nullptr || ws_bytes < meas.off)
    return fail(HATT_EWORKSPACE, "workspace too small: need " + std::to_string(meas.off) + " bytes");
  Ws wk(ws);
  st = hatt_run(true, sp, wk, (hipStream_t)stream);
  if (st == HATT_OK) g_err.clear();
  return st;
}

hatt_status hatt_plan(const hatt_tt *x, const hatt_tt *y, const hatt_opts *opts, int64_t *ell_out,
                      size_t *ws_bytes, int64_t *out_elems) {
  return plan_common(x, y, nullptr, opts, ell_out, ws_bytes, out_elems);
}

hatt_status hatt_recompress(const hatt_tt *x, const hatt_tt *y, const hatt_tt *sketch, const hatt_opts *opts,
                            double *out, int64_t out_stride, int64_t *out_rank, void *ws, size_t ws_bytes,
                            void *stream) {
  return recompress_common(x, y, nullptr, sketch, opts, out, out_stride, out_rank, ws, ws_bytes, stream);
}

hatt_status hatt_plan3(const hatt_tt *x, const hatt_tt *y, const hatt_tt *w, const hatt_opts *opts,
                       int64_t *ell_out, size_t *ws_bytes, int64_t *out_elems) {
  if (w == nullptr) return fail(HATT_EINVAL, "w: NULL tensor view");
  return plan_common(x, y, w, opts, ell_out, ws_bytes, out_elems);
}

hatt_status hatt_recompress3(const hatt_tt *x, const hatt_tt *y, const hatt_tt *w, const hatt_tt *sketch,
                             const hatt_opts *opts, double *out, int64_t out_stride, int64_t *out_rank, void *ws,
                             size_t ws_bytes, void *stream) {
  if (w == nullptr) return fail(HATT_EINVAL, "w: NULL tensor view");
  return recompress_common(x, y, w, sketch, opts, out, out_stride, out_rank, ws, ws_bytes, stream);
}

hatt_status hatt_recompress_noalloc(const hatt_tt *x, const hatt_tt *y, const hatt_tt *sketch, const hatt_opts *opts,
                                    double *out, int64_t out_stride, int64_t *out_rank, void *stream) {
  // the size check is host-only and comes before any device call
  size_t need = 0;
  hatt_status st = hatt_plan(x, y, opts, nullptr, &need, nullptr);
  if (st != HATT_OK) return st;
  if (need > kScratchBytes)
    return fail(HATT_EWORKSPACE, "hatt_recompress_noalloc: the problem needs " + std::to_string(need) +
                                     " bytes of scratch; the library's static scratch holds " +
                                     std::to_string(kScratchBytes) + " (use hatt_recompress with a workspace)");
  void *ws = nullptr;
  st = scratch_address(&ws);
  if (st != HATT_OK) return st;
  return hatt_recompress(x, y, sketch, opts, out, out_stride, out_rank, ws, kScratchBytes, stream);
}

// ---------------------------------------------------------------------------
// Uneven batches: every pair has its own shape.  Pairs are planned one by one
// and run on up to kBatchStreams library streams forked from the caller's
// stream (event wait) and joined back; pairs go largest first to the least
// loaded stream, and each stream reuses one workspace slot, so concurrent
// pairs never share scratch memory.  How many streams run at once is set by
// the process's hardware queues (HIP's GPU_MAX_HW_QUEUES, 4 by default).
constexpr int kBatchStreams = 32;
// Largest uneven batch accepted while the caller's stream is being captured
// into a HIP graph: the capture of a 512-pair batch (of the order of 10^5
// kernel nodes on 32 forked streams) ended the process on the host, and the
// largest captured batch known to replay correctly has 12 pairs.
constexpr int kBatchCaptureMaxPairs = 12;
// Serialises the library streams' fork / join sequence (and their creation)
// between host threads: the fork event and the streams are shared per device.
std::mutex g_batch_mu;

struct BatchStreams {
  int device = -1;
  hipStream_t s[kBatchStreams] = {};
  hipEvent_t fork = nullptr, join[kBatchStreams] = {};
};
std::vector<BatchStreams> g_bstreams;

static hatt_status batch_streams(BatchStreams **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(HATT_EDEVICE, "hipGetDevice failed");
  for (auto &b : g_bstreams)
    if (b.device == dev) {
      *out = &b;
      return HATT_OK;
    }
  BatchStreams b;
  b.device = dev;
  for (int k = 0; k < kBatchStreams; ++k) {
    if (hipStreamCreateWithFlags(&b.s[k], hipStreamNonBlocking) != hipSuccess)
      return fail(HATT_EDEVICE, "stream creation failed");
    if (hipEventCreateWithFlags(&b.join[k], hipEventDisableTiming) != hipSuccess)
      return fail(HATT_EDEVICE, "event creation failed");
  }
  if (hipEventCreateWithFlags(&b.fork, hipEventDisableTiming) != hipSuccess)
    return fail(HATT_EDEVICE, "event creation failed");
  g_bstreams.push_back(b);
  *out = &g_bstreams.back();
  return HATT_OK;
}

// Enqueues each library stream's pairs (in `order`) from a host thread of
// its own: a pair with many launches (wide truncations issue thousands) would
// otherwise hold the one enqueuing thread, and every other stream with it,
// until its own hardware queue has room again.  Single-threaded under graph
// capture, with the profiler on, or while the autotuner records (their
// records are not shared between threads).  run_pair(p, k) enqueues pair p
// on stream k; the first failure is reported after every thread has ended.
static hatt_status batch_enqueue(int streams, const std::vector<int> &order, const std::vector<int> &stream_of,
                                 bool threaded, int device,
                                 const std::function<hatt_status(int, int)> &run_pair) {
  if (!threaded || streams <= 1) {
    for (int p : order) {
      hatt_status st = run_pair(p, stream_of[p]);
      if (st != HATT_OK) return fail(st, "pair " + std::to_string(p) + ": " + g_err);
    }
    return HATT_OK;
  }
  std::vector<std::vector<int>> per(streams);
  for (int p : order) per[stream_of[p]].push_back(p);
  std::vector<hatt_status> sts(streams, HATT_OK);
  std::vector<std::string> msgs(streams);
  auto work = [&](int k) {
    if (hipSetDevice(device) != hipSuccess) {
      sts[k] = HATT_EDEVICE;
      msgs[k] = "hipSetDevice failed in an enqueuing thread";
      return;
    }
    for (int p : per[k]) {
      hatt_status st = run_pair(p, k);
      if (st != HATT_OK) {
        sts[k] = st;
        msgs[k] = "pair " + std::to_string(p) + ": " + g_err;
        return;
      }
    }
  };
  std::vector<std::thread> th;
  th.reserve(streams);
  for (int k = 0; k < streams; ++k) {
    if (per[k].empty()) continue;
    bool started = false;
    try {
      th.emplace_back(work, k);
      started = true;
    } catch (...) {
    }
    if (!started) work(k);  // no thread to be had: this stream from here
  }
  for (auto &t : th) t.join();
  for (int k = 0; k < streams; ++k)
    if (sts[k] != HATT_OK) return fail(sts[k], msgs[k]);
  return HATT_OK;
}

bool batch_threaded(hipStreamCaptureStatus cap) {
  return cap == hipStreamCaptureStatusNone && !g_prof.on && g_tune_mode != 1;
}

struct BatchPlan {
  std::vector<HattSpec> sp;
  std::vector<std::vector<int64_t>> req;  // per-pair width requests (rule widths)
  std::vector<int64_t> out_off, rank_off;
  size_t slot = 0;                        // workspace bytes of one slot
  int streams = 1;
  std::vector<int> stream_of;             // library stream of each pair
};

// Sec. 4 cost of one recompression at its widths (per train): the HaTT-1
// terms n r s l (4r + 4s + 6l) per interior core; a relative measure for
// ordering pairs.
static double batch_pair_cost(const HattSpec &sp) {
  double c = 0.0;
  for (int k = 0; k + 1 < sp.X.d; ++k) {
    const double n = (double)sp.X.n[k], r = (double)sp.X.r[k + 1], q = (double)sp.Y.r[k + 1],
                 l = (double)sp.ell[k + 1];
    c += n * r * q * l * (4.0 * r + 4.0 * q + 6.0 * l);
  }
  return (c + 1.0) * (double)sp.X.batch;
}

// Longest first onto the least loaded stream (each stream runs its pairs in
// order): the slowest stream finishes earlier than with a round robin.
static void batch_assign(BatchPlan *bp) {
  const int np = (int)bp->sp.size(), S = bp->streams;
  std::vector<int> order(np);
  std::vector<double> cost(np);
  for (int p = 0; p < np; ++p) {
    order[p] = p;
    cost[p] = batch_pair_cost(bp->sp[p]);
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<double> load(S, 0.0);
  bp->stream_of.assign(np, 0);
  for (int p : order) {
    int k = 0;
    for (int t = 1; t < S; ++t)
      if (load[t] < load[k]) k = t;
    bp->stream_of[p] = k;
    load[k] += cost[p];
  }
}

static hatt_status batch_prepare(int32_t npairs, const hatt_tt *x, const hatt_tt *y, const hatt_opts *o,
                                 bool need_data, BatchPlan *bp) {
  if (npairs < 1) return fail(HATT_EINVAL, "npairs must be >= 1");
  if (x == nullptr || y == nullptr || o == nullptr) return fail(HATT_EINVAL, "NULL argument");
  if (o->ell_bond != nullptr) return fail(HATT_EINVAL, "per-bond widths are not taken by the uneven batch");
  if (o->max_rank_bond != nullptr) return fail(HATT_EINVAL, "per-bond rank caps are not taken by the uneven batch");
  bp->sp.assign(npairs, HattSpec{});
  bp->req.assign(npairs, {});
  bp->out_off.assign(npairs + 1, 0);
  bp->rank_off.assign(npairs + 1, 0);
  size_t slot = 0;
  for (int32_t p = 0; p < npairs; ++p) {
    hatt_opts op = *o;
    op.seed = o->seed + (uint64_t)p;
    if (o->ell <= 0) {
      // width rule: l_k = max(r_k, s_k) + 8 (clamped by hatt_prepare)
      if (x[p].d < 1 || x[p].rank == nullptr || y[p].rank == nullptr || x[p].d != y[p].d)
        return fail(HATT_ESHAPE, "pair " + std::to_string(p) + ": bad order or ranks");
      auto &rq = bp->req[p];
      rq.assign(x[p].d + 1, 1);
      for (int k = 1; k < x[p].d; ++k) rq[k] = std::max(x[p].rank[k], y[p].rank[k]) + 8;
      op.ell = 1;
      op.ell_bond = rq.data();
    }
    HattSpec &sp = bp->sp[p];
    hatt_status st = hatt_prepare(&x[p], &y[p], nullptr, &op, &sp, need_data);
    if (st != HATT_OK) return fail(st, "pair " + std::to_string(p) + ": " + g_err);
    sp.o.ell_bond = nullptr;
    sp.sketch = nullptr;
    sp.sketch_stride = 0;
    sp.out = nullptr;
    sp.orank = nullptr;
    Ws meas(nullptr);
    st = hatt_run(false, sp, meas, nullptr);
    if (st != HATT_OK) return fail(st, "pair " + std::to_string(p) + ": " + g_err);
    slot = std::max(slot, (size_t)((meas.off + 255) / 256 * 256));
    std::vector<int64_t> off;
    int64_t tot;
    make_offsets(sp.X.n, sp.ell, &off, &tot);
    sp.ostride = tot;
    bp->out_off[p + 1] = bp->out_off[p] + tot * sp.X.batch;
    bp->rank_off[p + 1] = bp->rank_off[p] + (int64_t)sp.X.batch * (sp.X.d + 1);
  }
  bp->slot = std::max<size_t>(slot, 256);
  bp->streams = std::min<int>(kBatchStreams, npairs);
  batch_assign(bp);
  return HATT_OK;
}

hatt_status hatt_batched_plan(int32_t npairs, const hatt_tt *x, const hatt_tt *y, const hatt_opts *opts,
                              int64_t *out_offset, int64_t *rank_offset, int64_t *ell_out, size_t *ws_bytes) {
  BatchPlan bp;
  hatt_status st = batch_prepare(npairs, x, y, opts, false, &bp);
  if (st != HATT_OK) return st;
  if (out_offset)
    for (int32_t p = 0; p <= npairs; ++p) out_offset[p] = bp.out_off[p];
  if (rank_offset)
    for (int32_t p = 0; p <= npairs; ++p) rank_offset[p] = bp.rank_off[p];
  if (ell_out) {
    int64_t e = 0;
    for (int32_t p = 0; p < npairs; ++p)
      for (int64_t v : bp.sp[p].ell) ell_out[e++] = v;
  }
  if (ws_bytes) *ws_bytes = bp.slot * (size_t)bp.streams;
  g_err.clear();
  return HATT_OK;
}

hatt_status hatt_recompress_batched(int32_t npairs, const hatt_tt *x, const hatt_tt *y, const hatt_opts *opts,
                                    double *out, int64_t *out_rank, void *ws, size_t ws_bytes, void *stream) {
  BatchPlan bp;
  hatt_status st = batch_prepare(npairs, x, y, opts, true, &bp);
  if (st != HATT_OK) return st;
  if (out == nullptr || out_rank == nullptr) return fail(HATT_EINVAL, "out or out_rank is NULL");
  const size_t need = bp.slot * (size_t)bp.streams;
  if (ws == nullptr || ws_bytes < need)
    return fail(HATT_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  hipStream_t caller = (hipStream_t)stream;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(caller, &cap) != hipSuccess) return fail(HATT_EDEVICE, "hipStreamIsCapturing failed");
  if (cap != hipStreamCaptureStatusNone && npairs > kBatchCaptureMaxPairs)
    return fail(HATT_EUNSUPPORTED, "uneven batches of more than " + std::to_string(kBatchCaptureMaxPairs) +
                                       " pairs are not supported under HIP graph capture");
  std::lock_guard<std::mutex> lock(g_batch_mu);
  BatchStreams *bs = nullptr;
  st = batch_streams(&bs);
  if (st != HATT_OK) return st;
  if (hipEventRecord(bs->fork, caller) != hipSuccess) return fail(HATT_EDEVICE, "event record failed");
  for (int k = 0; k < bp.streams; ++k)
    if (hipStreamWaitEvent(bs->s[k], bs->fork, 0) != hipSuccess) return fail(HATT_EDEVICE, "stream wait failed");
  // enqueue in decreasing cost so each stream starts with its largest pair
  std::vector<int> order(npairs);
  for (int32_t p = 0; p < npairs; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return batch_pair_cost(bp.sp[a]) > batch_pair_cost(bp.sp[b]); });
  for (int32_t p : order) {
    bp.sp[p].out = out + bp.out_off[p];
    bp.sp[p].orank = out_rank + bp.rank_off[p];
  }
  st = batch_enqueue(bp.streams, order, bp.stream_of, batch_threaded(cap), bs->device, [&](int p, int k) {
    Ws w((char *)ws + (size_t)k * bp.slot);
    return hatt_run(true, bp.sp[p], w, bs->s[k]);
  });
  if (st != HATT_OK) return st;
  for (int k = 0; k < bp.streams; ++k) {
    if (hipEventRecord(bs->join[k], bs->s[k]) != hipSuccess) return fail(HATT_EDEVICE, "event record failed");
    if (hipStreamWaitEvent(caller, bs->join[k], 0) != hipSuccess) return fail(HATT_EDEVICE, "stream wait failed");
  }
  g_err.clear();
  return HATT_OK;
}

// ---------------------------------------------------------------------------
// Largest width the tolerance mode grows a bond to: the truncation's SVD
// takes at most kSvdBigMaxN columns.
constexpr int64_t kAdaptMaxWidth = kSvdBigMaxN;

// Bytes kept at the end of the tolerance mode's workspace for ||X|| of each
// train's untruncated result.
static size_t xnorm_slot_bytes(int batch) { return ((size_t)batch * sizeof(double) + 255) & ~(size_t)255; }

// Tolerance-mode truncation at tol sqrt(3) / 2, with the captured range's
// error (||z||^2 - ||X||^2 of the untruncated projection X) held below tol / 2:
// the two are orthogonal, so together they stay within tol.  The capture
// check can only resolve errors whose square exceeds the rounding of the two
// squared norms, so its threshold is never below kCaptureFloor ||z||^2.
constexpr double kTruncShare = 0.8660254037844386;  // sqrt(3) / 2
constexpr double kCaptureShare2 = 0.25;             // (1 / 2)^2
constexpr double kCaptureFloor = 256.0 * 2.220446049250313e-16;

// cap: the largest feasible widths (a bond at its cap is exact); lim: the
// widths the growth may reach (cap clamped to kAdaptMaxWidth).
static hatt_status adapt_prepare(const hatt_tt *x, const hatt_tt *y, const hatt_tt *w, const hatt_adapt_opts *ao,
                                 HattSpec *sp,
                                 std::vector<int64_t> *cap, std::vector<int64_t> *lim, std::vector<int64_t> *ell0,
                                 int *p, int *maxa, bool need_data) {
  if (ao == nullptr) return fail(HATT_EINVAL, "adapt opts is NULL");
  if (!(ao->tol > 0.0) || !std::isfinite(ao->tol)) return fail(HATT_EINVAL, "tol must be finite and > 0");
  hatt_opts o{};
  o.variant = ao->variant ? ao->variant : 1;
  o.ep = ao->ep;
  o.ell = 1;
  o.tol = ao->tol;
  o.seed = ao->seed;
  o.precision = ao->precision;
  hatt_status st = hatt_prepare(x, y, w, &o, sp, need_data);
  if (st != HATT_OK) return st;
  const int d = sp->X.d;
  *p = ao->oversample > 0 ? ao->oversample : 8;
  *maxa = ao->max_attempts > 0 ? ao->max_attempts : 8;
  std::vector<int64_t> big(d + 1, (int64_t)1 << 40), req(d + 1, 1);
  *cap = clamp_ell(sp->X.n, sp->X.r, sp->ryw, big);
  std::vector<int64_t> lreq(d + 1, kAdaptMaxWidth);
  *lim = clamp_ell(sp->X.n, sp->X.r, sp->ryw, lreq);
  for (int k = 1; k < d; ++k) {
    int64_t rmax = std::max(sp->X.r[k], sp->Y.r[k]);
    if (sp->three) rmax = std::max(rmax, sp->W.r[k]);
    req[k] = std::min(rmax + *p, kAdaptMaxWidth);
  }
  if (ao->ell_init != nullptr)
    for (int k = 1; k < d; ++k) req[k] = std::min(ao->ell_init[k], kAdaptMaxWidth);
  *ell0 = clamp_ell(sp->X.n, sp->X.r, sp->ryw, req);
  return HATT_OK;
}

// One decision of the tolerance rule for the P trains of one recompression
// at widths sp.ell: the bonds to grow, or a switch of the range finding to
// FP64 (neither: accept).  kept holds the kept ranks [P][d+1]; z2 and xn hold
// ||z||^2 and ||X|| per train (read only with `capture`).  Slack test: a bond
// below its cap keeps at most l_k - p.  A capture failure grows every bond
// below its cap; with every bond at its cap the sketch spans the product's
// range exactly up to the rounding of the sketches, so a failure there under
// FP32 or BF16 range finding is that rounding, and the next attempt runs in
// FP64.
struct AdaptStep {
  std::vector<int> grow;
  bool to_fp64 = false;
  bool accept() const { return grow.empty() && !to_fp64; }
};

static AdaptStep adapt_decide(const HattSpec &sp, const std::vector<int64_t> &cap, int p, const int64_t *kept,
                              bool capture, const double *z2, const double *xn, double tol) {
  const int d = sp.X.d, P = sp.X.batch;
  AdaptStep step;
  std::vector<int> &bad = step.grow;
  for (int k = 1; k < d; ++k) {
    bool b = false;
    for (int q = 0; q < P; ++q)
      if (kept[(size_t)q * (d + 1) + k] > sp.ell[k] - p && sp.ell[k] < cap[k]) b = true;
    if (b) bad.push_back(k);
  }
  // the captured range: ||z - X||^2 = ||z||^2 - ||X||^2 (X is an orthogonal
  // projection of z); when it exceeds (tol / 2)^2 ||z||^2 every bond below
  // its cap grows
  bool capture_bad = false;
  if (capture)
    for (int q = 0; q < P; ++q) {
      const double c2 = std::max(0.0, z2[q] - xn[q] * xn[q]);
      if (c2 > std::max(kCaptureShare2 * tol * tol, kCaptureFloor) * z2[q]) capture_bad = true;
    }
  if (bad.empty() && capture_bad) {
    for (int k = 1; k < d; ++k)
      if (sp.ell[k] < cap[k]) bad.push_back(k);
    if (bad.empty() && sp.o.precision != 0) step.to_fp64 = true;
  }
  return step;
}

// Growth of the failing bonds: l_k = min(lim_k, ceil(1.5 l_k) + p); a bond
// already at lim_k cannot grow (HATT_ENOTCONV).
static hatt_status adapt_grow(const std::vector<int64_t> &cur, const std::vector<int> &bad,
                              const std::vector<int64_t> &lim, int p, std::vector<int64_t> *ell) {
  *ell = cur;
  for (int k : bad) {
    if (cur[k] >= lim[k])
      return fail(HATT_ENOTCONV, "bond " + std::to_string(k) + " needs a sketch wider than " +
                                     std::to_string(lim[k]) + " (the truncation's SVD limit)");
    (*ell)[k] = std::min<int64_t>(lim[k], (int64_t)std::ceil(1.5 * (double)cur[k]) + p);
  }
  return HATT_OK;
}

static hatt_status adaptive_plan_common(const hatt_tt *x, const hatt_tt *y, const hatt_tt *w,
                                        const hatt_adapt_opts *opts, int64_t *cap_out, size_t *ws_bytes,
                                        int64_t *out_elems) {
  HattSpec sp{};
  std::vector<int64_t> cap_true, cap, ell0;
  int p, maxa;
  hatt_status st = adapt_prepare(x, y, w, opts, &sp, &cap_true, &cap, &ell0, &p, &maxa, false);
  if (st != HATT_OK) return st;
  sp.ell = cap;
  sp.sketch = nullptr;
  Ws ws(nullptr);
  st = hatt_run(false, sp, ws, nullptr);
  if (st != HATT_OK) return st;
  if (sp.o.precision != 0) {
    // a capture failure at the caps switches the attempts to FP64
    HattSpec s64 = sp;
    s64.o.precision = 0;
    Ws w64(nullptr);
    st = hatt_run(false, s64, w64, nullptr);
    if (st != HATT_OK) return st;
    ws.off = std::max(ws.off, w64.off);
  }
  if (cap_out)
    for (int k = 0; k <= sp.X.d; ++k) cap_out[k] = cap[k];
  // widths below the caps need no more than the caps' buffers up to the
  // integer effects of the QR tree shapes; keep a margin and re-check per
  // attempt.  Two factors also need ||x (.) y||^2 (run before the attempts,
  // in the same memory) and a slot for ||X|| at the end of the workspace.
  size_t need = ws.off + ws.off / 8 + ((size_t)4 << 20);
  if (!sp.three) {
    Ws wn(nullptr);
    GemmCtx gm{nullptr, 0, 0};
    st = hadamard_norm2_body(false, sp.X, sp.Y, nullptr, wn, gm, nullptr);
    if (st != HATT_OK) return st;
    need = std::max(need, wn.off) + xnorm_slot_bytes(sp.X.batch);
  }
  if (ws_bytes) *ws_bytes = need;
  if (out_elems) {
    std::vector<int64_t> off;
    int64_t tot;
    make_offsets(sp.X.n, cap, &off, &tot);
    *out_elems = tot;
  }
  g_err.clear();
  return HATT_OK;
}

static hatt_status adaptive_common(const hatt_tt *x, const hatt_tt *y, const hatt_tt *w3,
                                   const hatt_adapt_opts *opts, double *out, int64_t out_stride, int64_t *out_rank,
                                   int64_t *ell_out, int32_t *attempts_out, void *ws, size_t ws_bytes, void *stream) {
  HattSpec sp{};
  std::vector<int64_t> cap, lim, ell;
  int p, maxa;
  hatt_status st = adapt_prepare(x, y, w3, opts, &sp, &cap, &lim, &ell, &p, &maxa, true);
  if (st != HATT_OK) return st;
  if (out == nullptr || out_rank == nullptr || ell_out == nullptr || attempts_out == nullptr)
    return fail(HATT_EINVAL, "NULL output argument");
  const int d = sp.X.d, P = sp.X.batch;
  std::vector<int64_t> coff;
  int64_t ctot;
  make_offsets(sp.X.n, lim, &coff, &ctot);
  if (out_stride != 0 && out_stride < ctot) return fail(HATT_EINVAL, "out_stride smaller than the planned slot");
  sp.out = out;
  sp.ostride = out_stride ? out_stride : ctot;
  sp.orank = out_rank;
  sp.sketch = nullptr;
  hipStream_t strm = (hipStream_t)stream;
  std::vector<int64_t> host_rank((size_t)P * (d + 1));
  {
    // non-finite inputs: the rank decisions below would be meaningless.
    // The flags of the factors borrow out_rank (>= 2 P int64 slots, so room
    // for 3 P ints) until the first attempt.
    int *fl = reinterpret_cast<int *>(out_rank);
    const bool run = true;
    hipStream_t st = strm;
    const int nf = sp.three ? 3 : 2;
    LAUNCH(launch_finite_check(sp.X.data, sp.X.total, sp.X.stride, P, fl, st));
    LAUNCH(launch_finite_check(sp.Y.data, sp.Y.total, sp.Y.stride, P, fl + P, st));
    if (sp.three) LAUNCH(launch_finite_check(sp.W.data, sp.W.total, sp.W.stride, P, fl + 2 * P, st));
    std::vector<int> hf((size_t)nf * P);
    if (hipMemcpyAsync(hf.data(), fl, hf.size() * sizeof(int), hipMemcpyDeviceToHost, strm) != hipSuccess ||
        hipStreamSynchronize(strm) != hipSuccess)
      return fail(HATT_EDEVICE, "reading the finiteness flags failed");
    static const char *kNames[3] = {"x", "y", "w"};
    for (int q = 0; q < nf * P; ++q)
      if (hf[q] != 1)
        return fail(HATT_ENONFINITE, std::string(kNames[q / P]) + " train " + std::to_string(q % P) +
                                         " has a non-finite entry");
  }
  // two factors: ||x (.) y||^2 of every train for the capture check, the
  // truncation at tol sqrt(3) / 2, and ||X|| in a slot at the workspace's end
  const bool capture = !sp.three && d >= 2;
  const double tol = opts->tol;
  std::vector<double> z2((size_t)P, 0.0), xn((size_t)P, 0.0);
  size_t ws_att = ws_bytes;
  if (capture) {
    const size_t slot = xnorm_slot_bytes(P);
    if (ws == nullptr || ws_bytes < slot) return fail(HATT_EWORKSPACE, "workspace too small");
    ws_att = ws_bytes - slot;
    sp.xnorm = reinterpret_cast<double *>(static_cast<char *>(ws) + ws_att);
    sp.o.tol = tol * kTruncShare;
    Ws meas(nullptr);
    GemmCtx gm{nullptr, 0, 0};
    st = hadamard_norm2_body(false, sp.X, sp.Y, nullptr, meas, gm, nullptr);
    if (st != HATT_OK) return st;
    if (ws_att < meas.off)
      return fail(HATT_EWORKSPACE, "workspace too small: need " + std::to_string(meas.off + slot) + " bytes");
    Ws wn(ws);
    st = hadamard_norm2_body(true, sp.X, sp.Y, sp.xnorm, wn, gm, strm);
    if (st != HATT_OK) return st;
    if (hipMemcpyAsync(z2.data(), sp.xnorm, z2.size() * sizeof(double), hipMemcpyDeviceToHost, strm) != hipSuccess ||
        hipStreamSynchronize(strm) != hipSuccess)
      return fail(HATT_EDEVICE, "reading ||x (.) y|| failed");
  }
  for (int attempt = 0; attempt < maxa; ++attempt) {
    sp.ell = clamp_ell(sp.X.n, sp.X.r, sp.ryw, ell);
    sp.o.seed = opts->seed + (uint64_t)attempt;
    Ws meas(nullptr);
    st = hatt_run(false, sp, meas, nullptr);
    if (st != HATT_OK) return st;
    if (ws == nullptr || ws_att < meas.off)
      return fail(HATT_EWORKSPACE, "workspace too small: need " + std::to_string(meas.off) + " bytes");
    Ws w(ws);
    st = hatt_run(true, sp, w, strm);
    if (st != HATT_OK) return st;
    if (hipMemcpyAsync(host_rank.data(), out_rank, host_rank.size() * sizeof(int64_t), hipMemcpyDeviceToHost,
                       strm) != hipSuccess ||
        (capture &&
         hipMemcpyAsync(xn.data(), sp.xnorm, xn.size() * sizeof(double), hipMemcpyDeviceToHost, strm) != hipSuccess) ||
        hipStreamSynchronize(strm) != hipSuccess)
      return fail(HATT_EDEVICE, "reading the kept ranks failed");
    const AdaptStep step = adapt_decide(sp, cap, p, host_rank.data(), capture, z2.data(), xn.data(), tol);
    for (int k = 0; k <= d; ++k) ell_out[k] = sp.ell[k];
    *attempts_out = attempt + 1;
    if (step.accept()) {
      g_err.clear();
      return HATT_OK;
    }
    if (step.to_fp64) sp.o.precision = 0;
    st = adapt_grow(sp.ell, step.grow, lim, p, &ell);
    if (st != HATT_OK) return st;
  }
  return fail(HATT_ENOTCONV, "sketch widths did not converge within max_attempts");
}

hatt_status hatt_adaptive_plan(const hatt_tt *x, const hatt_tt *y, const hatt_adapt_opts *opts, int64_t *cap_out,
                               size_t *ws_bytes, int64_t *out_elems) {
  return adaptive_plan_common(x, y, nullptr, opts, cap_out, ws_bytes, out_elems);
}

hatt_status hatt_recompress_adaptive(const hatt_tt *x, const hatt_tt *y, const hatt_adapt_opts *opts, double *out,
                                     int64_t out_stride, int64_t *out_rank, int64_t *ell_out, int32_t *attempts_out,
                                     void *ws, size_t ws_bytes, void *stream) {
  return adaptive_common(x, y, nullptr, opts, out, out_stride, out_rank, ell_out, attempts_out, ws, ws_bytes, stream);
}

hatt_status hatt_adaptive_plan3(const hatt_tt *x, const hatt_tt *y, const hatt_tt *w, const hatt_adapt_opts *opts,
                                int64_t *cap_out, size_t *ws_bytes, int64_t *out_elems) {
  if (w == nullptr) return fail(HATT_EINVAL, "w: NULL tensor view");
  return adaptive_plan_common(x, y, w, opts, cap_out, ws_bytes, out_elems);
}

hatt_status hatt_recompress3_adaptive(const hatt_tt *x, const hatt_tt *y, const hatt_tt *w,
                                      const hatt_adapt_opts *opts, double *out, int64_t out_stride,
                                      int64_t *out_rank, int64_t *ell_out, int32_t *attempts_out, void *ws,
                                      size_t ws_bytes, void *stream) {
  if (w == nullptr) return fail(HATT_EINVAL, "w: NULL tensor view");
  return adaptive_common(x, y, w, opts, out, out_stride, out_rank, ell_out, attempts_out, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------------------
// Tolerance mode over an uneven batch.  Every pair follows the rule of
// hatt_recompress_adaptive with its own widths; an attempt round runs the
// attempts of all pairs not yet accepted at once on the library streams and
// ends with one host synchronisation, after which the decision of each pair
// is taken from its kept ranks and ||X|| (copied back together for the whole
// batch).  The workspace begins with a header (||z||^2, ||X|| and finiteness
// flags of every train); the rest is carved per round into one region per
// stream, as large as the largest pair that stream runs in that round, with
// fewer streams when the regions would not fit.
struct BatchAdapt {
  std::vector<HattSpec> sp;
  std::vector<std::vector<int64_t>> cap, lim, ell;
  std::vector<int64_t> out_off, rank_off, train_off;
  std::vector<bool> capture;
  int p = 8, maxa = 8;
  size_t header = 0;
  size_t need_min = 0;   // one region that fits any pair's attempt and its ||z|| pass
  size_t need_full = 0;  // regions for the min(npairs, streams) largest pairs
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static hatt_status batch_adapt_prepare(int32_t npairs, const hatt_tt *x, const hatt_tt *y, const hatt_adapt_opts *ao,
                                       bool need_data, BatchAdapt *ba) {
  if (npairs < 1) return fail(HATT_EINVAL, "npairs must be >= 1");
  if (x == nullptr || y == nullptr || ao == nullptr) return fail(HATT_EINVAL, "NULL argument");
  ba->sp.assign(npairs, HattSpec{});
  ba->cap.assign(npairs, {});
  ba->lim.assign(npairs, {});
  ba->ell.assign(npairs, {});
  ba->capture.assign(npairs, false);
  ba->out_off.assign(npairs + 1, 0);
  ba->rank_off.assign(npairs + 1, 0);
  ba->train_off.assign(npairs + 1, 0);
  std::vector<size_t> need(npairs, 0);
  int64_t eoff = 0;
  for (int32_t q = 0; q < npairs; ++q) {
    hatt_adapt_opts o = *ao;
    o.seed = ao->seed + (uint64_t)q;
    if (ao->ell_init != nullptr) {
      if (x[q].d < 1) return fail(HATT_ESHAPE, "pair " + std::to_string(q) + ": bad order");
      o.ell_init = ao->ell_init + eoff;
      eoff += x[q].d + 1;
    }
    HattSpec &sp = ba->sp[q];
    hatt_status st = adapt_prepare(&x[q], &y[q], nullptr, &o, &sp, &ba->cap[q], &ba->lim[q], &ba->ell[q], &ba->p,
                                   &ba->maxa, need_data);
    if (st != HATT_OK) return fail(st, "pair " + std::to_string(q) + ": " + g_err);
    sp.o.seed = o.seed;
    sp.sketch = nullptr;
    ba->capture[q] = sp.X.d >= 2;
    // any attempt: the buffers at the growth limit, with the single-pair
    // margin; the ||x (.) y|| pass runs in the same region before the attempts
    HattSpec at = sp;
    at.ell = ba->lim[q];
    Ws meas(nullptr);
    st = hatt_run(false, at, meas, nullptr);
    if (st != HATT_OK) return fail(st, "pair " + std::to_string(q) + ": " + g_err);
    if (at.o.precision != 0) {
      // a capture failure at the caps switches the attempts to FP64
      at.o.precision = 0;
      Ws w64(nullptr);
      st = hatt_run(false, at, w64, nullptr);
      if (st != HATT_OK) return fail(st, "pair " + std::to_string(q) + ": " + g_err);
      meas.off = std::max(meas.off, w64.off);
    }
    size_t nd = meas.off + meas.off / 8 + ((size_t)4 << 20);
    if (ba->capture[q]) {
      Ws wn(nullptr);
      GemmCtx gm{nullptr, 0, 0};
      st = hadamard_norm2_body(false, sp.X, sp.Y, nullptr, wn, gm, nullptr);
      if (st != HATT_OK) return fail(st, "pair " + std::to_string(q) + ": " + g_err);
      nd = std::max(nd, wn.off);
    }
    need[q] = align256(nd);
    std::vector<int64_t> off;
    int64_t tot;
    make_offsets(sp.X.n, ba->lim[q], &off, &tot);
    sp.ostride = tot;
    ba->out_off[q + 1] = ba->out_off[q] + tot * sp.X.batch;
    ba->rank_off[q + 1] = ba->rank_off[q] + (int64_t)sp.X.batch * (sp.X.d + 1);
    ba->train_off[q + 1] = ba->train_off[q] + sp.X.batch;
  }
  const int64_t T = ba->train_off[npairs];
  ba->header = 2 * align256((size_t)T * sizeof(double)) + align256((size_t)T * 2 * sizeof(int));
  std::vector<size_t> sorted = need;
  std::sort(sorted.begin(), sorted.end(), std::greater<size_t>());
  ba->need_min = ba->header + sorted[0];
  size_t full = ba->header;
  for (int k = 0; k < std::min<int>(npairs, kBatchStreams); ++k) full += sorted[k];
  ba->need_full = full;
  return HATT_OK;
}

// Streams and regions of one round: pairs `todo` with workspace needs `need`
// onto at most kBatchStreams streams, longest first onto the least loaded;
// regions as large as the largest pair of their stream, the stream count
// lowered until the regions fit in `avail` bytes.
static hatt_status batch_adapt_carve(const std::vector<int> &todo, const std::vector<double> &cost,
                                     const std::vector<size_t> &need, size_t avail, std::vector<int> *stream_of,
                                     std::vector<size_t> *region_off, int *streams) {
  std::vector<int> order(todo);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  for (int S = std::min<int>((int)todo.size(), kBatchStreams); S >= 1; --S) {
    std::vector<double> load(S, 0.0);
    std::vector<size_t> reg(S, 0);
    for (int q : order) {
      int k = 0;
      for (int t = 1; t < S; ++t)
        if (load[t] < load[k]) k = t;
      (*stream_of)[q] = k;
      load[k] += cost[q];
      reg[k] = std::max(reg[k], need[q]);
    }
    size_t tot = 0;
    region_off->assign(S + 1, 0);
    for (int k = 0; k < S; ++k) {
      (*region_off)[k] = tot;
      tot += reg[k];
    }
    (*region_off)[S] = tot;
    if (tot <= avail) {
      *streams = S;
      return HATT_OK;
    }
  }
  size_t big = 0;
  for (int q : todo) big = std::max(big, need[q]);
  return fail(HATT_EWORKSPACE, "workspace too small: a round needs " + std::to_string(big) +
                                   " bytes after the header, " + std::to_string(avail) + " available");
}

hatt_status hatt_batched_adaptive_plan(int32_t npairs, const hatt_tt *x, const hatt_tt *y,
                                       const hatt_adapt_opts *opts, int64_t *out_offset, int64_t *rank_offset,
                                       int64_t *cap_out, size_t *ws_min, size_t *ws_full) {
  BatchAdapt ba;
  hatt_status st = batch_adapt_prepare(npairs, x, y, opts, false, &ba);
  if (st != HATT_OK) return st;
  if (out_offset)
    for (int32_t q = 0; q <= npairs; ++q) out_offset[q] = ba.out_off[q];
  if (rank_offset)
    for (int32_t q = 0; q <= npairs; ++q) rank_offset[q] = ba.rank_off[q];
  if (cap_out) {
    int64_t e = 0;
    for (int32_t q = 0; q < npairs; ++q)
      for (int64_t v : ba.lim[q]) cap_out[e++] = v;
  }
  if (ws_min) *ws_min = ba.need_min;
  if (ws_full) *ws_full = ba.need_full;
  g_err.clear();
  return HATT_OK;
}

hatt_status hatt_recompress_batched_adaptive(int32_t npairs, const hatt_tt *x, const hatt_tt *y,
                                             const hatt_adapt_opts *opts, double *out, int64_t *out_rank,
                                             int64_t *ell_out, int32_t *attempts_out, void *ws, size_t ws_bytes,
                                             void *stream) {
  BatchAdapt ba;
  hatt_status st = batch_adapt_prepare(npairs, x, y, opts, true, &ba);
  if (st != HATT_OK) return st;
  if (out == nullptr || out_rank == nullptr || ell_out == nullptr || attempts_out == nullptr)
    return fail(HATT_EINVAL, "NULL output argument");
  if (ws == nullptr || ws_bytes < ba.need_min)
    return fail(HATT_EWORKSPACE, "workspace too small: need at least " + std::to_string(ba.need_min) + " bytes");
  hipStream_t caller = (hipStream_t)stream;
  hipStreamCaptureStatus capst = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(caller, &capst) != hipSuccess) return fail(HATT_EDEVICE, "hipStreamIsCapturing failed");
  if (capst != hipStreamCaptureStatusNone)
    return fail(HATT_EUNSUPPORTED, "the tolerance mode synchronises per round and cannot be captured");
  std::lock_guard<std::mutex> lock(g_batch_mu);
  BatchStreams *bs = nullptr;
  st = batch_streams(&bs);
  if (st != HATT_OK) return st;
  const int64_t T = ba.train_off[npairs];
  char *base = static_cast<char *>(ws);
  double *z2d = reinterpret_cast<double *>(base);
  double *xnd = reinterpret_cast<double *>(base + align256((size_t)T * sizeof(double)));
  int *fld = reinterpret_cast<int *>(base + 2 * align256((size_t)T * sizeof(double)));
  char *arena = base + ba.header;
  const size_t avail = ws_bytes - ba.header;
  std::vector<int> stream_of(npairs, 0);
  std::vector<size_t> region;
  std::vector<double> cost(npairs, 0.0);
  std::vector<size_t> need(npairs, 0);
  int S = 1;
  auto fork = [&](int nstreams) -> hatt_status {
    if (hipEventRecord(bs->fork, caller) != hipSuccess) return fail(HATT_EDEVICE, "event record failed");
    for (int k = 0; k < nstreams; ++k)
      if (hipStreamWaitEvent(bs->s[k], bs->fork, 0) != hipSuccess) return fail(HATT_EDEVICE, "stream wait failed");
    return HATT_OK;
  };
  auto join = [&](int nstreams) -> hatt_status {
    for (int k = 0; k < nstreams; ++k) {
      if (hipEventRecord(bs->join[k], bs->s[k]) != hipSuccess) return fail(HATT_EDEVICE, "event record failed");
      if (hipStreamWaitEvent(caller, bs->join[k], 0) != hipSuccess) return fail(HATT_EDEVICE, "stream wait failed");
    }
    return HATT_OK;
  };
  std::vector<int> todo(npairs);
  for (int32_t q = 0; q < npairs; ++q) todo[q] = q;

  // set-up round: finiteness of x and y, then ||x (.) y||^2 per train
  std::vector<double> z2((size_t)T, 0.0), xn((size_t)T, 0.0);
  {
    for (int q : todo) {
      Ws wn(nullptr);
      GemmCtx gm{nullptr, 0, 0};
      if (ba.capture[q]) {
        st = hadamard_norm2_body(false, ba.sp[q].X, ba.sp[q].Y, nullptr, wn, gm, nullptr);
        if (st != HATT_OK) return fail(st, "pair " + std::to_string(q) + ": " + g_err);
      }
      need[q] = align256(std::max<size_t>(wn.off, 256));
      cost[q] = batch_pair_cost(ba.sp[q]);
    }
    st = batch_adapt_carve(todo, cost, need, avail, &stream_of, &region, &S);
    if (st != HATT_OK) return st;
    st = fork(S);
    if (st != HATT_OK) return st;
    st = batch_enqueue(S, todo, stream_of, batch_threaded(capst), bs->device, [&](int q, int k) -> hatt_status {
      const HattSpec &sp = ba.sp[q];
      const bool run = true;
      int *fl = fld + 2 * ba.train_off[q];
      const int P = sp.X.batch;
      hipStream_t st = bs->s[k];
      LAUNCH(launch_finite_check(sp.X.data, sp.X.total, sp.X.stride, P, fl, st));
      LAUNCH(launch_finite_check(sp.Y.data, sp.Y.total, sp.Y.stride, P, fl + P, st));
      if (!ba.capture[q]) return HATT_OK;
      Ws wn(arena + region[k]);
      GemmCtx gm{nullptr, 0, 0};
      return hadamard_norm2_body(true, sp.X, sp.Y, z2d + ba.train_off[q], wn, gm, st);
    });
    if (st != HATT_OK) return st;
    st = join(S);
    if (st != HATT_OK) return st;
    std::vector<int> hf((size_t)2 * T);
    if (hipMemcpyAsync(hf.data(), fld, hf.size() * sizeof(int), hipMemcpyDeviceToHost, caller) != hipSuccess ||
        hipMemcpyAsync(z2.data(), z2d, z2.size() * sizeof(double), hipMemcpyDeviceToHost, caller) != hipSuccess ||
        hipStreamSynchronize(caller) != hipSuccess)
      return fail(HATT_EDEVICE, "reading the finiteness flags and ||x (.) y|| failed");
    for (int q : todo) {
      const int P = ba.sp[q].X.batch;
      for (int t = 0; t < 2 * P; ++t)
        if (hf[2 * ba.train_off[q] + t] != 1)
          return fail(HATT_ENONFINITE, "pair " + std::to_string(q) + ": " + (t < P ? "x" : "y") + " train " +
                                           std::to_string(t % P) + " has a non-finite entry");
    }
  }

  // attempt rounds
  const double tol = opts->tol;
  std::vector<int64_t> host_rank((size_t)ba.rank_off[npairs]);
  std::vector<std::vector<int64_t>> used(npairs);
  std::string stuck;
  int nstuck = 0;
  for (int attempt = 0; attempt < ba.maxa && !todo.empty(); ++attempt) {
    for (int q : todo) {
      HattSpec &sp = ba.sp[q];
      sp.ell = clamp_ell(sp.X.n, sp.X.r, sp.ryw, ba.ell[q]);
      sp.o.seed = opts->seed + (uint64_t)q + (uint64_t)attempt;
      sp.o.tol = ba.capture[q] ? tol * kTruncShare : tol;
      sp.out = out + ba.out_off[q];
      sp.orank = out_rank + ba.rank_off[q];
      sp.xnorm = ba.capture[q] ? xnd + ba.train_off[q] : nullptr;
      Ws meas(nullptr);
      st = hatt_run(false, sp, meas, nullptr);
      if (st != HATT_OK) return fail(st, "pair " + std::to_string(q) + ": " + g_err);
      need[q] = align256(std::max<size_t>(meas.off, 256));
      cost[q] = batch_pair_cost(sp);
    }
    st = batch_adapt_carve(todo, cost, need, avail, &stream_of, &region, &S);
    if (st != HATT_OK) return st;
    st = fork(S);
    if (st != HATT_OK) return st;
    // largest first, so each stream starts with its costliest pair
    std::vector<int> order(todo);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    st = batch_enqueue(S, order, stream_of, batch_threaded(capst), bs->device, [&](int q, int k) {
      Ws w(arena + region[k]);
      return hatt_run(true, ba.sp[q], w, bs->s[k]);
    });
    if (st != HATT_OK) return st;
    st = join(S);
    if (st != HATT_OK) return st;
    if (hipMemcpyAsync(host_rank.data(), out_rank, host_rank.size() * sizeof(int64_t), hipMemcpyDeviceToHost,
                       caller) != hipSuccess ||
        hipMemcpyAsync(xn.data(), xnd, xn.size() * sizeof(double), hipMemcpyDeviceToHost, caller) != hipSuccess ||
        hipStreamSynchronize(caller) != hipSuccess)
      return fail(HATT_EDEVICE, "reading the kept ranks failed");
    // a pair whose failing bond cannot grow stops there (its last result in
    // place); the others go on
    std::vector<int> next;
    for (int q : todo) {
      const HattSpec &sp = ba.sp[q];
      const AdaptStep step =
          adapt_decide(sp, ba.cap[q], ba.p, host_rank.data() + ba.rank_off[q], ba.capture[q],
                       z2.data() + ba.train_off[q], xn.data() + ba.train_off[q], tol);
      used[q] = sp.ell;
      attempts_out[q] = attempt + 1;
      if (step.accept()) continue;
      if (step.to_fp64) ba.sp[q].o.precision = 0;
      if (adapt_grow(sp.ell, step.grow, ba.lim[q], ba.p, &ba.ell[q]) != HATT_OK) {
        if (stuck.empty()) stuck = "pair " + std::to_string(q) + ": " + g_err;
        ++nstuck;
        continue;
      }
      next.push_back(q);
    }
    todo.swap(next);
  }
  int64_t e = 0;
  for (int32_t q = 0; q < npairs; ++q)
    for (int64_t v : used[q]) ell_out[e++] = v;
  if (!stuck.empty())
    return fail(HATT_ENOTCONV, stuck + " (" + std::to_string(nstuck) + " pairs at the width limit, " +
                                   std::to_string(todo.size()) + " out of attempts)");
  if (!todo.empty())
    return fail(HATT_ENOTCONV, "pair " + std::to_string(todo[0]) + ": sketch widths did not converge within " +
                                   "max_attempts (" + std::to_string(todo.size()) + " pairs unconverged)");
  g_err.clear();
  return HATT_OK;
}

hatt_status tt_hadamard_explicit(const hatt_tt *x, const hatt_tt *y, double *out, int64_t out_stride,
                                 void *stream) {
  Shape X, Y;
  hatt_status rc = read_tt(x, "x", &X, true);
  if (rc != HATT_OK) return rc;
  rc = read_tt(y, "y", &Y, true);
  if (rc != HATT_OK) return rc;
  if (X.d != Y.d || X.batch != Y.batch || X.n != Y.n) return fail(HATT_ESHAPE, "x and y shapes differ");
  if (out == nullptr) return fail(HATT_EINVAL, "out is NULL");
  std::vector<int64_t> rr(X.d + 1), off;
  for (int k = 0; k <= X.d; ++k) rr[k] = X.r[k] * Y.r[k];
  int64_t tot;
  make_offsets(X.n, rr, &off, &tot);
  if (out_stride != 0 && out_stride < tot) return fail(HATT_EINVAL, "out_stride smaller than one output train");
  const int64_t os = out_stride ? out_stride : tot;
  const bool run = true;
  hipStream_t st = (hipStream_t)stream;
  for (int k = 0; k < X.d; ++k) {
    PkpArgs pa{X.data + X.off[k], Y.data + Y.off[k], out + off[k], X.r[k], X.r[k + 1], Y.r[k], Y.r[k + 1],
               X.n[k], X.stride, Y.stride, os, X.batch};
    LAUNCH(launch_pkp(pa, st));
  }
  g_err.clear();
  return HATT_OK;
}

static hatt_status round_prepare(const hatt_tt *a, RoundSpec *rs, Shape *A, bool need_data) {
  hatt_status st = read_tt(a, "a", A, need_data);
  if (st != HATT_OK) return st;
  rs->n = A->n;
  rs->rin = A->r;
  rs->cap = round_caps(A->n, A->r);
  rs->src = A->data;
  rs->sstride = A->stride;
  rs->in_place = false;
  rs->batch = A->batch;
  return HATT_OK;
}

hatt_status tt_round_plan(const hatt_tt *a, int64_t *cap_out, size_t *ws_bytes, int64_t *out_elems) {
  RoundSpec rs{};
  Shape A;
  hatt_status st = round_prepare(a, &rs, &A, false);
  if (st != HATT_OK) return st;
  rs.norm_only = false;
  Ws ws(nullptr);
  GemmCtx gm{nullptr, 0, 0};
  st = round_run(false, rs, ws, gm, nullptr);
  if (st != HATT_OK) return st;
  if (cap_out)
    for (int k = 0; k <= A.d; ++k) cap_out[k] = rs.cap[k];
  if (ws_bytes) *ws_bytes = ws.off;
  if (out_elems) {
    std::vector<int64_t> off;
    int64_t tot;
    make_offsets(A.n, rs.cap, &off, &tot);
    *out_elems = tot;
  }
  g_err.clear();
  return HATT_OK;
}

hatt_status tt_round(const hatt_tt *a, int64_t max_rank, double tol, double *out, int64_t out_stride,
                     int64_t *out_rank, void *ws, size_t ws_bytes, void *stream) {
  RoundSpec rs{};
  Shape A;
  hatt_status st = round_prepare(a, &rs, &A, true);
  if (st != HATT_OK) return st;
  if (out == nullptr || out_rank == nullptr) return fail(HATT_EINVAL, "out or out_rank is NULL");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(HATT_EINVAL, "tol must be finite and >= 0");
  std::vector<int64_t> off;
  int64_t otot;
  make_offsets(A.n, rs.cap, &off, &otot);
  if (out_stride != 0 && out_stride < otot) return fail(HATT_EINVAL, "out_stride smaller than one output train");
  rs.out = out;
  rs.ostride = out_stride ? out_stride : otot;
  rs.orank = out_rank;
  rs.max_rank = max_rank;
  rs.tol = tol;
  Ws meas(nullptr);
  GemmCtx gm{nullptr, 0, 0};
  st = round_run(false, rs, meas, gm, nullptr);
  if (st != HATT_OK) return st;
  if (ws == nullptr || ws_bytes < meas.off)
    return fail(HATT_EWORKSPACE, "workspace too small: need " + std::to_string(meas.off) + " bytes");
  Ws w(ws);
  GemmCtx g2{nullptr, 0, 0};
  st = round_run(true, rs, w, g2, (hipStream_t)stream);
  if (st == HATT_OK) g_err.clear();
  return st;
}

hatt_status tt_norm_plan(const hatt_tt *a, size_t *ws_bytes) {
  RoundSpec rs{};
  Shape A;
  hatt_status st = round_prepare(a, &rs, &A, false);
  if (st != HATT_OK) return st;
  rs.norm_only = true;
  Ws ws(nullptr);
  GemmCtx gm{nullptr, 0, 0};
  st = round_run(false, rs, ws, gm, nullptr);
  if (st != HATT_OK) return st;
  if (ws_bytes) *ws_bytes = ws.off;
  g_err.clear();
  return HATT_OK;
}

hatt_status tt_norm(const hatt_tt *a, double *out, void *ws, size_t ws_bytes, void *stream) {
  RoundSpec rs{};
  Shape A;
  hatt_status st = round_prepare(a, &rs, &A, true);
  if (st != HATT_OK) return st;
  if (out == nullptr) return fail(HATT_EINVAL, "out is NULL");
  rs.norm_only = true;
  rs.norm_out = out;
  Ws meas(nullptr);
  GemmCtx gm{nullptr, 0, 0};
  st = round_run(false, rs, meas, gm, nullptr);
  if (st != HATT_OK) return st;
  if (ws == nullptr || ws_bytes < meas.off)
    return fail(HATT_EWORKSPACE, "workspace too small: need " + std::to_string(meas.off) + " bytes");
  Ws w(ws);
  GemmCtx g2{nullptr, 0, 0};
  st = round_run(true, rs, w, g2, (hipStream_t)stream);
  if (st == HATT_OK) g_err.clear();
  return st;
}

static hatt_status norm2_prepare(const hatt_tt *x, const hatt_tt *y, Shape *X, Shape *Y, bool need_data) {
  hatt_status st = read_tt(x, "x", X, need_data);
  if (st != HATT_OK) return st;
  st = read_tt(y, "y", Y, need_data);
  if (st != HATT_OK) return st;
  if (X->d != Y->d || X->n != Y->n || X->batch != Y->batch)
    return fail(HATT_ESHAPE, "x and y differ in order, mode sizes or batch");
  return HATT_OK;
}

hatt_status hatt_hadamard_norm2_plan(const hatt_tt *x, const hatt_tt *y, size_t *ws_bytes) {
  Shape X, Y;
  hatt_status st = norm2_prepare(x, y, &X, &Y, false);
  if (st != HATT_OK) return st;
  Ws meas(nullptr);
  GemmCtx gm{nullptr, 0, 0};
  st = hadamard_norm2_body(false, X, Y, nullptr, meas, gm, nullptr);
  if (st != HATT_OK) return st;
  if (ws_bytes) *ws_bytes = meas.off;
  g_err.clear();
  return HATT_OK;
}

hatt_status hatt_hadamard_norm2(const hatt_tt *x, const hatt_tt *y, double *out, void *ws, size_t ws_bytes,
                                void *stream) {
  Shape X, Y;
  hatt_status st = norm2_prepare(x, y, &X, &Y, true);
  if (st != HATT_OK) return st;
  if (out == nullptr) return fail(HATT_EINVAL, "out is NULL");
  Ws meas(nullptr);
  GemmCtx gm{nullptr, 0, 0};
  st = hadamard_norm2_body(false, X, Y, nullptr, meas, gm, nullptr);
  if (st != HATT_OK) return st;
  if (ws == nullptr || ws_bytes < meas.off)
    return fail(HATT_EWORKSPACE, "workspace too small: need " + std::to_string(meas.off) + " bytes");
  Ws w(ws);
  st = hadamard_norm2_body(true, X, Y, out, w, gm, (hipStream_t)stream);
  if (st == HATT_OK) g_err.clear();
  return st;
}

hatt_status tt_scale(const hatt_tt *a, const double *alpha, int32_t invert, void *stream) {
  Shape A;
  hatt_status rc = read_tt(a, "a", &A, true);
  if (rc != HATT_OK) return rc;
  if (alpha == nullptr) return fail(HATT_EINVAL, "alpha is NULL");
  if (invert != 0 && invert != 1) return fail(HATT_EINVAL, "invert must be 0 or 1");
  const bool run = true;
  hipStream_t st = (hipStream_t)stream;
  LAUNCH(launch_scale_by(A.data, A.r[0] * A.n[0] * A.r[1], A.stride, alpha, invert, A.batch, st));
  g_err.clear();
  return HATT_OK;
}

hatt_status tt_check_finite(const hatt_tt *a, int32_t *flag, void *stream) {
  Shape A;
  hatt_status rc = read_tt(a, "a", &A, true);
  if (rc != HATT_OK) return rc;
  if (flag == nullptr) return fail(HATT_EINVAL, "flag is NULL");
  const bool run = true;
  hipStream_t st = (hipStream_t)stream;
  LAUNCH(launch_finite_check(A.data, A.total, A.stride, A.batch, flag, st));
  g_err.clear();
  return HATT_OK;
}

hatt_status hatt_sketch_fill(uint64_t seed, int32_t d, const int64_t *n, const int64_t *ell, double *out,
                             void *stream) {
  if (d < 1 || n == nullptr || ell == nullptr || out == nullptr)
    return fail(HATT_EINVAL, "sketch_fill: bad arguments");
  if (ell[0] != 1 || ell[d] != 1) return fail(HATT_ESHAPE, "sketch_fill: ell[0] and ell[d] must be 1");
  int64_t off = 0;
  for (int k = 0; k < d; ++k) {
    if (n[k] < 1 || ell[k] < 1) return fail(HATT_ESHAPE, "sketch_fill: sizes must be >= 1");
  }
  const bool run = true;
  hipStream_t st = (hipStream_t)stream;
  for (int k = 0; k < d; ++k) {
    const int64_t cnt = ell[k] * n[k] * ell[k + 1];
    LAUNCH(launch_sketch_fill(seed, k, cnt, 1.0 / sqrt((double)cnt), out + off, st));
    off += cnt;
  }
  g_err.clear();
  return HATT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Learned start widths (hatt_rankpred_*).

static hatt_status rp_pairs(int32_t npairs, const hatt_tt *x, const hatt_tt *y, std::vector<Shape> *X,
                            std::vector<Shape> *Y, int64_t *rows, bool need_data) {
  if (npairs < 1) return fail(HATT_EINVAL, "npairs must be >= 1");
  if (x == nullptr || y == nullptr) return fail(HATT_EINVAL, "NULL argument");
  X->assign(npairs, Shape{});
  Y->assign(npairs, Shape{});
  *rows = 0;
  for (int32_t p = 0; p < npairs; ++p) {
    hatt_status st = read_tt(&x[p], "x", &(*X)[p], need_data);
    if (st == HATT_OK) st = read_tt(&y[p], "y", &(*Y)[p], need_data);
    if (st != HATT_OK) return fail(st, "pair " + std::to_string(p) + ": " + g_err);
    const Shape &a = (*X)[p], &b = (*Y)[p];
    if (a.d != b.d || a.n != b.n) return fail(HATT_ESHAPE, "pair " + std::to_string(p) + ": x and y shapes differ");
    for (int k = 1; k < a.d; ++k)
      if (a.r[k] > kRpMaxRank || b.r[k] > kRpMaxRank)
        return fail(HATT_EUNSUPPORTED, "pair " + std::to_string(p) + ": bond rank above 2048");
    *rows += a.d - 1;
  }
  return HATT_OK;
}

hatt_status hatt_rankpred_features(int32_t npairs, const hatt_tt *x, const hatt_tt *y, float *feat, void *stream) {
  std::vector<Shape> X, Y;
  int64_t rows;
  hatt_status st = rp_pairs(npairs, x, y, &X, &Y, &rows, true);
  if (st != HATT_OK) return st;
  if (feat == nullptr && rows > 0) return fail(HATT_EINVAL, "feat is NULL");
  const bool run = true;
  hipStream_t strm = (hipStream_t)stream;
  hipStream_t st_ = strm;
  int64_t row = 0;
  for (int32_t p = 0; p < npairs; ++p) {
    const Shape &a = X[p], &b = Y[p];
    for (int k0 = 1; k0 < a.d; k0 += kRpMaxBonds) {
      const int nb = std::min(kRpMaxBonds, a.d - k0);
      RpFeatArgs fa{};
      for (int t = 0; t < nb; ++t) {
        const int c = k0 + t - 1;  // 0-based core of bond k0 + t
        fa.cx[t] = a.data + a.off[c];
        fa.cy[t] = b.data + b.off[c];
        fa.rxp[t] = (int)a.r[c];
        fa.rxn[t] = (int)a.r[c + 1];
        fa.ryp[t] = (int)b.r[c];
        fa.ryn[t] = (int)b.r[c + 1];
        fa.n[t] = (int)a.n[c];
      }
      fa.k0 = k0;
      fa.d = a.d;
      fa.out = feat + (row + k0 - 1) * kRpIn;
      {
        hipStream_t st = st_;
        LAUNCH(launch_rp_features(fa, nb, st));
      }
    }
    row += a.d - 1;
  }
  g_err.clear();
  return HATT_OK;
}

hatt_status hatt_rankpred_fit_stats(const float *feat, const float *label, int64_t rows, float *stats, void *stream) {
  if (feat == nullptr || label == nullptr || stats == nullptr) return fail(HATT_EINVAL, "NULL argument");
  if (rows < 1) return fail(HATT_EINVAL, "rows must be >= 1");
  const bool run = true;
  hipStream_t st = (hipStream_t)stream;
  LAUNCH(launch_rp_stats(feat, label, rows, stats, st));
  g_err.clear();
  return HATT_OK;
}

hatt_status hatt_rankpred_forward(const float *theta, const float *stats, const float *feat, int64_t rows,
                                  float *pred, void *stream) {
  if (rows < 0) return fail(HATT_EINVAL, "rows must be >= 0");
  if (rows == 0) {
    g_err.clear();
    return HATT_OK;
  }
  if (theta == nullptr || stats == nullptr || feat == nullptr || pred == nullptr)
    return fail(HATT_EINVAL, "NULL argument");
  const bool run = true;
  hipStream_t st = (hipStream_t)stream;
  LAUNCH(launch_rp_forward(theta, stats, feat, rows, pred, st));
  g_err.clear();
  return HATT_OK;
}

size_t hatt_rankpred_ws_bytes(int64_t batch) {
  if (batch < 1) return 0;
  const int64_t nblk = (batch + kRpRowsPerBlock - 1) / kRpRowsPerBlock;
  return (size_t)nblk * (kRpTheta + 1) * sizeof(float);
}

static hatt_status rp_grad_common(const float *theta, const float *stats, const float *feat, const float *label,
                                  const int32_t *idx, int64_t batch, float *grad, float *loss, const RpAdam &ad,
                                  void *ws, size_t ws_bytes, void *stream) {
  if (theta == nullptr || stats == nullptr || feat == nullptr || label == nullptr || idx == nullptr)
    return fail(HATT_EINVAL, "NULL argument");
  if (batch < 1 || batch > ((int64_t)1 << 31)) return fail(HATT_EINVAL, "batch must be in [1, 2^31]");
  const size_t need = hatt_rankpred_ws_bytes(batch);
  if (ws == nullptr || ws_bytes < need)
    return fail(HATT_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  const int64_t nblk = (batch + kRpRowsPerBlock - 1) / kRpRowsPerBlock;
  float *part = (float *)ws;
  float *lpart = part + nblk * kRpTheta;
  const bool run = true;
  hipStream_t st = (hipStream_t)stream;
  LAUNCH(launch_rp_grad(theta, stats, feat, label, idx, batch, part, lpart, grad, loss, ad, st));
  g_err.clear();
  return HATT_OK;
}

hatt_status hatt_rankpred_grad(const float *theta, const float *stats, const float *feat, const float *label,
                               const int32_t *idx, int64_t batch, float *grad, float *loss, void *ws,
                               size_t ws_bytes, void *stream) {
  if (grad == nullptr) return fail(HATT_EINVAL, "grad is NULL");
  RpAdam ad{};
  return rp_grad_common(theta, stats, feat, label, idx, batch, grad, loss, ad, ws, ws_bytes, stream);
}

hatt_status hatt_rankpred_train_step(float *theta, float *adam_m, float *adam_v, int64_t step,
                                     const hatt_adam_opts *opts, const float *stats, const float *feat,
                                     const float *label, const int32_t *idx, int64_t batch, float *loss, void *ws,
                                     size_t ws_bytes, void *stream) {
  if (adam_m == nullptr || adam_v == nullptr) return fail(HATT_EINVAL, "NULL Adam state");
  if (step < 1) return fail(HATT_EINVAL, "step counts from 1");
  double lr = 1e-3, b1 = 0.9, b2 = 0.999, eps = 1e-8;
  if (opts != nullptr) {
    if (opts->lr > 0) lr = opts->lr;
    if (opts->beta1 > 0) b1 = opts->beta1;
    if (opts->beta2 > 0) b2 = opts->beta2;
    if (opts->eps > 0) eps = opts->eps;
  }
  if (!(b1 < 1.0) || !(b2 < 1.0)) return fail(HATT_EINVAL, "Adam betas must be < 1");
  RpAdam ad{theta, adam_m, adam_v, (float)lr, (float)b1, (float)b2, (float)eps,
            (float)(1.0 / (1.0 - std::pow(b1, (double)step))), (float)(1.0 / (1.0 - std::pow(b2, (double)step)))};
  return rp_grad_common(theta, stats, feat, label, idx, batch, nullptr, loss, ad, ws, ws_bytes, stream);
}

hatt_status hatt_rankpred_labels(int32_t d, const int64_t *kept, const int64_t *cap, int32_t oversample,
                                 float *out) {
  if (d < 1 || kept == nullptr || cap == nullptr || (out == nullptr && d > 1))
    return fail(HATT_EINVAL, "rankpred_labels: bad arguments");
  const int64_t p = oversample > 0 ? oversample : 8;
  for (int k = 1; k < d; ++k) {
    if (kept[k] < 1 || cap[k] < 1) return fail(HATT_EINVAL, "rankpred_labels: ranks and caps must be >= 1");
    out[2 * (k - 1)] = (float)std::log((double)kept[k]);
    out[2 * (k - 1) + 1] = (float)std::log((double)std::min(cap[k], kept[k] + p));
  }
  g_err.clear();
  return HATT_OK;
}

hatt_status hatt_rankpred_widths(int32_t npairs, const hatt_tt *x, const hatt_tt *y, const float *pred,
                                 double margin, int32_t oversample, int64_t *ell_out, int64_t *rho_out) {
  std::vector<Shape> X, Y;
  int64_t rows;
  hatt_status st = rp_pairs(npairs, x, y, &X, &Y, &rows, false);
  if (st != HATT_OK) return st;
  if (pred == nullptr || ell_out == nullptr) return fail(HATT_EINVAL, "NULL argument");
  if (!(margin >= 0.0) || !std::isfinite(margin)) return fail(HATT_EINVAL, "margin must be finite and >= 0");
  const int p = oversample > 0 ? oversample : 8;
  int64_t row = 0, e = 0;
  for (int32_t q = 0; q < npairs; ++q) {
    const Shape &a = X[q], &b = Y[q];
    const int d = a.d;
    std::vector<int64_t> req(d + 1, 1), rho(d + 1, 1);
    for (int k = 1; k < d; ++k, ++row) {
      const double la = (double)pred[2 * row], lb = (double)pred[2 * row + 1];
      if (!std::isfinite(la) || !std::isfinite(lb))
        return fail(HATT_ENONFINITE, "non-finite prediction in row " + std::to_string(row));
      const double w = std::max(std::exp(lb), std::exp(la) + (double)p);
      const double lw = std::ceil((1.0 + margin) * w), lr = std::ceil(std::exp(la));
      req[k] = (int64_t)std::max(1.0, std::min(lw, 9.0e15));
      rho[k] = (int64_t)std::max(1.0, std::min(lr, 9.0e15));
    }
    const std::vector<int64_t> ell = clamp_ell(a.n, a.r, b.r, req);
    for (int k = 0; k <= d; ++k, ++e) {
      ell_out[e] = ell[k];
      if (rho_out) rho_out[e] = rho[k];
    }
  }
  g_err.clear();
  return HATT_OK;
}
