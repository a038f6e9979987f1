// Host runtime and C ABI of libtucker_als: argument validation, workspace
// carving, the per-mode ALS loop (Algorithm 3.3 with the stop test of
// eq. E5.01), the t-/st-HOSVD-ALS drivers (Algorithms 3.4 / 3.5), TTM and
// Tucker reconstruction (Section 2).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "tk_kernels.h"

namespace tk {
namespace {

constexpr int NWG_MAX = 2048;     // upper bound on partial sums of one reduction
constexpr size_t ALIGN = 256;

inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

inline size_t dsize(int dt) { return dt == TK_F64 ? 8 : dt == TK_F32 ? 4 : 2; }
inline int cdtype(int dt) { return dt == TK_F64 ? TK_F64 : TK_F32; }

// Bump allocator over the caller's workspace.  With base == nullptr it only
// measures.
struct Arena {
  char* base;
  size_t cap, off;
  bool ok;
  Arena(void* b, size_t c) : base((char*)b), cap(c), off(0), ok(true) {}
  void* take(size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    if (off > cap) ok = false;
    return base ? (void*)(base + o) : nullptr;
  }
};

#define HIPCHK(x)                         \
  do {                                    \
    if ((x) != hipSuccess) return TK_ERR_HIP; \
  } while (0)

View mode_view(int N, const int64_t* dims, int n) {
  View v;
  v.P = 1;
  for (int k = 0; k < n; ++k) v.P *= dims[k];
  v.I = dims[n];
  v.Q = 1;
  for (int k = n + 1; k < N; ++k) v.Q *= dims[k];
  return v;
}

int64_t numel(int N, const int64_t* dims) {
  int64_t s = 1;
  for (int k = 0; k < N; ++k) s *= dims[k];
  return s;
}

bool valid_dims(int N, const int64_t* dims) {
  if (!dims || N < 1 || N > TK_MAX_ORDER) return false;
  double tot = 1.0;
  for (int k = 0; k < N; ++k) {
    if (dims[k] <= 0) return false;
    tot *= (double)dims[k];
  }
  return tot < 9.0e18;
}

bool valid_ranks(int N, const int64_t* dims, const int32_t* ranks) {
  if (!ranks) return false;
  for (int n = 0; n < N; ++n) {
    if (ranks[n] < 1 || ranks[n] > dims[n] || ranks[n] > 64) return false;
    double others = 1.0;
    for (int k = 0; k < N; ++k)
      if (k != n) others *= ranks[k];
    if (N > 1 && (double)ranks[n] > others) return false;
  }
  return true;
}

bool valid_dtype(int dt) { return dt == TK_F64 || dt == TK_F32 || dt == TK_BF16; }

// ---------------------------------------------------------------------------
// Device status block read back once per sweep.
struct DevStatus {
  int status;
  // failure of the speculative preparation made by sweep k, in slot k & 1
  int prep_status[2];
  // failure of a mode's final QR whose check is left to the next read
  int qr_status;
  // sweep k, slot k & 1: [0] = res^2, [1] = tr(Gq^{-1} G_V)
  double res[2][2];
  double norm2;
  double rsum;
};

// Workspace of one mode solve on view v with rank R.
struct ModeWs {
  double *L, *Lnext, *Lacc, *CL, *Wq, *GV, *Q1;
  void *Lq, *Lr;               // compute type
  void *parts;                 // lacc/Y partials (compute type)
  double *gparts, *sparts;     // Gram partials, scalar partials
  double* rtmp;                // first-stage sums of the two-stage reductions
  void* V;                     // generic path: J x R (compute type)
  DevStatus* st;
};

void carve_mode(Arena& ar, int xdt, const View& v, int R, ModeWs& w) {
  const int cdt = cdtype(xdt);
  const size_t cs = dsize(cdt);
  const int64_t IR = v.I * (int64_t)R;
  w.L = (double*)ar.take(IR * 8);
  w.Lnext = (double*)ar.take(IR * 8);
  w.Lacc = (double*)ar.take(IR * 8);
  w.Q1 = (double*)ar.take(IR * 8);
  w.CL = (double*)ar.take(64 * 64 * 8);
  w.Wq = (double*)ar.take(64 * 64 * 8);
  w.GV = (double*)ar.take(64 * 64 * 8);
  w.Lq = ar.take(IR * cs);
  w.Lr = ar.take(IR * cs);
  w.parts = ar.take((size_t)NWG_MAX * IR * cs);
  w.gparts = (double*)ar.take((size_t)NWG_MAX * R * R * 8);
  w.sparts = (double*)ar.take((size_t)NWG_MAX * 8 * 2);
  w.rtmp = (double*)ar.take((size_t)(REDUCE_GROUPS / 4) * IR * 8);
  w.st = (DevStatus*)ar.take(sizeof(DevStatus));
  if (!fused_supported(xdt, v, R, TK_RESID_EXPLICIT)) w.V = ar.take((size_t)v.J() * R * cs);
  else w.V = nullptr;
}

struct Opts {
  double tol;
  int max_iters;
  int resid_mode;
  uint64_t seed;
  const int32_t* order;
  int svec;
  const void* const* init_U;
};

int read_opts(const tk_als_opts* o, int N, Opts& out) {
  out.tol = 1e-4;
  out.max_iters = 50;
  out.resid_mode = TK_RESID_AUTO;
  out.seed = 0;
  out.order = nullptr;
  out.svec = 0;
  out.init_U = nullptr;
  if (!o) return TK_OK;
  if (o->struct_size < sizeof(tk_als_opts)) return TK_ERR_INVALID_ARG;
  if (!(o->tol >= 0.0) || o->max_iters < 0) return TK_ERR_INVALID_ARG;
  if (o->resid_mode != TK_RESID_AUTO && o->resid_mode != TK_RESID_TRACE &&
      o->resid_mode != TK_RESID_EXPLICIT)
    return TK_ERR_INVALID_ARG;
  if (o->compute != TK_COMPUTE_AS_STORAGE) return TK_ERR_UNSUPPORTED_DTYPE;
  out.tol = o->tol;
  out.max_iters = o->max_iters;
  out.resid_mode = o->resid_mode;
  out.seed = o->seed;
  out.order = o->order;
  out.svec = o->singular_vectors != 0;
  out.init_U = o->init_U;
  if (out.order) {
    bool seen[TK_MAX_ORDER] = {false};
    for (int k = 0; k < N; ++k) {
      int m = out.order[k];
      if (m < 0 || m >= N || seen[m]) return TK_ERR_INVALID_ARG;
      seen[m] = true;
    }
  }
  return TK_OK;
}

// ---------------------------------------------------------------------------
// Small FP64 building blocks

// Reduced QR (CholeskyQR2) of the FP64 m x r matrix L into Q (FP64), one
// workgroup; Q1 is m x r scratch.
void qr_enqueue(const double* L, int64_t m, int r, double* Q, double* Q1, int* status,
                hipStream_t s) {
  StepArgs a{};
  a.m = m; a.r = r; a.ops = STEP_QR;
  a.Qin = L; a.Q1 = Q1; a.Qout = Q;
  a.status = status;
  launch_mode_step(a, TK_F64, s);
}

// The status block is read through a small pinned host buffer of the calling
// thread (allocated on first use, kept for the life of the thread: a copy
// into pageable memory goes through a runtime staging buffer and costs a
// longer round trip on every sweep).
// While a call of the allocation-free entry point runs on this thread, the
// buffer is not allocated (an earlier allocation is still used).
thread_local bool t_no_alloc = false;

DevStatus* pinned_status() {
  thread_local DevStatus* p = nullptr;
  thread_local bool tried = false;
  if (!tried && !t_no_alloc) {
    tried = true;
    if (hipHostMalloc((void**)&p, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess) p = nullptr;
  }
  return p;
}

int read_status(const DevStatus* d, DevStatus* h, hipStream_t s) {
  DevStatus* ph = pinned_status();
  HIPCHK(hipMemcpyAsync(ph ? ph : h, d, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (ph) *h = *ph;
  return TK_OK;
}

// ||X||^2 in FP64 (deterministic two-stage reduction).
int norm2_enqueue(const void* X, int xdt, int64_t n, double* sparts, double* out,
                  double* rtmp, hipStream_t s) {
  int chunks = (int)std::min<int64_t>(NWG_MAX, std::max<int64_t>(1, ceil_div(n, 65536)));
  launch_norm2_parts(X, xdt, n, chunks, sparts, s);
  launch_reduce_parts<double>(sparts, chunks, 1, 1, out, rtmp, s);
  return TK_OK;
}

struct ModeResult {
  int iters, converged, sweeps;
  int form;             // residual form the stop test used
  int qr_failed;        // a status read found an earlier mode's deferred QR failure
  double resid;
};

// The residual form of a mode solve, TK_RESID_AUTO resolved.  With FP32
// accumulation the trace form's res^2 = ||B||^2 - tr(...) carries a rounding of
// about 2^-24 sqrt((I + 64) / J) ||B||^2 (rounding of the I-term sums of V and of
// the fibre sums, averaged over J fibres), so at a relative residual rho its
// error on res is that over 2 rho ||B||.  The explicit form is chosen when this
// error could exceed a quarter of eta ||A|| at rho = 1e-4 (taking ||B|| ~ ||A||);
// it costs one more small product per fibre and no tensor traffic.  FP64
// storage, and eta = 0 (no stop test), keep the trace form.
int resolve_resid_form(int resid_mode, int xdt, const View& v, double tol) {
  if (resid_mode != TK_RESID_AUTO) return resid_mode;
  if (cdtype(xdt) == TK_F64 || !(tol > 0.0)) return TK_RESID_TRACE;
  const double crit = 4.0 * 0x1p-24 * sqrt((double)(v.I + 64) / (double)v.J());
  return crit > 1e-4 * tol ? TK_RESID_EXPLICIT : TK_RESID_TRACE;
}

// BF16 sweeps with the trace residual multiply the BF16 tensor by L~ rounded to
// BF16 precision (one BF16 term; the trace form takes the Gram of the rounded
// values, so it is the residual of exactly the subspace swept).  The explicit
// residual sums ||a_j - L v_j||^2 with L itself, which is consistent with v_j
// only for the FP32 L~ (three BF16 terms): there L~ is not rounded.
inline bool lq_rounded(int xdt, int resid_form) {
  return xdt == TK_BF16 && resid_form == TK_RESID_TRACE;
}

// Y (FP64, I x R) = B_(n) S  (Section 5 initial sketch), partial-reduced;
// with norm2 != null the same pass also yields ||B||_F^2.
void init_enqueue(const void* X, int xdt, const View& v, int R, uint64_t seed, int mode,
                  ModeWs& w, double* Yout, double* norm2, hipStream_t s) {
  const int64_t IR = v.I * (int64_t)R;
  if (fused_supported(xdt, v, R, TK_RESID_TRACE)) {
    FusedArgs f{};
    f.X = X; f.x_dtype = xdt; f.v = v; f.R = R;
    f.lacc_parts = (float*)w.parts;
    f.sketch = 1; f.seed = seed; f.mode = mode;
    f.norm2_parts = norm2 ? w.sparts : nullptr;
    int nwg = launch_fused(f, NWG_MAX, s);
    launch_reduce_parts<float>((const float*)w.parts, nwg, IR, IR, Yout, w.rtmp, s);
    if (norm2) launch_reduce_parts<double>(w.sparts, FUSED_WAVES * nwg, 1, 1, norm2, w.rtmp, s);
  } else {
    LpassArgs a{};
    a.X = X; a.x_dtype = xdt; a.v = v; a.v_kind = 1; a.R = R; a.seed = seed; a.mode = mode;
    a.parts = w.parts;
    a.norm2_parts = norm2 ? w.sparts : nullptr;
    int chunks = lpass_chunks(v, R, NWG_MAX);
    launch_lpass(a, chunks, s);
    if (cdtype(xdt) == TK_F64)
      launch_reduce_parts<double>((const double*)w.parts, chunks, IR, IR, Yout, w.rtmp, s);
    else
      launch_reduce_parts<float>((const float*)w.parts, chunks, IR, IR, Yout, w.rtmp, s);
    if (norm2)
      launch_reduce_parts<double>(w.sparts, lpass_blocks(v, chunks), 1, 1, norm2, w.rtmp, s);
  }
}

// The mode step may run on a cooperative grid with its Gram partials in the
// sweep's G_V partial buffer (free while it runs: G_V is reduced before, and
// the next fused pass writes it after).  Not in the allocation-free entry
// point, whose callers may capture the stream into a graph.
void mode_step_grid(StepArgs& a, ModeWs& w, int R) {
  if (t_no_alloc) return;
  a.gpart = w.gparts;
  a.gpart_cap = (int64_t)NWG_MAX * R * R;
}

// The step that follows the initial pass: L = Q of the reduced QR of Lacc,
// then L~, its quantised Gram factor (and L for the explicit residual) for
// the first sweep.
void init_finish_enqueue(const View& v, int R, int xdt, int resid_mode, ModeWs& w,
                         hipStream_t s) {
  StepArgs a{};
  a.m = v.I; a.r = R; a.ops = STEP_QR | STEP_PREP;
  a.Qin = w.Lacc; a.Q1 = w.Q1; a.Qout = w.L;
  mode_step_grid(a, w, R);
  a.Lq = w.Lq; a.Lr = resid_mode == TK_RESID_EXPLICIT ? w.Lr : nullptr; a.Wq = w.Wq;
  a.lq_bf16 = lq_rounded(xdt, resid_mode);
  a.status = &w.st->status; a.prep_status = &w.st->prep_status[0];
  launch_mode_step(a, cdtype(xdt), s);
}

// One sweep of Algorithm 3.3 from w.L, whose L~ (w.Lq), inverse Gram factor (w.Wq)
// and compute-type copy (w.Lr, explicit residual) are already prepared:
// R-update (never stored when fused), L-update into w.Lnext, residual into
// st->res[slot], and the speculative preparation of the sweep from w.Lnext
// (its failure into st->prep_status[slot]).  ||X||^2 is norm2, or *norm2p on
// the device when norm2p is non-null.
void sweep_enqueue(const void* X, int xdt, const View& v, int R, double norm2,
                   int resid_mode, ModeWs& w, hipStream_t s, int slot = 0,
                   const double* norm2p = nullptr) {
  const int64_t IR = v.I * (int64_t)R;
  const int cdt = cdtype(xdt);
  const bool expl = resid_mode == TK_RESID_EXPLICIT;
  int nres = 0;
  if (fused_supported(xdt, v, R, resid_mode)) {
    FusedArgs f{};
    f.X = X; f.x_dtype = xdt; f.v = v; f.R = R;
    f.Lq = (const float*)w.Lq;
    f.lq_bf16 = lq_rounded(xdt, resid_mode);   // the preparation rounded L~ so
    f.Lr = expl ? (const float*)w.Lr : nullptr;
    f.lacc_parts = (float*)w.parts;
    f.gv_parts = w.gparts;
    f.resid_parts = w.sparts;
    int nwg = launch_fused(f, NWG_MAX, s);
    launch_reduce_parts<float>((const float*)w.parts, nwg, IR, IR, w.Lacc, w.rtmp, s);
    launch_reduce_parts<double>(w.gparts, FUSED_WAVES * nwg, (int64_t)R * R, (int64_t)R * R,
                                w.GV, w.rtmp, s);
    nres = FUSED_WAVES * nwg;
  } else {
    VpassArgs a{};
    a.X = X; a.x_dtype = xdt; a.v = v;
    a.W = w.Lq; a.w_ldi = R; a.w_ldo = 1; a.O = R;
    a.out = w.V; a.out_kind = 0;
    a.Lr = expl ? w.Lr : nullptr;
    a.resid_parts = expl ? w.sparts : nullptr;
    launch_vpass(a, NWG_MAX, &nres, s);
    int gch = (int)std::min<int64_t>(NWG_MAX, std::max<int64_t>(1, ceil_div(v.J(), 4096)));
    launch_gram_parts(w.V, cdt, v.J(), R, gch, w.gparts, s);
    launch_reduce_parts<double>(w.gparts, gch, (int64_t)R * R, (int64_t)R * R, w.GV, w.rtmp, s);
    LpassArgs l{};
    l.X = X; l.x_dtype = xdt; l.v = v; l.v_kind = 0; l.V = w.V; l.R = R;
    l.parts = w.parts;
    int chunks = lpass_chunks(v, R, NWG_MAX);
    launch_lpass(l, chunks, s);
    if (cdt == TK_F64)
      launch_reduce_parts<double>((const double*)w.parts, chunks, IR, IR, w.Lacc, w.rtmp, s);
    else
      launch_reduce_parts<float>((const float*)w.parts, chunks, IR, IR, w.Lacc, w.rtmp, s);
  }
  StepArgs a{};
  a.m = v.I; a.r = R; a.ops = STEP_SOLVE | STEP_PREP | STEP_PREP_SPECULATIVE;
  a.Lacc = w.Lacc; a.GV = w.GV; a.Lnext = w.Lnext; a.norm2 = norm2; a.norm2p = norm2p;
  mode_step_grid(a, w, R);
  if (expl) {
    launch_reduce_parts<double>(w.sparts, nres, 1, 1, &w.st->rsum, w.rtmp, s);
    a.rsum = &w.st->rsum;
  }
  a.res2 = w.st->res[slot];
  a.Lq = w.Lq; a.Lr = expl ? w.Lr : nullptr; a.Wq = w.Wq;
  a.lq_bf16 = lq_rounded(xdt, resid_mode);
  a.status = &w.st->status; a.prep_status = &w.st->prep_status[slot];
  launch_mode_step(a, cdt, s);
}

// Algorithm 3.3 on the mode view of X with rank R, initial guess of
// Section 5, stop test E5.01 (first at k = 1, against norm_a = ||A||_F of the
// input tensor; norm_a < 0: the norm of X).  normx2 = ||X||_F^2 of the
// tensor being swept (trace form of the residual); when it is negative on
// entry the initial pass computes it and returns it there.  On return U64
// (FP64 I x R) holds Q of the reduced QR of the returned L.  With L0 (I x R,
// device, FP64 or FP32 as l0_dt; may alias U64) the iteration starts from the Q
// of L0's reduced QR instead of the sketch (a warm start: only the span of L_0
// matters to Algorithm 3.3), and ||X||^2 comes from a pass of its own.  With
// defer_qr, w.st is the caller's status block for the whole call: its failure
// flags are kept from earlier modes (and checked by every read), and the final
// QR's failure is left in qr_status for the caller's next read instead of being
// read back here; a read that finds an earlier mode's QR failure returns it
// with mr.qr_failed set.
int mode_solve(const void* X, int xdt, const View& v, int R, const Opts& o, double& normx2,
               double norm_a, int mode, ModeWs& w, double* U64, ModeResult& mr,
               hipStream_t s, const void* L0 = nullptr, int l0_dt = TK_F64,
               bool defer_qr = false) {
  mr.iters = 0; mr.converged = 1; mr.sweeps = 0; mr.resid = 0.0; mr.qr_failed = 0;
  const int form = resolve_resid_form(o.resid_mode, xdt, v, o.tol);
  mr.form = form;
  DevStatus h{};
  const bool want_norm = normx2 < 0.0;
  if (defer_qr) HIPCHK(hipMemsetAsync(w.st->prep_status, 0, sizeof(w.st->prep_status), s));
  else HIPCHK(hipMemsetAsync(w.st, 0, sizeof(DevStatus), s));
  auto read = [&]() -> int {
    int r2 = read_status(w.st, &h, s);
    if (r2) return r2;
    if (h.qr_status) {
      mr.qr_failed = 1;
      return h.qr_status;
    }
    return TK_OK;
  };
  if (R == v.I) {
    if (want_norm) {
      norm2_enqueue(X, xdt, v.P * v.I * v.Q, w.sparts, &w.st->norm2, w.rtmp, s);
      int rc = read();
      if (rc) return rc;
      normx2 = h.norm2;
      if (!isfinite(normx2)) return TK_ERR_NONFINITE;
    }
    launch_identity<double>(U64, v.I, s);
    return TK_OK;
  }
  if (L0) {
    if (want_norm) norm2_enqueue(X, xdt, v.P * v.I * v.Q, w.sparts, &w.st->norm2, w.rtmp, s);
    if (l0_dt == TK_F64)
      HIPCHK(hipMemcpyAsync(w.Lacc, L0, (size_t)v.I * R * 8, hipMemcpyDeviceToDevice, s));
    else
      launch_widen<float>((const float*)L0, v.I * (int64_t)R, w.Lacc, s);
  } else {
    init_enqueue(X, xdt, v, R, o.seed, mode, w, w.Lacc, want_norm ? &w.st->norm2 : nullptr, s);
  }
  init_finish_enqueue(v, R, xdt, form, w, s);
  // The stop test first runs after sweep 1, so with max_iters >= 1 the initial
  // step and sweeps 0 and 1 are enqueued back to back and checked by one
  // status read: ||X||^2 reaches the sweeps on the device, sweep 0 keeps its
  // residual and its preparation status in slot 0, and every failure flag is
  // sticky (kernels after a failed step run on stale but in-range data and
  // their results are discarded with the error).
  const bool defer = o.max_iters >= 1;
  const double* n2p = want_norm ? &w.st->norm2 : nullptr;
  bool have_norm = !want_norm;
  int rc = TK_OK;
  auto take_status = [&]() -> int {
    int r2 = read();
    if (r2) return r2;
    if (!have_norm) {
      normx2 = h.norm2;
      if (!isfinite(normx2)) return TK_ERR_NONFINITE;
      have_norm = true;
    }
    return h.status;
  };
  if (!defer) {
    rc = take_status();
    if (rc) return rc;
  }
  double nA = 0.0;
  double res_prev = 0.0;
  for (int k = 0;; ++k) {
    sweep_enqueue(X, xdt, v, R, normx2, form, w, s, k & 1, n2p);
    mr.sweeps++;
    if (defer && k == 0) {
      // sweep 1 starts from L_1, prepared speculatively by sweep 0
      std::swap(w.L, w.Lnext);
      continue;
    }
    rc = take_status();
    if (rc) return rc;
    nA = norm_a >= 0.0 ? norm_a : sqrt(normx2);
    if (defer && k == 1) {
      if (h.prep_status[0]) return h.prep_status[0];
      const double r0 = h.res[0][0];
      res_prev = sqrt(r0 > 0.0 ? r0 : 0.0);
      if (!isfinite(res_prev)) return TK_ERR_NONFINITE;
    }
    const double r2 = h.res[k & 1][0];
    double res = sqrt(r2 > 0.0 ? r2 : 0.0);
    if (!isfinite(res)) return TK_ERR_NONFINITE;
    mr.resid = res;
    mr.iters = k;
    if (k >= 1 && fabs(res_prev - res) <= o.tol * nA) { mr.converged = 1; break; }
    if (k >= o.max_iters) { mr.converged = 0; break; }
    // the next sweep starts from L_{k+1}, whose preparation ran speculatively
    if (h.prep_status[k & 1]) return h.prep_status[k & 1];
    std::swap(w.L, w.Lnext);
    res_prev = res;
  }
  if (defer_qr) {
    qr_enqueue(w.L, v.I, R, U64, w.Q1, &w.st->qr_status, s);
    return TK_OK;
  }
  qr_enqueue(w.L, v.I, R, U64, w.Q1, &w.st->status, s);
  rc = read_status(w.st, &h, s);
  if (rc) return rc;
  return h.status;
}

// Singular vectors of X_(mode) inside the span of the orthonormal Q (FP64 I x R;
// Section 3, after Algorithm 3.4): M = Q^T X_(mode) X_(mode)^T Q from one streaming
// pass with Q (in the compute dtype) as L~, its eigenvectors W (FP64 Jacobi) into w.CL
// (the eigenvalues into w.Wq, unused afterwards), and Q W into w.Lnext.
int svec_enqueue(const void* X, int xdt, const View& v, int R, const double* Q, ModeWs& w,
                 hipStream_t s) {
  const int64_t IR = v.I * (int64_t)R;
  const int64_t RR = (int64_t)R * R;
  const int cdt = cdtype(xdt);
  if (cdt == TK_F64) launch_convert<double>(Q, IR, (double*)w.Lq, s);
  else launch_convert<float>(Q, IR, (float*)w.Lq, s);
  if (fused_supported(xdt, v, R, TK_RESID_TRACE)) {
    FusedArgs f{};
    f.X = X; f.x_dtype = xdt; f.v = v; f.R = R;
    f.Lq = (const float*)w.Lq;
    f.lacc_parts = (float*)w.parts;
    f.gv_parts = w.gparts;
    int nwg = launch_fused(f, NWG_MAX, s);
    launch_reduce_parts<double>(w.gparts, FUSED_WAVES * nwg, RR, RR, w.GV, w.rtmp, s);
  } else {
    VpassArgs a{};
    a.X = X; a.x_dtype = xdt; a.v = v;
    a.W = w.Lq; a.w_ldi = R; a.w_ldo = 1; a.O = R;
    a.out = w.V; a.out_kind = 0;
    int nres = 0;
    launch_vpass(a, NWG_MAX, &nres, s);
    int gch = (int)std::min<int64_t>(NWG_MAX, std::max<int64_t>(1, ceil_div(v.J(), 4096)));
    launch_gram_parts(w.V, cdt, v.J(), R, gch, w.gparts, s);
    launch_reduce_parts<double>(w.gparts, gch, RR, RR, w.GV, w.rtmp, s);
  }
  launch_sym_eig(w.GV, R, w.CL, w.Wq, &w.st->status, s);
  launch_rotate(Q, v.I, R, w.CL, w.Lnext, s);
  DevStatus h{};
  int rc = read_status(w.st, &h, s);
  if (rc) return rc;
  // the deferred check of the QR that made Q
  return h.qr_status ? h.qr_status : h.status;
}

// ---------------------------------------------------------------------------
// Workspace plan of the drivers.

// Workspace bound of a mode solve over every mode at the untruncated shape
// (the largest view a mode can be solved on, whatever the st-HOSVD order),
// in the storage dtype and, for st-HOSVD, the compute dtype of the
// truncated intermediates.
size_t max_mode_ws(int xdt, int N, const int64_t* dims, const int32_t* ranks, bool st) {
  size_t mx = 0;
  for (int n = 0; n < N; ++n) {
    View v = mode_view(N, dims, n);
    for (int pass = 0; pass < (st ? 2 : 1); ++pass) {
      Arena ar(nullptr, (size_t)-1);
      ModeWs w;
      carve_mode(ar, pass == 0 ? xdt : cdtype(xdt), v, ranks[n], w);
      mx = std::max(mx, ar.off);
    }
  }
  return mx;
}

// Elements of each ping-pong buffer holding intermediate tensors of a TTM
// chain: bounded by the largest single-mode truncation of the input, which
// covers every processing order.
int64_t chain_elems(int N, const int64_t* dims, const int32_t* ranks) {
  int64_t tot = numel(N, dims), mx = 1;
  for (int n = 0; n < N; ++n) mx = std::max(mx, tot / dims[n] * ranks[n]);
  return mx;
}

size_t driver_ws(int which, int xdt, int N, const int64_t* dims, const int32_t* ranks) {
  size_t mw = max_mode_ws(xdt, N, dims, ranks, which == 1);
  const size_t cs = dsize(cdtype(xdt));
  const int64_t e = chain_elems(N, dims, ranks);
  size_t u64 = 0;
  for (int n = 0; n < N; ++n) u64 += align_up((size_t)dims[n] * ranks[n] * 8);
  return align_up(mw) + 2 * align_up(e * cs) + u64 + 4096;
}

int ttm_enqueue(const void* X, int xdt, int N, const int64_t* dims, int mode, const void* M,
                int64_t J, int trans, void* Y, hipStream_t s) {
  View v = mode_view(N, dims, mode);
  if (fused_ttm_supported(xdt, v, J)) {
    // matrix cores; the matrix is FP32 (the compute type of FP32 / BF16 data)
    FusedArgs f{};
    f.X = X; f.x_dtype = xdt; f.v = v; f.R = (int)J;
    f.Lq = (const float*)M;
    if (trans) { f.lq_ldi = J; f.lq_ldo = 1; }
    else { f.lq_ldi = 1; f.lq_ldo = v.I; }
    f.y = (float*)Y;
    launch_fused(f, NWG_MAX, s);
    return TK_OK;
  }
  VpassArgs a{};
  a.X = X; a.x_dtype = xdt; a.v = v;
  a.W = M;
  if (trans) { a.w_ldi = J; a.w_ldo = 1; }
  else { a.w_ldi = 1; a.w_ldo = v.I; }
  a.O = J; a.out = Y; a.out_kind = 1;
  int used = 0;
  return launch_vpass(a, NWG_MAX, &used, s);
}

int run_driver(int which, const void* A, int32_t adt, int32_t N, const int64_t* dims,
               const int32_t* ranks, const tk_als_opts* opts, void* const* U, void* G,
               void* ws, size_t ws_bytes, tk_als_info* info, void* stream) {
  if (info) memset(info, 0, sizeof(*info));
  if (!valid_dtype(adt)) return TK_ERR_UNSUPPORTED_DTYPE;
  if (!A || !U || !G || !valid_dims(N, dims) || !valid_ranks(N, dims, ranks))
    return TK_ERR_INVALID_ARG;
  for (int n = 0; n < N; ++n)
    if (!U[n]) return TK_ERR_INVALID_ARG;
  Opts o;
  int rc = read_opts(opts, N, o);
  if (rc) return rc;
  const int32_t* order = which == 1 ? o.order : nullptr;
  size_t need = driver_ws(which, adt, N, dims, ranks);
  if (!ws || ws_bytes < need) return TK_ERR_WORKSPACE_TOO_SMALL;

  hipStream_t s = (hipStream_t)stream;
  const int cdt = cdtype(adt);
  const size_t cs = dsize(cdt);
  const int64_t ech = chain_elems(N, dims, ranks);
  Arena ar(ws, ws_bytes);
  void* bufA = ar.take(ech * cs);
  void* bufB = ar.take(ech * cs);
  double* U64[TK_MAX_ORDER];
  for (int n = 0; n < N; ++n) U64[n] = (double*)ar.take((size_t)dims[n] * ranks[n] * 8);
  // one status block for the whole call: a mode's final QR reports a failure
  // through the next read (the next mode's, or the one at the end)
  DevStatus* cst = (DevStatus*)ar.take(sizeof(DevStatus));
  Arena mar(ar.base + ar.off, ar.cap - ar.off);
  HIPCHK(hipMemsetAsync(cst, 0, sizeof(DevStatus), s));

  int mstat[TK_MAX_ORDER];
  for (int n = 0; n < N; ++n) mstat[n] = TK_SKIPPED;
  // On a failure: its mode's status, TK_SKIPPED stays on the modes not reached.
  auto fail = [&](int n, int code) -> int {
    mstat[n] = code;
    if (info) {
      for (int k = 0; k < N; ++k) info->mode_status[k] = mstat[k];
      info->status = code;
    }
    return code;
  };
  // ||A||^2 (E5.01 uses the input's norm for every mode) comes out of the
  // first mode's initial pass over A; in st-HOSVD each later mode's initial
  // pass yields ||B||^2 of the truncated tensor it sweeps.
  double norm2 = -1.0;
  int worst = TK_OK;
  int64_t cur[TK_MAX_ORDER];
  for (int k = 0; k < N; ++k) cur[k] = dims[k];
  const void* B = A;
  int bdt = adt;
  int prev = -1;  // the mode whose final QR is checked by the next read
  for (int t = 0; t < N; ++t) {
    const int n = order ? order[t] : t;
    View v = mode_view(N, which == 1 ? cur : dims, n);
    const int R = ranks[n];
    Arena tmp = mar;
    ModeWs w;
    carve_mode(tmp, which == 1 ? bdt : adt, v, R, w);
    w.st = cst;
    ModeResult mr;
    double normb2 = (which == 1 && t > 0) ? -1.0 : norm2;
    const void* L0 = o.init_U ? o.init_U[n] : nullptr;
    rc = mode_solve(which == 1 ? B : A, which == 1 ? bdt : adt, v, R, o, normb2,
                    norm2 >= 0.0 ? sqrt(norm2) : -1.0, n, w, U64[n], mr, s, L0, cdt, true);
    if (rc == TK_OK && norm2 < 0.0) {
      norm2 = normb2;
      if (info) info->norm_a = sqrt(norm2);
    }
    if (info) {
      info->iters[n] = mr.iters;
      info->converged[n] = mr.converged;
      info->resid[n] = mr.resid;
      info->resid_form[n] = mr.form;
      info->sweeps += mr.sweeps;
    }
    if (mr.qr_failed && prev >= 0) return fail(prev, rc);
    if (rc < 0) return fail(n, rc);
    mstat[n] = mr.converged ? TK_OK : TK_NOT_CONVERGED;
    if (!mr.converged) worst = TK_NOT_CONVERGED;
    prev = n;
    const double* Uf = U64[n];
    if (which == 0 && o.svec) {
      rc = svec_enqueue(A, adt, v, R, U64[n], w, s);
      if (rc) return fail(n, rc);
      prev = -1;
      Uf = w.Lnext;
    }
    // factor in the caller's dtype
    const int64_t IR = v.I * (int64_t)R;
    if (cdt == TK_F64) launch_convert<double>(Uf, IR, (double*)U[n], s);
    else launch_convert<float>(Uf, IR, (float*)U[n], s);
    if (which == 1) {
      // B <- B x_n U_n^T (equals Algorithm 3.5's R_hat R^T)
      void* dst = (t == N - 1) ? G : ((t % 2 == 0) ? bufA : bufB);
      rc = ttm_enqueue(B, bdt, N, cur, n, U[n], R, 1, dst, s);
      if (rc) return fail(n, rc);
      cur[n] = R;
      B = dst;
      bdt = cdt;
    }
  }
  if (which == 0) {
    // G = A x_1 U_1^T ... x_N U_N^T (the core of Algorithm 3.4)
    for (int t = 0; t < N; ++t) {
      void* dst = (t == N - 1) ? G : ((t % 2 == 0) ? bufA : bufB);
      rc = ttm_enqueue(B, bdt, N, cur, t, U[t], ranks[t], 1, dst, s);
      if (rc) return fail(t, rc);
      cur[t] = ranks[t];
      B = dst;
      bdt = cdt;
    }
  }
  // the last mode's QR status (the read also waits for the whole stream)
  DevStatus h{};
  rc = read_status(cst, &h, s);
  if (rc) return fail(prev >= 0 ? prev : (order ? order[N - 1] : N - 1), rc);
  if (h.qr_status && prev >= 0) return fail(prev, h.qr_status);
  if (hipGetLastError() != hipSuccess) return fail(order ? order[N - 1] : N - 1, TK_ERR_HIP);
  if (h.status) return fail(order ? order[N - 1] : N - 1, h.status);
  if (info) {
    for (int k = 0; k < N; ++k) info->mode_status[k] = mstat[k];
    info->status = worst;
  }
  return worst;
}

// Workspace of hooi_refine: that of st-HOSVD-ALS (whose bound covers every mode
// solve on the truncated tensors Y of either dtype) and one status block.
size_t hooi_ws(int xdt, int N, const int64_t* dims, const int32_t* ranks) {
  return driver_ws(1, xdt, N, dims, ranks) + align_up(sizeof(DevStatus)) + 4096;
}

// G = A x_1 U_1^T ... x_N U_N^T through the ping-pong buffers; returns the status of
// the TTM launches.
int core_chain(const void* A, int adt, int N, const int64_t* dims, const int32_t* ranks,
               void* const* U, void* G, void* bufA, void* bufB, hipStream_t s) {
  int64_t cur[TK_MAX_ORDER];
  for (int k = 0; k < N; ++k) cur[k] = dims[k];
  const void* B = A;
  int bdt = adt;
  for (int t = 0; t < N; ++t) {
    void* dst = (t == N - 1) ? G : ((t % 2 == 0) ? bufA : bufB);
    int rc = ttm_enqueue(B, bdt, N, cur, t, U[t], ranks[t], 1, dst, s);
    if (rc) return rc;
    cur[t] = ranks[t];
    B = dst;
    bdt = cdtype(adt);
  }
  return TK_OK;
}

// HOOI (higher-order orthogonal iteration) from the caller's orthonormal factors, the
// refinement the paper applies to t-/st-HOSVD(-ALS) results (Section 6.3, Table 6.3-2).
// An outer iteration replaces, for n = 0..N-1 in turn, U_n by an orthonormal basis of
// the dominant R_n-dimensional left subspace of Y_(n), Y = A x_{k != n} U_k^T: ALS
// (Algorithm 3.3) on Y_(n) warm-started from U_n, then QR.  The core is
// G = Y x_{N-1} U_{N-1}^T of the last mode, and the error
// ||A - A_hat|| / ||A|| = sqrt(||A||^2 - ||G||^2) / ||A|| (orthonormal factors); the
// iteration stops when it changes by at most tol.
int run_hooi(const void* A, int32_t adt, int32_t N, const int64_t* dims, const int32_t* ranks,
             const tk_als_opts* opts, double tol, int32_t max_iters, void* const* U, void* G,
             void* ws, size_t ws_bytes, tk_hooi_info* info, void* stream) {
  if (info) memset(info, 0, sizeof(*info));
  if (!valid_dtype(adt)) return TK_ERR_UNSUPPORTED_DTYPE;
  if (!A || !U || !G || !valid_dims(N, dims) || !valid_ranks(N, dims, ranks) ||
      !(tol >= 0.0) || max_iters < 0)
    return TK_ERR_INVALID_ARG;
  for (int n = 0; n < N; ++n)
    if (!U[n]) return TK_ERR_INVALID_ARG;
  Opts o;
  int rc = read_opts(opts, N, o);
  if (rc) return rc;
  const size_t need = hooi_ws(adt, N, dims, ranks);
  if (!ws || ws_bytes < need) return TK_ERR_WORKSPACE_TOO_SMALL;

  hipStream_t s = (hipStream_t)stream;
  const int cdt = cdtype(adt);
  const size_t cs = dsize(cdt);
  const int64_t ech = chain_elems(N, dims, ranks);
  Arena ar(ws, ws_bytes);
  void* bufA = ar.take(ech * cs);
  void* bufB = ar.take(ech * cs);
  double* U64[TK_MAX_ORDER];
  for (int n = 0; n < N; ++n) U64[n] = (double*)ar.take((size_t)dims[n] * ranks[n] * 8);
  DevStatus* hs = (DevStatus*)ar.take(sizeof(DevStatus));
  Arena mar(ar.base + ar.off, ar.cap - ar.off);
  int64_t gsize = 1;
  for (int n = 0; n < N; ++n) gsize *= ranks[n];

  for (int n = 0; n < N; ++n) {
    const int64_t IR = dims[n] * (int64_t)ranks[n];
    if (cdt == TK_F64) launch_widen<double>((const double*)U[n], IR, U64[n], s);
    else launch_widen<float>((const float*)U[n], IR, U64[n], s);
  }
  // ||A||^2, then the error of the starting factors
  DevStatus h{};
  {
    Arena tmp = mar;
    ModeWs w;
    carve_mode(tmp, adt, mode_view(N, dims, 0), ranks[0], w);
    HIPCHK(hipMemsetAsync(hs, 0, sizeof(DevStatus), s));
    norm2_enqueue(A, adt, numel(N, dims), w.sparts, &hs->norm2, w.rtmp, s);
    rc = read_status(hs, &h, s);
    if (rc) return rc;
  }
  const double nA2 = h.norm2;
  if (!isfinite(nA2)) return TK_ERR_NONFINITE;
  const double nA = sqrt(nA2);
  if (info) info->norm_a = nA;
  auto error_of_core = [&](double& err) -> int {
    Arena tmp = mar;
    ModeWs w;
    carve_mode(tmp, adt, mode_view(N, dims, 0), ranks[0], w);
    norm2_enqueue(G, cdt, gsize, w.sparts, &hs->norm2, w.rtmp, s);
    int r2 = read_status(hs, &h, s);
    if (r2) return r2;
    if (!isfinite(h.norm2)) return TK_ERR_NONFINITE;
    const double d = nA2 - h.norm2;
    err = nA2 > 0.0 ? sqrt(d > 0.0 ? d : 0.0) / nA : 0.0;
    return TK_OK;
  };
  rc = core_chain(A, adt, N, dims, ranks, U, G, bufA, bufB, s);
  if (rc) return rc;
  double err_prev = 0.0;
  rc = error_of_core(err_prev);
  if (rc) return rc;
  if (info) { info->relerr_init = err_prev; info->relerr = err_prev; }

  int result = TK_NOT_CONVERGED;
  for (int it = 1; it <= max_iters; ++it) {
    for (int n = 0; n < N; ++n) {
      // Y = A x_{k != n} U_k^T
      int64_t cur[TK_MAX_ORDER];
      for (int k = 0; k < N; ++k) cur[k] = dims[k];
      const void* B = A;
      int bdt = adt;
      int t = 0;
      for (int k = 0; k < N; ++k) {
        if (k == n) continue;
        void* dst = (t % 2 == 0) ? bufA : bufB;
        rc = ttm_enqueue(B, bdt, N, cur, k, U[k], ranks[k], 1, dst, s);
        if (rc) return rc;
        cur[k] = ranks[k];
        B = dst;
        bdt = cdt;
        ++t;
      }
      const View v = mode_view(N, cur, n);
      const int R = ranks[n];
      Arena tmp = mar;
      ModeWs w;
      carve_mode(tmp, bdt, v, R, w);
      ModeResult mr;
      double ny2 = -1.0;
      rc = mode_solve(B, bdt, v, R, o, ny2, nA, n, w, U64[n], mr, s, U64[n], TK_F64);
      if (info) info->sweeps += mr.sweeps;
      if (rc < 0) {
        if (info) info->status = rc;
        return rc;
      }
      const int64_t IR = v.I * (int64_t)R;
      if (cdt == TK_F64) launch_convert<double>(U64[n], IR, (double*)U[n], s);
      else launch_convert<float>(U64[n], IR, (float*)U[n], s);
      if (n == N - 1) {
        rc = ttm_enqueue(B, bdt, N, cur, n, U[n], R, 1, G, s);
        if (rc) return rc;
      }
    }
    double err = 0.0;
    rc = error_of_core(err);
    if (rc) return rc;
    if (info) { info->iters = it; info->relerr = err; }
    if (fabs(err_prev - err) <= tol) {
      result = TK_OK;
      break;
    }
    err_prev = err;
  }
  if (max_iters == 0) result = TK_OK;
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  if (info) { info->converged = result == TK_OK; info->status = result; }
  return result;
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" {

const char* tk_status_string(int32_t st) {
  switch (st) {
    case TK_OK: return "TK_OK";
    case TK_NOT_CONVERGED: return "TK_NOT_CONVERGED";
    case TK_SKIPPED: return "TK_SKIPPED";
    case TK_ERR_INVALID_ARG: return "TK_ERR_INVALID_ARG";
    case TK_ERR_UNSUPPORTED_DTYPE: return "TK_ERR_UNSUPPORTED_DTYPE";
    case TK_ERR_WORKSPACE_TOO_SMALL: return "TK_ERR_WORKSPACE_TOO_SMALL";
    case TK_ERR_RANK_DEFICIENT: return "TK_ERR_RANK_DEFICIENT";
    case TK_ERR_NONFINITE: return "TK_ERR_NONFINITE";
    case TK_ERR_HIP: return "TK_ERR_HIP";
  }
  return "TK_UNKNOWN_STATUS";
}

int hooi_refine(const void* A, int32_t a_dtype, int32_t N, const int64_t* dims,
                const int32_t* ranks, const tk_als_opts* opts, double tol, int32_t max_iters,
                void* const* U, void* G, void* ws, size_t ws_bytes, tk_hooi_info* info,
                void* stream) {
  return run_hooi(A, a_dtype, N, dims, ranks, opts, tol, max_iters, U, G, ws, ws_bytes, info,
                  stream);
}

size_t hooi_workspace_bytes(int32_t a_dtype, int32_t N, const int64_t* dims,
                            const int32_t* ranks) {
  if (!valid_dtype(a_dtype) || !valid_dims(N, dims) || !valid_ranks(N, dims, ranks)) return 0;
  return hooi_ws(a_dtype, N, dims, ranks);
}

int st_order_auto(int32_t N, const int64_t* dims, const int32_t* ranks, int32_t* order) {
  if (!order || !valid_dims(N, dims) || !valid_ranks(N, dims, ranks)) return TK_ERR_INVALID_ARG;
  // each term is below 64^8 * 2^63 and there are at most 8 of them
  using u128 = unsigned __int128;
  int perm[TK_MAX_ORDER];
  for (int k = 0; k < N; ++k) perm[k] = k;
  u128 best = 0;
  bool have = false;
  do {
    u128 cost = 0;
    for (int n = 0; n < N; ++n) {
      u128 r = 1, i = 1;
      for (int k = 0; k <= n; ++k) r *= (u128)ranks[perm[k]];
      for (int k = n; k < N; ++k) i *= (u128)dims[perm[k]];
      cost += r * i;
    }
    // permutations come in lexicographic order: keep the first of equal cost
    if (!have || cost < best) {
      best = cost;
      have = true;
      for (int k = 0; k < N; ++k) order[k] = perm[k];
    }
  } while (std::next_permutation(perm, perm + N));
  return TK_OK;
}

size_t als_workspace_bytes(int32_t which, int32_t a_dtype, int32_t N, const int64_t* dims,
                           const int32_t* ranks) {
  if ((which != 0 && which != 1) || !valid_dtype(a_dtype) || !valid_dims(N, dims) ||
      !valid_ranks(N, dims, ranks))
    return 0;
  return driver_ws(which, a_dtype, N, dims, ranks);
}

int als_sthosvd(const void* A, int32_t a_dtype, int32_t N, const int64_t* dims,
                const int32_t* ranks, const tk_als_opts* opts, void* const* U, void* G,
                void* ws, size_t ws_bytes, tk_als_info* info, void* stream) {
  return run_driver(1, A, a_dtype, N, dims, ranks, opts, U, G, ws, ws_bytes, info, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free st-HOSVD-ALS: the workspace is a file-scope device array, one
// copy per GPU, held until the process ends.  In host code `scratch` only names
// the symbol; its device address on the current GPU comes from
// hipGetSymbolAddress, taken once per device and kept.
namespace tk {
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex& scratch_mutex() {
  static std::mutex mu;
  return mu;
}

int scratch_address(void** out) {
  static void* addr[NOALLOC_MAX_DEVICES] = {nullptr};
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return TK_ERR_HIP;
  std::lock_guard<std::mutex> g(scratch_mutex());
  if (!addr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    addr[dev] = p;
  }
  *out = addr[dev];
  return TK_OK;
}

}  // namespace
}  // namespace tk

extern "C" {

size_t als_sthosvd_noalloc_max_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

int als_sthosvd_noalloc(const void* A, int32_t a_dtype, int32_t N, const int64_t* dims,
                        const int32_t* ranks, const tk_als_opts* opts, void* const* U, void* G,
                        tk_als_info* info, void* stream) {
  if (info) memset(info, 0, sizeof(*info));
  if (!valid_dtype(a_dtype)) return TK_ERR_UNSUPPORTED_DTYPE;
  if (!A || !U || !G || !valid_dims(N, dims) || !valid_ranks(N, dims, ranks))
    return TK_ERR_INVALID_ARG;
  if (driver_ws(1, a_dtype, N, dims, ranks) > NOALLOC_SCRATCH_BYTES)
    return TK_ERR_WORKSPACE_TOO_SMALL;
  void* ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc) return rc;
  struct NoAlloc {
    bool prev;
    NoAlloc() : prev(t_no_alloc) { t_no_alloc = true; }
    ~NoAlloc() { t_no_alloc = prev; }
  } guard;
  return run_driver(1, A, a_dtype, N, dims, ranks, opts, U, G, ws, NOALLOC_SCRATCH_BYTES, info,
                    stream);
}

int als_thosvd(const void* A, int32_t a_dtype, int32_t N, const int64_t* dims,
               const int32_t* ranks, const tk_als_opts* opts, void* const* U, void* G,
               void* ws, size_t ws_bytes, tk_als_info* info, void* stream) {
  return run_driver(0, A, a_dtype, N, dims, ranks, opts, U, G, ws, ws_bytes, info, stream);
}

int ttm(const void* X, int32_t x_dtype, int32_t N, const int64_t* dims, int32_t mode,
        const void* M, int32_t m_dtype, int64_t J, int32_t trans_m, void* Y, int32_t y_dtype,
        void* stream) {
  if (!valid_dtype(x_dtype) || !valid_dtype(m_dtype) || !valid_dtype(y_dtype))
    return TK_ERR_UNSUPPORTED_DTYPE;
  if (m_dtype != cdtype(x_dtype) || y_dtype != cdtype(x_dtype)) return TK_ERR_UNSUPPORTED_DTYPE;
  if (!X || !M || !Y || !valid_dims(N, dims) || mode < 0 || mode >= N || J < 1 ||
      (trans_m != 0 && trans_m != 1))
    return TK_ERR_INVALID_ARG;
  int rc = ttm_enqueue(X, x_dtype, N, dims, mode, M, J, trans_m, Y, (hipStream_t)stream);
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? TK_OK : TK_ERR_HIP;
}

size_t tucker_reconstruct_workspace_bytes(int32_t dtype, int32_t N, const int32_t* ranks,
                                          const int64_t* dims) {
  if ((dtype != TK_F64 && dtype != TK_F32) || !valid_dims(N, dims) || !ranks) return 0;
  int64_t cur[TK_MAX_ORDER];
  for (int k = 0; k < N; ++k) {
    if (ranks[k] < 1) return 0;
    cur[k] = ranks[k];
  }
  int64_t ea = 1, eb = 1;
  for (int t = 0; t < N - 1; ++t) {
    cur[t] = dims[t];
    int64_t e = numel(N, cur);
    if (t % 2 == 0) ea = std::max(ea, e);
    else eb = std::max(eb, e);
  }
  return align_up(ea * dsize(dtype)) + align_up(eb * dsize(dtype)) + 256;
}

int tucker_reconstruct(const void* G, int32_t dtype, int32_t N, const int32_t* ranks,
                       const int64_t* dims, const void* const* U, void* out, void* ws,
                       size_t ws_bytes, void* stream) {
  if (dtype != TK_F64 && dtype != TK_F32) return TK_ERR_UNSUPPORTED_DTYPE;
  if (!G || !U || !out || !valid_dims(N, dims) || !ranks) return TK_ERR_INVALID_ARG;
  for (int n = 0; n < N; ++n)
    if (!U[n] || ranks[n] < 1) return TK_ERR_INVALID_ARG;
  size_t need = tucker_reconstruct_workspace_bytes(dtype, N, ranks, dims);
  if (N > 1 && (!ws || ws_bytes < need)) return TK_ERR_WORKSPACE_TOO_SMALL;
  hipStream_t s = (hipStream_t)stream;
  int64_t cur[TK_MAX_ORDER];
  for (int k = 0; k < N; ++k) cur[k] = ranks[k];
  int64_t ea = 1;
  {
    int64_t c2[TK_MAX_ORDER];
    for (int k = 0; k < N; ++k) c2[k] = ranks[k];
    for (int t = 0; t < N - 1; t += 2) {
      c2[t] = dims[t];
      ea = std::max(ea, numel(N, c2));
      if (t + 1 < N) c2[t + 1] = dims[t + 1];
    }
  }
  Arena ar(ws, ws_bytes);
  int64_t eA = 1, eB = 1;
  {
    int64_t c3[TK_MAX_ORDER];
    for (int k = 0; k < N; ++k) c3[k] = ranks[k];
    for (int t = 0; t < N - 1; ++t) {
      c3[t] = dims[t];
      if (t % 2 == 0) eA = std::max(eA, numel(N, c3));
      else eB = std::max(eB, numel(N, c3));
    }
  }
  void* bufA = ar.take(eA * dsize(dtype));
  void* bufB = ar.take(eB * dsize(dtype));
  const void* X = G;
  for (int t = 0; t < N; ++t) {
    void* dst = (t == N - 1) ? out : ((t % 2 == 0) ? bufA : bufB);
    int rc = ttm_enqueue(X, dtype, N, cur, t, U[t], dims[t], 0, dst, s);
    if (rc) return rc;
    cur[t] = dims[t];
    X = dst;
  }
  return hipGetLastError() == hipSuccess ? TK_OK : TK_ERR_HIP;
}

size_t contract_allbut_workspace_bytes(int32_t dtype, int32_t N, const int64_t* xdims,
                                       int32_t mode, int64_t J) {
  if ((dtype != TK_F64 && dtype != TK_F32) || !valid_dims(N, xdims) || mode < 0 ||
      mode >= N || J < 1 || J > 64)
    return 0;
  View v = mode_view(N, xdims, mode);
  int chunks = lpass_chunks(v, J, NWG_MAX);
  return align_up((size_t)chunks * v.I * J * dsize(dtype)) + align_up(v.I * J * 8) +
         align_up((size_t)(REDUCE_GROUPS / 4) * v.I * J * 8) + 256;
}

int contract_allbut(const void* X, const void* Y, int32_t dtype, int32_t N,
                    const int64_t* xdims, int32_t mode, int64_t J, void* K, void* ws,
                    size_t ws_bytes, void* stream) {
  if (dtype != TK_F64 && dtype != TK_F32) return TK_ERR_UNSUPPORTED_DTYPE;
  if (!X || !Y || !K || !valid_dims(N, xdims) || mode < 0 || mode >= N || J < 1 || J > 64)
    return TK_ERR_INVALID_ARG;
  size_t need = contract_allbut_workspace_bytes(dtype, N, xdims, mode, J);
  if (!ws || ws_bytes < need) return TK_ERR_WORKSPACE_TOO_SMALL;
  hipStream_t s = (hipStream_t)stream;
  View v = mode_view(N, xdims, mode);
  int chunks = lpass_chunks(v, J, NWG_MAX);
  Arena ar(ws, ws_bytes);
  void* parts = ar.take((size_t)chunks * v.I * J * dsize(dtype));
  double* red = (double*)ar.take(v.I * J * 8);
  double* rtmp = (double*)ar.take((size_t)(REDUCE_GROUPS / 4) * v.I * J * 8);
  LpassArgs a{};
  a.X = X; a.x_dtype = dtype; a.v = v; a.v_kind = 2; a.V = Y; a.R = J; a.parts = parts;
  launch_lpass(a, chunks, s);
  const int64_t n = v.I * J;
  if (dtype == TK_F64) {
    launch_reduce_parts<double>((const double*)parts, chunks, n, n, red, rtmp, s);
    launch_convert<double>(red, n, (double*)K, s);
  } else {
    launch_reduce_parts<float>((const float*)parts, chunks, n, n, red, rtmp, s);
    launch_convert<float>(red, n, (float*)K, s);
  }
  return hipGetLastError() == hipSuccess ? TK_OK : TK_ERR_HIP;
}

int als_init_step(const void* A, int32_t a_dtype, int32_t N, const int64_t* dims, int32_t mode,
                  int32_t R, uint64_t seed, void* Y, void* L0, double* norm2, void* ws,
                  size_t ws_bytes, void* stream) {
  if (!valid_dtype(a_dtype)) return TK_ERR_UNSUPPORTED_DTYPE;
  if (!A || !Y || !L0 || !norm2 || !valid_dims(N, dims) || mode < 0 || mode >= N || R < 1 ||
      R > 64 || R > dims[mode])
    return TK_ERR_INVALID_ARG;
  View v = mode_view(N, dims, mode);
  Arena meas(nullptr, (size_t)-1);
  ModeWs w;
  carve_mode(meas, a_dtype, v, R, w);
  if (!ws || ws_bytes < meas.off) return TK_ERR_WORKSPACE_TOO_SMALL;
  Arena ar(ws, ws_bytes);
  carve_mode(ar, a_dtype, v, R, w);
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipMemsetAsync(w.st, 0, sizeof(DevStatus), s));
  init_enqueue(A, a_dtype, v, R, seed, mode, w, (double*)Y, &w.st->norm2, s);
  qr_enqueue((const double*)Y, v.I, R, (double*)L0, w.Q1, &w.st->status, s);
  DevStatus h{};
  int rc = read_status(w.st, &h, s);
  if (rc) return rc;
  *norm2 = h.norm2;
  return h.status;
}

int als_sweep_step(const void* A, int32_t a_dtype, int32_t N, const int64_t* dims,
                   int32_t mode, int32_t R, const void* L, void* L_next, double norm2,
                   int32_t resid_mode, double* res2, void* ws, size_t ws_bytes,
                   void* stream) {
  if (!valid_dtype(a_dtype)) return TK_ERR_UNSUPPORTED_DTYPE;
  if (!A || !L || !L_next || !res2 || !valid_dims(N, dims) || mode < 0 || mode >= N ||
      R < 1 || R > 64 || R > dims[mode] ||
      (resid_mode != TK_RESID_TRACE && resid_mode != TK_RESID_EXPLICIT))
    return TK_ERR_INVALID_ARG;
  View v = mode_view(N, dims, mode);
  Arena meas(nullptr, (size_t)-1);
  ModeWs w;
  carve_mode(meas, a_dtype, v, R, w);
  if (!ws || ws_bytes < meas.off) return TK_ERR_WORKSPACE_TOO_SMALL;
  Arena ar(ws, ws_bytes);
  carve_mode(ar, a_dtype, v, R, w);
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipMemsetAsync(w.st, 0, sizeof(DevStatus), s));
  HIPCHK(hipMemcpyAsync(w.L, L, v.I * (size_t)R * 8, hipMemcpyDeviceToDevice, s));
  {
    // L~, its quantised Gram factor and the compute-type L for this sweep
    StepArgs p{};
    p.m = v.I; p.r = R; p.ops = STEP_PREP;
    p.Qin = w.L;
    mode_step_grid(p, w, R);
    p.Lq = w.Lq; p.Lr = resid_mode == TK_RESID_EXPLICIT ? w.Lr : nullptr; p.Wq = w.Wq;
    p.lq_bf16 = lq_rounded(a_dtype, resid_mode);
    p.status = &w.st->status; p.prep_status = &w.st->prep_status[0];
    launch_mode_step(p, cdtype(a_dtype), s);
  }
  sweep_enqueue(A, a_dtype, v, R, norm2, resid_mode, w, s);
  HIPCHK(hipMemcpyAsync(L_next, w.Lnext, v.I * (size_t)R * 8, hipMemcpyDeviceToDevice, s));
  DevStatus h{};
  int rc = read_status(w.st, &h, s);
  if (rc) return rc;
  *res2 = h.res[0][0];
  return h.status;
}

int qr_f64(const void* L, int64_t m, int32_t r, void* Q, void* Rhat, void* ws, size_t ws_bytes,
           void* stream) {
  if (!L || !Q || Rhat || m < 1 || r < 1 || r > 64 || r > m) return TK_ERR_INVALID_ARG;
  size_t need = align_up(m * (size_t)r * 8) + 2 * align_up(64 * 64 * 8) + align_up(64);
  if (!ws || ws_bytes < need) return TK_ERR_WORKSPACE_TOO_SMALL;
  Arena ar(ws, ws_bytes);
  double* Q1 = (double*)ar.take(m * (size_t)r * 8);
  double* C1 = (double*)ar.take(64 * 64 * 8);
  double* C2 = (double*)ar.take(64 * 64 * 8);
  DevStatus* st = (DevStatus*)ar.take(sizeof(DevStatus));
  (void)C1; (void)C2;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipMemsetAsync(st, 0, sizeof(DevStatus), s));
  qr_enqueue((const double*)L, m, r, (double*)Q, Q1, &st->status, s);
  DevStatus h{};
  int rc = read_status(st, &h, s);
  if (rc) return rc;
  return h.status;
}

}  // extern "C"

namespace tk {
namespace {

// ---------------------------------------------------------------------------
// Batched st-HOSVD-ALS: persistent launch captured in a HIP graph.

constexpr int BATCH_WG_PER_CU = 2;
constexpr int BATCH_CUS = 256;

struct BatchPlan {
  bool persistent;
  int64_t belems;
  int nwg;
  size_t desc_bytes, slot_bytes, total;
};

BatchPlan plan_batch(int count, const int64_t* dims3, const int32_t* ranks3) {
  BatchPlan p{};
  p.persistent = true;
  int64_t be = 1;
  size_t seq = 0;
  for (int t = 0; t < count; ++t) {
    const int64_t* d = dims3 + 3 * t;
    const int32_t* r = ranks3 + 3 * t;
    int32_t d32[3] = {(int32_t)d[0], (int32_t)d[1], (int32_t)d[2]};
    if (d[0] > 128 || d[1] > 128 || d[2] > 128 || !batched_shape_ok(d32, r)) p.persistent = false;
    be = std::max(be, (int64_t)r[0] * d[1] * d[2]);
    be = std::max(be, (int64_t)r[0] * r[1] * d[2]);
    seq = std::max(seq, driver_ws(1, TK_F32, 3, d, r));
  }
  p.belems = be;
  p.nwg = std::min(count, BATCH_WG_PER_CU * BATCH_CUS);
  p.desc_bytes = align_up(batched_desc_bytes() * count);
  p.slot_bytes = align_up(batched_slot_bytes(be));
  if (p.persistent)
    p.total = p.desc_bytes + align_up(4 * (size_t)count) + align_up(12 * (size_t)count) + 256 +
              p.slot_bytes * p.nwg;
  else
    p.total = seq;
  return p;
}

// Autotuned tile shape per (count bucket, largest mode size, largest rank),
// kept for the process and, when TK_AUTOTUNE_CACHE names a file, in that
// file as "key cfg" lines.
std::map<std::string, int>& tune_cache() {
  static std::map<std::string, int> m;
  return m;
}
std::mutex& tune_mutex() {
  static std::mutex mu;
  return mu;
}

std::string tune_key(int count, const int64_t* dims3, const int32_t* ranks3) {
  int64_t mi = 0;
  int mr = 0, cb = 1;
  for (int t = 0; t < 3 * count; ++t) {
    mi = std::max(mi, dims3[t]);
    mr = std::max(mr, (int)ranks3[t]);
  }
  while (cb < count) cb <<= 1;
  char buf[128];
  snprintf(buf, sizeof buf, "gfx950/batched/n%d/i%lld/r%d", cb, (long long)mi, mr);
  return buf;
}

int tune_lookup(const std::string& key) {
  std::lock_guard<std::mutex> g(tune_mutex());
  auto& m = tune_cache();
  auto it = m.find(key);
  if (it != m.end()) return it->second;
  const char* path = getenv("TK_AUTOTUNE_CACHE");
  if (path) {
    if (FILE* f = fopen(path, "r")) {
      char k[256];
      int c;
      while (fscanf(f, "%255s %d", k, &c) == 2) m[k] = c;
      fclose(f);
    }
    it = m.find(key);
    if (it != m.end()) return it->second;
  }
  return -1;
}

void tune_store(const std::string& key, int cfg) {
  std::lock_guard<std::mutex> g(tune_mutex());
  tune_cache()[key] = cfg;
  if (const char* path = getenv("TK_AUTOTUNE_CACHE")) {
    if (FILE* f = fopen(path, "a")) {
      fprintf(f, "%s %d\n", key.c_str(), cfg);
      fclose(f);
    }
  }
}

// Instantiated graphs of the batched launch, by launch key (buffers, shapes,
// options, tile shape); a small cache, oldest entry evicted.
struct GraphCache {
  std::mutex mu;
  std::vector<std::pair<std::string, hipGraphExec_t>> entries;
};
GraphCache& graph_cache() {
  static GraphCache* c = new GraphCache();   // kept until the process ends
  return *c;
}
constexpr size_t GRAPH_CACHE_MAX = 8;

hipGraphExec_t graph_lookup(const std::string& key) {
  GraphCache& c = graph_cache();
  std::lock_guard<std::mutex> g(c.mu);
  for (auto& e : c.entries)
    if (e.first == key) return e.second;
  return nullptr;
}

void graph_store(const std::string& key, hipGraphExec_t exec) {
  GraphCache& c = graph_cache();
  std::lock_guard<std::mutex> g(c.mu);
  if (c.entries.size() >= GRAPH_CACHE_MAX) {
    (void)hipGraphExecDestroy(c.entries.front().second);
    c.entries.erase(c.entries.begin());
  }
  c.entries.emplace_back(key, exec);
}

// FNV-1a over the descriptor table (part of the launch key).
uint64_t desc_hash(const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

// Times every tile shape on the batch itself (second of two runs each).
int autotune_batched(const BatchLaunch& L, hipStream_t s, int* best_out) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  float best = 1e30f;
  int bc = 0;
  for (int cfg = 0; cfg < BATCHED_CONFIGS; ++cfg) {
    float ms = 0.0f;
    for (int rep = 0; rep < 2; ++rep) {
      HIPCHK(hipEventRecord(e0, s));
      launch_batched(L, cfg, s);
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    }
    if (ms < best) { best = ms; bc = cfg; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *best_out = bc;
  return TK_OK;
}

}  // namespace
}  // namespace tk

extern "C" {

size_t als_sthosvd_batched_workspace_bytes(int32_t count, const int64_t* dims3,
                                           const int32_t* ranks3) {
  if (count < 1 || !dims3 || !ranks3) return 0;
  for (int t = 0; t < count; ++t)
    if (!valid_dims(3, dims3 + 3 * t) || !valid_ranks(3, dims3 + 3 * t, ranks3 + 3 * t))
      return 0;
  return plan_batch(count, dims3, ranks3).total;
}

int als_sthosvd_batched(const void* A_packed, int32_t a_dtype, int32_t count,
                        const int64_t* dims3, const int32_t* ranks3, const int64_t* a_off,
                        const tk_als_opts* opts, void* U_packed, const int64_t* u_off,
                        void* G_packed, const int64_t* g_off, int32_t* iters, int32_t* status,
                        void* ws, size_t ws_bytes, void* stream) {
  if (a_dtype != TK_F32) return TK_ERR_UNSUPPORTED_DTYPE;
  if (!A_packed || count < 1 || !dims3 || !ranks3 || !a_off || !U_packed || !u_off ||
      !G_packed || !g_off)
    return TK_ERR_INVALID_ARG;
  size_t need = als_sthosvd_batched_workspace_bytes(count, dims3, ranks3);
  if (need == 0) return TK_ERR_INVALID_ARG;
  if (!ws || ws_bytes < need) return TK_ERR_WORKSPACE_TOO_SMALL;
  Opts o;
  int rc = read_opts(opts, 3, o);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const BatchPlan plan = plan_batch(count, dims3, ranks3);
  int worst = TK_OK;
  if (!plan.persistent) {
    // shapes beyond the persistent kernel's limits: one tensor at a time
    for (int t = 0; t < count; ++t) {
      const float* A = (const float*)A_packed + a_off[t];
      void* U[3];
      for (int n = 0; n < 3; ++n) U[n] = (float*)U_packed + u_off[3 * t + n];
      void* G = (float*)G_packed + g_off[t];
      tk_als_info info;
      tk_als_opts o2;
      memset(&o2, 0, sizeof(o2));
      o2.struct_size = sizeof(o2);
      o2.tol = o.tol; o2.max_iters = o.max_iters; o2.resid_mode = o.resid_mode; o2.seed = o.seed;
      rc = run_driver(1, A, TK_F32, 3, dims3 + 3 * t, ranks3 + 3 * t, &o2, U, G, ws, ws_bytes,
                      &info, stream);
      if (status) status[t] = rc;
      if (iters)
        for (int n = 0; n < 3; ++n) iters[3 * t + n] = info.iters[n];
      if (rc < 0 && (worst >= 0 || rc < worst)) worst = rc;
      else if (rc > 0 && worst == TK_OK) worst = rc;
    }
    return worst;
  }
  // descriptor table, largest tensors first (the work queue then balances)
  std::vector<int> ord(count);
  for (int t = 0; t < count; ++t) ord[t] = t;
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
    return dims3[3 * x] * dims3[3 * x + 1] * dims3[3 * x + 2] >
           dims3[3 * y] * dims3[3 * y + 1] * dims3[3 * y + 2];
  });
  std::vector<char> hdesc(plan.desc_bytes);
  for (int k = 0; k < count; ++k) {
    const int t = ord[k];
    fill_desc(hdesc.data(), k, t, a_off[t], g_off[t], u_off + 3 * t, dims3 + 3 * t,
              ranks3 + 3 * t);
  }
  Arena ar(ws, ws_bytes);
  void* ddesc = ar.take(plan.desc_bytes);
  int32_t* dstatus = (int32_t*)ar.take(4 * (size_t)count);
  int32_t* diters = (int32_t*)ar.take(12 * (size_t)count);
  int* queue = (int*)ar.take(256);
  char* scratch = (char*)ar.take(plan.slot_bytes * plan.nwg);
  HIPCHK(hipMemcpyAsync(ddesc, hdesc.data(), batched_desc_bytes() * count,
                        hipMemcpyHostToDevice, s));
  BatchLaunch L{};
  L.A = (const float*)A_packed; L.desc = ddesc; L.count = count;
  L.U = (float*)U_packed; L.G = (float*)G_packed;
  L.status = dstatus; L.iters = diters; L.queue = queue;
  L.scratch = scratch; L.slot_bytes = (int64_t)plan.slot_bytes; L.belems = plan.belems;
  L.tol = o.tol; L.max_iters = o.max_iters; L.resid_mode = o.resid_mode; L.seed = o.seed;
  L.nwg = plan.nwg;
  const std::string key = tune_key(count, dims3, ranks3);
  int cfg = tune_lookup(key);
  if (cfg < 0) {
    rc = autotune_batched(L, s, &cfg);
    if (rc) return rc;
    tune_store(key, cfg);
  }
  // the queue reset and the persistent kernel, captured once in a graph on a
  // private stream and replayed on the caller's stream; the instantiated graph
  // is kept for later calls with the same launch (buffers, shapes, options)
  char gk[512];
  snprintf(gk, sizeof gk, "%s/cfg%d/A%p/U%p/G%p/ws%p/n%d/t%.17g/m%d/r%d/s%llu/h%016llx",
           key.c_str(), cfg, A_packed, U_packed, G_packed, ws, count, o.tol, o.max_iters,
           o.resid_mode, (unsigned long long)o.seed,
           (unsigned long long)desc_hash(hdesc.data(), batched_desc_bytes() * count));
  hipGraphExec_t exec = graph_lookup(gk);
  if (!exec) {
    hipStream_t cs;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      launch_batched(L, cfg, cs);
      ok = hipStreamEndCapture(cs, &graph) == hipSuccess;
    }
    if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
    if (!ok) {
      if (exec) (void)hipGraphExecDestroy(exec);
      return TK_ERR_HIP;
    }
    graph_store(gk, exec);
  }
  bool ok = hipGraphLaunch(exec, s) == hipSuccess;
  if (ok) ok = hipStreamSynchronize(s) == hipSuccess;
  if (!ok) return TK_ERR_HIP;
  std::vector<int32_t> hs(count), hi(3 * (size_t)count);
  HIPCHK(hipMemcpy(hs.data(), dstatus, 4 * (size_t)count, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(hi.data(), diters, 12 * (size_t)count, hipMemcpyDeviceToHost));
  for (int t = 0; t < count; ++t) {
    if (status) status[t] = hs[t];
    if (iters)
      for (int n = 0; n < 3; ++n) iters[3 * t + n] = hi[3 * t + n];
    const int rc2 = hs[t];
    if (rc2 < 0 && (worst >= 0 || rc2 < worst)) worst = rc2;
    else if (rc2 > 0 && worst == TK_OK) worst = rc2;
  }
  return worst;
}

}  // extern "C"

extern "C" int als_sweep_kernel(const void* A, int32_t a_dtype, int32_t N, const int64_t* dims,
                                int32_t mode, int32_t R, const float* Lq, double* Lacc,
                                double* GV, int32_t reduce, void* ws, size_t ws_bytes,
                                void* stream) {
  if (a_dtype != TK_F32 && a_dtype != TK_BF16) return TK_ERR_UNSUPPORTED_DTYPE;
  if (!A || !Lq || !valid_dims(N, dims) || mode < 0 || mode >= N || R < 1 || R > 64 ||
      R > dims[mode] || (reduce && (!Lacc || !GV)))
    return TK_ERR_INVALID_ARG;
  View v = mode_view(N, dims, mode);
  Arena meas(nullptr, (size_t)-1);
  ModeWs w;
  carve_mode(meas, a_dtype, v, R, w);
  if (!ws || ws_bytes < meas.off) return TK_ERR_WORKSPACE_TOO_SMALL;
  Arena ar(ws, ws_bytes);
  carve_mode(ar, a_dtype, v, R, w);
  hipStream_t s = (hipStream_t)stream;
  const int64_t IR = v.I * (int64_t)R;
  if (a_dtype == TK_BF16) {
    // BF16 sweeps multiply by L~ rounded to BF16 precision (as the drivers
    // prepare it): round a copy
    HIPCHK(hipMemcpyAsync(w.Lr, Lq, (size_t)IR * 4, hipMemcpyDeviceToDevice, s));
    launch_round_bf16((float*)w.Lr, IR, s);
    Lq = (const float*)w.Lr;
  }
  if (fused_supported(a_dtype, v, R, TK_RESID_TRACE)) {
    FusedArgs f{};
    f.X = A; f.x_dtype = a_dtype; f.v = v; f.R = R;
    f.Lq = Lq;
    f.lq_bf16 = a_dtype == TK_BF16;
    f.lacc_parts = (float*)w.parts;
    f.gv_parts = w.gparts;
    int nwg = launch_fused(f, NWG_MAX, s);
    if (reduce) {
      launch_reduce_parts<float>((const float*)w.parts, nwg, IR, IR, Lacc, w.rtmp, s);
      launch_reduce_parts<double>(w.gparts, FUSED_WAVES * nwg, (int64_t)R * R, (int64_t)R * R, GV,
                                  w.rtmp, s);
    }
  } else {
    VpassArgs a{};
    a.X = A; a.x_dtype = a_dtype; a.v = v;
    a.W = Lq; a.w_ldi = R; a.w_ldo = 1; a.O = R;
    a.out = w.V; a.out_kind = 0;
    int nres = 0;
    launch_vpass(a, NWG_MAX, &nres, s);
    int gch = (int)std::min<int64_t>(NWG_MAX, std::max<int64_t>(1, ceil_div(v.J(), 4096)));
    launch_gram_parts(w.V, TK_F32, v.J(), R, gch, w.gparts, s);
    LpassArgs l{};
    l.X = A; l.x_dtype = a_dtype; l.v = v; l.v_kind = 0; l.V = w.V; l.R = R;
    l.parts = w.parts;
    int chunks = lpass_chunks(v, R, NWG_MAX);
    launch_lpass(l, chunks, s);
    if (reduce) {
      launch_reduce_parts<double>(w.gparts, gch, (int64_t)R * R, (int64_t)R * R, GV, w.rtmp, s);
      launch_reduce_parts<float>((const float*)w.parts, chunks, IR, IR, Lacc, w.rtmp, s);
    }
  }
  return hipGetLastError() == hipSuccess ? TK_OK : TK_ERR_HIP;
}
