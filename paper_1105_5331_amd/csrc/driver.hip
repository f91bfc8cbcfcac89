// Host side of the C ABI: argument checks, the objective/gradient and ALS
// sweep built from the device kernels, the N-GMRES iteration (Section 2.1,
// Steps I-III) with its Moré–Thuente line search, and cp_decompose.
//
// Everything iterate-sized stays on the device.  Per N-GMRES iteration the
// host reads back: rho at the top (1 double), the slope g(u_bar)^T d after
// Step II (1 double), and (f, phi') for every line-search trial (2 doubles).
#include "common.hpp"
#include "linesearch.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

using namespace cpng;
using cpng::ls::LS_CONVERGED;

struct cp_ngmres_state {
  const cp_tensor* T = nullptr;
  Shape s;
  int R = 0;
  int64_t L = 0;
  cp_options opt{};
  hipStream_t st = nullptr;
  int prec = CP_PREC_FP64;
  bool switched = false;
  int it = 0;
  double f = 0.0, rho = 0.0, normT = 0.0;
  int n_fg = 0, n_restarts = 0, n_fallback = 0, switch_iter = -1;
  bool stalled = false;   // a line search in reduced precision ended without a Wolfe point
  bool cg_fresh = true;   // N-CG: the next direction is -g (start, switch, failed search)
  // The left partial X_L in the handle's ybuf is the one at u (the last
  // evaluation was at u, in N-GMRES rescaled for u's normalisation) while
  // xl_ok and no call has written ybuf since (ywrites, ybuf's address): the
  // next ALS sweep then skips its left pass (mttkrp_tree = 1; N-GMRES with
  // ALS as the one-step process, and ALS).
  bool xl_ok = false;
  uint64_t xl_token = 0;
  void* xl_ptr = nullptr;
  bool reuse_xl = false;   // the Steps I-II being enqueued take X_L from ybuf
  // f(u_bar) and the slope g(u_bar)^T d of the last N-GMRES iteration (Steps I-II)
  bool have_last = false;
  double last_fbar = 0.0, last_slope = 0.0;
  // device buffers
  double* mem = nullptr;
  double *u, *g, *ubar, *gbar, *uhat, *d, *ut, *gt, *gbest, *scal;  // scal: 8 doubles
  double *winU, *winG;
  int wcap = 0, wcount = 0, whead = 0;   // ring buffer: slot (whead + j) % wcap, j oldest first
  // Step II / line-search values: host copy (pinned) and device copy
  StepPar* hpar = nullptr;
  StepPar* dpar = nullptr;
  // Captured launch sequences of the two device phases of an iteration
  // (Steps I-II up to the slope; one line-search evaluation), replayed with
  // hipGraphLaunch.  Used only on a non-null stream without profiling.
  struct Captured {
    hipGraphExec_t exec = nullptr;
    cp_handle* h = nullptr;
    uint64_t gen = 0;
    int prec = -1;
    bool warm = false;     // ran once eagerly at the current precision
    bool failed = false;   // capture not possible: stay eager
    int64_t passes = 0;    // passes over T per replay
    uint64_t ywrites = 0;  // writes of the handle's ybuf per replay
  } cap[3];
};

namespace {

bool is_f64_acc(int p) { return p == CP_PREC_FP64 || p == CP_PREC_FP32IN_FP64ACC; }

// N-GMRES with either one-step process keeps the window of iterates
bool uses_window(int method) { return method == CP_METHOD_NGMRES || method == CP_METHOD_NGMRES_SD; }

int check_prec(cp_handle* h, const cp_tensor* T, int p) {
  if (p < 0 || p > 3) return fail(h, CP_EINVAL, "unknown precision %d", p);
  if ((p == CP_PREC_FP32 || p == CP_PREC_BF16X3) && T->dtype != CP_F32)
    return fail(h, CP_EINVAL, "precision %d needs a float32 tensor", p);
  if (p == CP_PREC_BF16X3 && T->sparse)
    return fail(h, CP_EINVAL, "BF16X3 applies to dense tensors only");
  return CP_OK;
}

int check_tensor(cp_handle* h, const cp_tensor* T, Shape* s) {
  if (!T) return fail(h, CP_EINVAL, "null tensor");
  CP_TRY(make_shape(h, T->order, T->dims, s));
  if (T->dtype != CP_F32 && T->dtype != CP_F64) return fail(h, CP_EINVAL, "bad dtype %d", T->dtype);
  if (!T->sparse && !T->values) return fail(h, CP_EINVAL, "dense tensor without values");
  if (!T->sparse && s->total() > (int64_t(1) << 40))
    return fail(h, CP_EINVAL, "dense tensor too large");
  return CP_OK;
}

int check_mttkrp_args(cp_handle* h, const cp_tensor* T, const double* u, int R, int mode, int p,
                      const double* M_out, Shape* s) {
  CP_TRY(check_tensor(h, T, s));
  if (R < 1) return fail(h, CP_EINVAL, "rank %d < 1", R);
  if (mode < 0 || mode >= s->N) return fail(h, CP_EINVAL, "mode %d outside 0..%d", mode, s->N - 1);
  if (!u || !M_out) return fail(h, CP_EINVAL, "null factor or output pointer");
  CP_TRY(check_prec(h, T, p));
  if (T->sparse && R > 64) return fail(h, CP_EINVAL, "sparse MTTKRP supports R <= 64");
  return CP_OK;
}

int check_rank(cp_handle* h, int R) {
  if (R < 1 || R > 64) return fail(h, CP_EINVAL, "rank %d outside 1..64", R);
  return CP_OK;
}

int mttkrp_any(cp_handle* h, const cp_tensor* T, const Shape& s, const double* u, int R, int mode,
               int prec, double* M, hipStream_t st) {
  if (T->sparse) return sparse_mttkrp(h, T, s, u, R, mode, prec, M, st);
  return dense_mttkrp(h, T, s, u, R, mode, prec, M, st);
}

// Internal buffers: M for every mode (sum_dims x R), S/Gbar/Gam, scalars.
struct Scratch {
  double* M;      // N blocks, mode n at off[n]*R
  double* S;      // N R R
  double* Gbar;   // N R R
  double* Gam;    // R R
  double* dot;    // 4 doubles
};

int mode_buffers(cp_handle* h, const Shape& s, int R, hipStream_t st, Scratch* sc) {
  const size_t L = (size_t)s.sum_dims() * R;
  const size_t need = L + (size_t)(2 * s.N * R * R + R * R + 8);
  CP_TRY(ensure(h, h->mbuf, sizeof(double) * need, st));
  double* b = static_cast<double*>(h->mbuf.ptr);
  sc->M = b;
  sc->S = b + L;
  sc->Gbar = sc->S + s.N * R * R;
  sc->Gam = sc->Gbar + s.N * R * R;
  sc->dot = sc->Gam + R * R;
  return CP_OK;
}

// Buffers of the two-level evaluation (tree.hip): the partial of each mode
// group with more than one mode, float64, in the handle's workspace.
struct TreeBufs {
  int split = 0;            // 0: one MTTKRP pass per mode
  double* XL = nullptr;     // modes [0, split)
  double* XR = nullptr;     // modes [split, N)
};

int tree_setup(cp_handle* h, const cp_tensor* T, const Shape& s, int R, int prec, bool tree,
               hipStream_t st, TreeBufs* tb) {
  *tb = TreeBufs{};
  if (!tree) return CP_OK;
  const int split = tree_split(T, s, prec);
  if (!split) return CP_OK;
  const size_t nl = tree_partial_elems(s, split, R, true);
  const size_t nr = tree_partial_elems(s, split, R, false);
  CP_TRY(ensure(h, h->ybuf, sizeof(double) * (nl + nr), st));
  double* b = static_cast<double*>(h->ybuf.ptr);
  h->ywrites++;   // the caller writes (at least one of) the partials
  tb->split = split;
  if (nl) tb->XL = b;
  if (nr) tb->XR = b + nl;
  return CP_OK;
}

// The left partial of the two-level evaluation of S's tensor in the handle's
// ybuf, where that evaluation has one (dense, order >= 3, left group of two
// or more modes) and ybuf is large enough to hold it.
bool tree_left_buffer(cp_handle* h, const cp_tensor* T, const Shape& s, int R, int prec, int* split,
                      double** XL) {
  const int sp = tree_split(T, s, prec);
  if (!sp) return false;
  const size_t nl = tree_partial_elems(s, sp, R, true);
  const size_t nr = tree_partial_elems(s, sp, R, false);
  if (!nl || !h->ybuf.ptr || h->ybuf.bytes < sizeof(double) * (nl + nr)) return false;
  *split = sp;
  *XL = static_cast<double*>(h->ybuf.ptr);
  return true;
}

// M^(n) from its group's partial (formed beforehand), or by its own pass over T.
int mode_mttkrp(cp_handle* h, const cp_tensor* T, const Shape& s, const double* u, int R, int n,
                int prec, const TreeBufs& tb, double* Mn, hipStream_t st) {
  if (tb.XL && n < tb.split) return tree_mode(h, s, 0, tb.split, tb.XL, u, R, n, Mn, st);
  if (tb.XR && n >= tb.split) return tree_mode(h, s, tb.split, s.N, tb.XR, u, R, n, Mn, st);
  return mttkrp_any(h, T, s, u, R, n, prec, Mn, st);
}

// f and g at u: all N MTTKRPs at the same point (Section 2.3), the gradient
// epilogue G^(n) = -M^(n) + A^(n) Gammabar^(n) and the objective from the
// last mode's M and Gamma.  With `tree` != 0 (dense, order >= 3) the MTTKRPs
// come from the two group partials: T is streamed twice, or, with tree == 1
// where the two-sided kernel covers the shape, once for both partials.
int objective_grad_impl(cp_handle* h, const cp_tensor* T, const Shape& s, const double* u, int R,
                        int prec, double* f_out, double* g_out, hipStream_t st, int tree = 1) {
  Scratch sc;
  CP_TRY(mode_buffers(h, s, R, st, &sc));
  CP_TRY(gram_all(h, s, u, R, sc.S, sc.Gbar, sc.Gam, st));
  TreeBufs tb;
  CP_TRY(tree_setup(h, T, s, R, prec, tree != 0, st, &tb));
  int one = 1;
  if (tree == 1 && tb.XL && tb.XR) {
    one = tree_partials_one_pass(h, T, s, u, R, prec, tb.split, tb.XL, tb.XR, st);
    if (one < 0) return one;
  }
  if (one != CP_OK) {
    if (tb.XL) CP_TRY(tree_partial(h, T, s, u, R, prec, tb.split, true, tb.XL, st));
    if (tb.XR) CP_TRY(tree_partial(h, T, s, u, R, prec, tb.split, false, tb.XR, st));
  }
  struct EpiScope {   // the pending epilogue never outlives one MTTKRP call
    cp_handle* h;
    ~EpiScope() { h->epi = GradEpi{}; }
  };
  int all = 1;   // every mode from the partials in one launch when covered
  if (tb.XL && tb.XR) {
    all = tree_all_modes(h, s, tb.split, tb.XL, tb.XR, u, R, sc.M, sc.Gbar, g_out, st);
    if (all < 0) return all;
  }
  for (int n = 0; n < s.N && all != CP_OK; ++n) {
    double* Mn = sc.M + s.off[n] * R;
    const double* An = u + s.off[n] * R;
    double* Gn = g_out ? g_out + s.off[n] * R : nullptr;
    bool fused = false;
    {
      EpiScope scope{h};
      if (Gn) h->epi = GradEpi{An, sc.Gbar + n * R * R, Gn, false};
      CP_TRY(mode_mttkrp(h, T, s, u, R, n, prec, tb, Mn, st));
      fused = h->epi.used;
    }
    if (Gn && !fused)
      CP_TRY(grad_epilogue(h, Mn, An, sc.Gbar + n * R * R, s.dims[n], R, Gn, st));
  }
  if (f_out) {
    const int n = s.N - 1;
    CP_TRY(objective_from_dot(h, u + s.off[n] * R, sc.M + s.off[n] * R, s.dims[n] * R,
                              T->norm_sq, sc.Gam, R, f_out, st));
  }
  return CP_OK;
}

// One ALS sweep (Section 2.3): for n = 1..N in order, A^(n) = M^(n) Gammabar^(n)^-1
// with the factors updated so far.  With `tree`, the left group's partial is
// formed first (the right factors are untouched until the split) and the
// right group's once the left modes are updated.
// With xl_ready the left partial at u is already in the handle's ybuf (the
// caller's last evaluation was at u) and is not formed again.
int als_sweep_impl(cp_handle* h, const cp_tensor* T, const Shape& s, double* u, int R, int prec,
                   int normalize_after, hipStream_t st, bool tree = true, bool xl_ready = false) {
  Scratch sc;
  CP_TRY(mode_buffers(h, s, R, st, &sc));
  TreeBufs tb;
  CP_TRY(tree_setup(h, T, s, R, prec, tree, st, &tb));
  if (tb.XL && !xl_ready) CP_TRY(tree_partial(h, T, s, u, R, prec, tb.split, true, tb.XL, st));
  for (int n = 0; n < s.N; ++n) {
    if (tb.XR && n == tb.split) CP_TRY(tree_partial(h, T, s, u, R, prec, tb.split, false, tb.XR, st));
    // Grams (after mode 0 only the mode updated last changed) and the factor of Gbar^(n)
    CP_TRY(gram_all(h, s, u, R, sc.S, sc.Gbar, nullptr, st, n, n == 0 ? -1 : n - 1));
    double* Mn = sc.M + s.off[n] * R;
    CP_TRY(mode_mttkrp(h, T, s, u, R, n, prec, tb, Mn, st));
    CP_TRY(mode_solve(h, Mn, nullptr, s.dims[n], R, u + s.off[n] * R, st));
  }
  if (normalize_after) CP_TRY(normalize(h, s, u, R, nullptr, st));
  return CP_OK;
}

// Blocking readback of n doubles from device memory.
int readback(cp_handle* h, const double* src, int n, double* dst, hipStream_t st) {
  CP_HIP(h, hipMemcpyAsync(h->pinned, src, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  CP_HIP(h, hipStreamSynchronize(st));
  for (int i = 0; i < n; ++i) dst[i] = h->pinned[i];
  return CP_OK;
}

enum { PHASE_STEP12 = 0, PHASE_EVAL = 1, PHASE_STEP12_XL = 2 };

// The device work of Step II from u_bar and g_bar: the accelerated u_hat
// over the window (normalised), d = u_hat - u_bar and the slope g(u_bar)^T d
// (scal[1]).  Expects the window size and oldest slot in S->dpar.
int enqueue_step2(cp_handle* h, cp_ngmres_state* S) {
  CP_TRY(step2(h, S->L, S->winU, S->winG, S->wcap, S->dpar, S->ubar, S->gbar, S->opt.eps,
               S->uhat, S->scal + 8, S->st));
  if (S->opt.normalize_accel) CP_TRY(normalize(h, S->s, S->uhat, S->R, nullptr, S->st));
  CP_TRY(sub_to(h, S->uhat, S->ubar, S->d, S->L, S->st));
  CP_TRY(dot(h, S->gbar, S->d, S->L, S->scal + 1, S->st));
  return CP_OK;
}

// The device work of Steps I and II with ALS as the one-step process: u_bar =
// M(u_i), f and g at u_bar (scal[0]), then Step II (scal[1]).
int enqueue_step12(cp_handle* h, cp_ngmres_state* S) {
  CP_HIP(h, hipMemcpyAsync(S->dpar, S->hpar, sizeof(StepPar), hipMemcpyHostToDevice, S->st));
  CP_HIP(h, hipMemcpyAsync(S->ubar, S->u, sizeof(double) * S->L, hipMemcpyDeviceToDevice, S->st));
  CP_TRY(als_sweep_impl(h, S->T, S->s, S->ubar, S->R, S->prec, 1, S->st, S->opt.mttkrp_tree != 0,
                        S->reuse_xl));
  CP_TRY(objective_grad_impl(h, S->T, S->s, S->ubar, S->R, S->prec, S->scal, S->gbar, S->st,
                             S->opt.mttkrp_tree));
  return enqueue_step2(h, S);
}

// The device work of one line-search trial: u_t = u_bar + beta d, f and g
// at u_t, and g(u_t)^T d (scal[0], scal[1]).
int enqueue_eval(cp_handle* h, cp_ngmres_state* S) {
  CP_HIP(h, hipMemcpyAsync(S->dpar, S->hpar, sizeof(StepPar), hipMemcpyHostToDevice, S->st));
  CP_TRY(axpy_par(h, S->ubar, S->dpar, S->d, S->ut, S->L, S->st));
  CP_TRY(objective_grad_impl(h, S->T, S->s, S->ut, S->R, S->prec, S->scal, S->gt, S->st,
                             S->opt.mttkrp_tree));
  CP_TRY(dot(h, S->gt, S->d, S->L, S->scal + 1, S->st));
  return CP_OK;
}

void drop_captured(cp_ngmres_state::Captured& c) {
  if (c.exec) (void)hipGraphExecDestroy(c.exec);
  c.exec = nullptr;
  c.warm = false;
}

// Runs a phase: eagerly the first time at a precision (that sizes every
// workspace slice), then captured once and replayed.  A capture that fails
// (e.g. a slice would have to grow) falls back to eager launches for good.
// The host values in S->hpar are copied to the device inside the phase, so
// a replay uses the current ones.
int run_phase(cp_handle* h, cp_ngmres_state* S, int ph) {
  S->reuse_xl = ph == PHASE_STEP12_XL;
  auto enqueue = [&]() { return ph == PHASE_EVAL ? enqueue_eval(h, S) : enqueue_step12(h, S); };
  cp_ngmres_state::Captured& c = S->cap[ph];
  if (!S->st || h->prof || c.failed) return enqueue();
  if (c.h != h || c.gen != h->gen || c.prec != S->prec) drop_captured(c);
  if (c.exec) {
    CP_HIP(h, hipGraphLaunch(c.exec, S->st));
    h->t_passes += c.passes;
    h->ywrites += c.ywrites;
    return CP_OK;
  }
  if (!c.warm) {
    CP_TRY(enqueue());
    c.warm = true;
    c.h = h;
    c.gen = h->gen;
    c.prec = S->prec;
    return CP_OK;
  }
  const uint64_t gen0 = h->gen;
  const int64_t passes0 = h->t_passes;
  const uint64_t ywrites0 = h->ywrites;
  if (hipStreamBeginCapture(S->st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    c.failed = true;
    return enqueue();
  }
  const int rc = enqueue();
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(S->st, &graph);
  (void)hipGetLastError();
  hipGraphExec_t exec = nullptr;
  bool ok = rc >= 0 && e == hipSuccess && graph && h->gen == gen0;
  if (ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    exec = nullptr;
    ok = false;
  }
  if (graph) (void)hipGraphDestroy(graph);
  if (!ok) {   // nothing of the capture ran: do the phase eagerly
    c.failed = true;
    h->t_passes = passes0;
    h->ywrites = ywrites0;
    return enqueue();
  }
  c.exec = exec;
  c.h = h;
  c.gen = h->gen;
  c.prec = S->prec;
  c.passes = h->t_passes - passes0;   // counted while recording, run by the launch below
  c.ywrites = h->ywrites - ywrites0;
  CP_HIP(h, hipGraphLaunch(c.exec, S->st));
  return CP_OK;
}

// Evaluate phi(beta) = f(ubar + beta d), phi'(beta) = g(ubar + beta d)^T d.
int ls_eval(cp_handle* h, cp_ngmres_state* S, double beta, double* f, double* dphi) {
  S->hpar->beta = beta;
  CP_TRY(run_phase(h, S, PHASE_EVAL));
  S->n_fg++;
  double v[2];
  CP_TRY(readback(h, S->scal, 2, v, S->st));
  *f = v[0];
  *dphi = v[1];
  if (!std::isfinite(v[0]) || !std::isfinite(v[1]))
    return fail(h, CP_ENOTFINITE, "objective or slope not finite in the line search");
  return CP_OK;
}

// Runs the search from (f0, g0 < 0).  On return *beta, *f_acc hold the accepted
// step and objective and S->gt (converged) or S->gbest (fallback) its gradient.
int more_thuente(cp_handle* h, cp_ngmres_state* S, double f0, double g0, double* beta,
                 double* f_acc, const double** g_acc, int* nfev_out, int* status_out) {
  ls::MoreThuente mt;
  double stp = mt.start(S->opt, f0, g0);
  for (;;) {
    double f, g;
    CP_TRY(ls_eval(h, S, stp, &f, &g));
    bool keep = false;
    const int status = mt.feed(f, g, &keep);
    // the trial's gradient is kept for a fallback only while the search goes
    // on (a final trial's gradient is still in S->gt)
    if (keep)
      CP_HIP(h, hipMemcpyAsync(S->gbest, S->gt, sizeof(double) * S->L, hipMemcpyDeviceToDevice, S->st));
    if (status >= 0) {
      *nfev_out = mt.nfev;
      *status_out = status;
      *beta = mt.acc_beta;
      *f_acc = mt.acc_f;
      *g_acc = mt.acc_grad == ls::MoreThuente::ACC_LAST ? S->gt
             : mt.acc_grad == ls::MoreThuente::ACC_BEST ? S->gbest : nullptr;
      return CP_OK;
    }
    stp = mt.stp;
  }
}

double* win_u(cp_ngmres_state* S, int j) { return S->winU + (size_t)((S->whead + j) % S->wcap) * S->L; }
double* win_g(cp_ngmres_state* S, int j) { return S->winG + (size_t)((S->whead + j) % S->wcap) * S->L; }

int window_push(cp_handle* h, cp_ngmres_state* S) {
  if (S->wcount == S->wcap) {   // drop the oldest
    S->whead = (S->whead + 1) % S->wcap;
    S->wcount--;
  }
  const int j = S->wcount;
  CP_TRY(copy2(h, S->u, win_u(S, j), S->g, win_g(S, j), S->L, S->st));
  S->wcount++;
  return CP_OK;
}

int eval_current(cp_handle* h, cp_ngmres_state* S) {
  CP_TRY(objective_grad_impl(h, S->T, S->s, S->u, S->R, S->prec, S->scal, S->g, S->st,
                             S->opt.mttkrp_tree));
  S->n_fg++;
  CP_TRY(dot(h, S->g, S->g, S->L, S->scal + 1, S->st));
  double v[2];
  CP_TRY(readback(h, S->scal, 2, v, S->st));
  S->f = v[0];
  S->rho = std::sqrt(std::max(0.0, v[1])) / S->normT;
  if (!std::isfinite(S->f) || !std::isfinite(S->rho))
    return fail(h, CP_ENOTFINITE, "objective or gradient not finite");
  return CP_OK;
}

// Precision schedule: once rho is small enough (or would stop the run), move
// the bulk to the final precision, re-evaluate at the current iterate and
// restart the window.  Triggers: rho <= switch_rho; once rho <= 1e-2, a line
// search that found no Wolfe point in reduced precision (its objective noise
// is then comparable to the decrease it looks for); or rho <= stop_tol on a
// gradient that was not accumulated in float64 (so the stop is certified in
// float64).  *switched_now tells whether it switched.
int maybe_switch(cp_handle* h, cp_ngmres_state* S, bool* switched_now) {
  const cp_options& o = S->opt;
  *switched_now = false;
  if (S->switched || S->prec == o.final_precision) return CP_OK;
  const bool trig = (o.switch_rho > 0.0 && S->rho <= o.switch_rho) ||
                    (o.switch_rho > 0.0 && o.switch_on_stall && S->stalled && S->rho <= 1e-2) ||
                    (S->rho <= o.stop_tol && !is_f64_acc(S->prec) && is_f64_acc(o.final_precision));
  if (!trig) return CP_OK;
  S->prec = o.final_precision;
  S->switched = true;
  S->switch_iter = S->it;
  *switched_now = true;
  CP_TRY(eval_current(h, S));
  S->wcount = 0;
  S->whead = 0;
  S->cg_fresh = true;
  return window_push(h, S);
}

// One N-CG iteration (comparison method, Section 2.4): line search along d
// from u, then d = -g + gamma d with the Polak-Ribiere gamma clipped at 0.
// u is not normalised.  S->ubar holds the line search's base point.
int ncg_step(cp_handle* h, cp_ngmres_state* S, cp_iter_info* rec, int* rc_out) {
  const int64_t L = S->L;
  if (S->cg_fresh) {
    CP_TRY(cg_direction(h, S->g, 0.0, S->d, L, S->st));
    S->cg_fresh = false;
  }
  double slope;
  CP_TRY(dot(h, S->g, S->d, L, S->scal + 1, S->st));
  CP_TRY(readback(h, S->scal + 1, 1, &slope, S->st));
  if (!(slope < 0.0)) {   // not a descent direction: steepest descent
    rec->restart = 1;
    S->n_restarts++;
    CP_TRY(cg_direction(h, S->g, 0.0, S->d, L, S->st));
    CP_TRY(dot(h, S->g, S->d, L, S->scal + 1, S->st));
    CP_TRY(readback(h, S->scal + 1, 1, &slope, S->st));
  }
  CP_HIP(h, hipMemcpyAsync(S->ubar, S->u, sizeof(double) * L, hipMemcpyDeviceToDevice, S->st));
  double beta = 0.0, fnew = S->f;
  int nfev = 0, status = 0;
  const double* gacc = nullptr;
  CP_TRY(more_thuente(h, S, S->f, slope, &beta, &fnew, &gacc, &nfev, &status));
  rec->nfev = nfev;
  rec->ls_status = status;
  const bool restart_next = status != LS_CONVERGED;
  if (restart_next) {
    S->n_fallback++;
    *rc_out = CP_LS_FALLBACK;
    if (!is_f64_acc(S->prec)) S->stalled = true;
  }
  if (!gacc) {
    beta = 0.0;
    fnew = S->f;
  }
  rec->beta = beta;
  const double* gnew = gacc ? gacc : S->g;
  if (beta != 0.0) CP_TRY(axpy_to(h, S->ubar, beta, S->d, S->u, L, S->st));
  // g_new . (g_new - g), g . g and g_new . g_new in one readback
  double v[3];
  CP_TRY(sub_to(h, gnew, S->g, S->uhat, L, S->st));
  CP_TRY(dot(h, gnew, S->uhat, L, S->scal + 4, S->st));
  CP_TRY(dot(h, S->g, S->g, L, S->scal + 5, S->st));
  CP_TRY(dot(h, gnew, gnew, L, S->scal + 6, S->st));
  CP_TRY(readback(h, S->scal + 4, 3, v, S->st));
  const double gamma = restart_next ? 0.0 : std::max(0.0, v[0] / v[1]);
  CP_TRY(cg_direction(h, gnew, gamma, S->d, L, S->st));
  if (gnew != S->g)
    CP_HIP(h, hipMemcpyAsync(S->g, gnew, sizeof(double) * L, hipMemcpyDeviceToDevice, S->st));
  S->f = fnew;
  S->rho = std::sqrt(std::max(0.0, v[2])) / S->normT;
  if (!std::isfinite(S->f) || !std::isfinite(S->rho))
    return fail(h, CP_ENOTFINITE, "objective or gradient not finite");
  return CP_OK;
}

// Step I with steepest descent as the one-step process (CP_METHOD_NGMRES_SD):
// d = -g/||g||_2 from u_i, the Moré–Thuente search of Step III along it from
// S->ubar = u_i, u_bar = u_i + beta d (the last trial point itself when it
// was accepted), normalised with the accepted gradient carried over (Section
// 2.3 end).  A zero gradient leaves u_bar = u_i, g_bar = g_i.  On return
// S->ubar, S->gbar hold u_bar, g(u_bar) and *fbar is f(u_bar).
int sd_step1(cp_handle* h, cp_ngmres_state* S, double* fbar, int* nfev_out) {
  const int64_t L = S->L;
  const size_t bytes = sizeof(double) * L;
  *nfev_out = 0;
  *fbar = S->f;
  CP_TRY(dot(h, S->g, S->g, L, S->scal + 4, S->st));
  double gg;
  CP_TRY(readback(h, S->scal + 4, 1, &gg, S->st));
  const double gn = std::sqrt(std::max(0.0, gg));
  CP_HIP(h, hipMemcpyAsync(S->ubar, S->u, bytes, hipMemcpyDeviceToDevice, S->st));
  if (!(gn > 0.0)) {
    CP_HIP(h, hipMemcpyAsync(S->gbar, S->g, bytes, hipMemcpyDeviceToDevice, S->st));
    return CP_OK;
  }
  CP_TRY(neg_div_to(h, S->g, gn, S->d, L, S->st));
  double slope;
  CP_TRY(dot(h, S->g, S->d, L, S->scal + 4, S->st));
  CP_TRY(readback(h, S->scal + 4, 1, &slope, S->st));
  double beta = 0.0, fnew = S->f;
  int status = 0;
  const double* gacc = nullptr;
  CP_TRY(more_thuente(h, S, S->f, slope, &beta, &fnew, &gacc, nfev_out, &status));
  if (!gacc) {
    beta = 0.0;
    fnew = S->f;
  }
  const double* gnew = gacc ? gacc : S->g;
  if (beta != 0.0) {
    if (gnew == S->gt) CP_HIP(h, hipMemcpyAsync(S->ubar, S->ut, bytes, hipMemcpyDeviceToDevice, S->st));
    else CP_TRY(axpy_to(h, S->u, beta, S->d, S->ubar, L, S->st));
  }
  CP_HIP(h, hipMemcpyAsync(S->gbar, gnew, bytes, hipMemcpyDeviceToDevice, S->st));
  CP_TRY(normalize(h, S->s, S->ubar, S->R, S->gbar, S->st));
  *fbar = fnew;
  return CP_OK;
}

}  // namespace

// ============================== C ABI =====================================
// ---- workspace of the allocation-free MTTKRP ------------------------------
// One array per device, part of the library's code object: the loader places
// it when the library is loaded on a device, so cp_mttkrp_noalloc never
// allocates.  Its size bounds the workspace of one call (a 128^4, R = 32
// BF16x3 MTTKRP takes about 19 MB of it).  Host code never passes `scratch`
// itself to a kernel (on the host that name is not a device address); it
// uses the address hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[kMaxDevices];
void* g_scratch_ptr[kMaxDevices];
int g_scratch_err[kMaxDevices];

// Called by cp_create with h->device current: looks the array's device
// address up once per device and records it (or the failure) in the handle.
void scratch_setup(cp_handle* h) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  const int d = h->device;
  if (d < 0 || d >= kMaxDevices) {
    h->scratch = nullptr;
    h->scratch_err = (int)hipErrorInvalidDevice;
    return;
  }
  if (!g_scratch_done[d]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      (void)hipGetLastError();   // do not leave the error for the next call to report
      p = nullptr;
    }
    g_scratch_ptr[d] = p;
    g_scratch_err[d] = (int)e;
    g_scratch_done[d] = true;
  }
  h->scratch = g_scratch_ptr[d];
  h->scratch_err = g_scratch_err[d];
}

}  // namespace

extern "C" {

void cp_options_default(cp_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->method = CP_METHOD_NGMRES;
  o->window = 20;
  o->eps = 1e-12;
  o->ls_ftol = 1e-4;
  o->ls_gtol = 1e-2;
  o->ls_stp0 = 1.0;
  o->ls_maxfev = 20;
  o->ls_xtol = 1e-15;
  o->ls_stpmin = 1e-15;
  o->ls_stpmax = 1e15;
  o->max_iter = 1000;
  o->precision = CP_PREC_FP64;
  o->final_precision = CP_PREC_FP64;
  o->switch_rho = 0.0;
  o->normalize_accel = 1;
  o->trace = nullptr;
  o->trace_cap = 0;
  o->mttkrp_tree = 1;
  o->switch_on_stall = 1;
  o->stop_tol = 0.0;
  o->init = CP_INIT_GIVEN;
  o->seed = 0;
}

int cp_create(int device, size_t workspace_bytes, cp_handle** out) {
  if (!out) return CP_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CP_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return CP_EDEVICE;
  auto* h = new (std::nothrow) cp_handle();
  if (!h) return CP_ENOMEM;
  h->device = device;
  if (hipHostMalloc(reinterpret_cast<void**>(&h->pinned), 64 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&h->flags), 16 * sizeof(int)) != hipSuccess) {
    delete h;
    return CP_ENOMEM;
  }
  (void)hipMemset(h->flags, 0, 16 * sizeof(int));
  scratch_setup(h);
  if (workspace_bytes > 0 && ensure(h, h->part, workspace_bytes, nullptr) != CP_OK) {
    cp_destroy(h);
    return CP_ENOMEM;
  }
  *out = h;
  return CP_OK;
}

int cp_destroy(cp_handle* h) {
  if (!h) return CP_OK;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  DevBuf* bufs[] = {&h->part, &h->part2, &h->stage, &h->mbuf, &h->small, &h->red, &h->carry, &h->otab,
                    &h->ybuf};
  for (DevBuf* b : bufs)
    if (b->ptr) (void)hipFree(b->ptr);
  if (h->pinned) (void)hipHostFree(h->pinned);
  if (h->flags) (void)hipFree(h->flags);
  for (auto& v : h->ev_pending)
    for (auto& pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  delete h;
  return CP_OK;
}

int cp_profile(cp_handle* h, int32_t enable) {
  if (!h) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  CP_HIP(h, hipDeviceSynchronize());
  // pending events of the previous session are dropped unread
  for (auto& v : h->ev_pending) {
    for (auto& pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    v.clear();
  }
  for (int k = 0; k < cp_handle::kKernelIds; ++k) {
    h->prof_launches[k] = 0;
    h->prof_ms[k] = 0.0;
  }
  h->prof = enable != 0;
  return CP_OK;
}

int cp_stream_read(cp_handle* h, const void* buf, size_t bytes, hipStream_t stream) {
  if (!h) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  return stream_read(h, buf, bytes, stream);
}

int cp_sparse_gather_read(cp_handle* h, const cp_tensor* T, const double* u, int32_t R,
                          int32_t mode, hipStream_t st) {
  if (!h) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  Shape s;
  CP_TRY(check_tensor(h, T, &s));
  if (!T->sparse) return fail(h, CP_EINVAL, "cp_sparse_gather_read needs a sparse tensor");
  if (R < 1 || R > 64) return fail(h, CP_EINVAL, "rank %d outside 1..64", R);
  if (mode < 0 || mode >= s.N) return fail(h, CP_EINVAL, "mode %d outside 0..%d", mode, s.N - 1);
  if (!u) return fail(h, CP_EINVAL, "null factor pointer");
  return sparse_gather_ref(h, T, s, u, R, mode, st);
}

int cp_profile_select(cp_handle* h, uint32_t kernel_mask) {
  if (!h || (kernel_mask & ~0xFFu) != 0) return CP_EINVAL;
  h->prof_mask = kernel_mask;
  return CP_OK;
}

int cp_profile_read(cp_handle* h, int32_t kernel, int64_t* launches, double* total_ms) {
  if (!h || kernel < 0 || kernel >= cp_handle::kKernelIds || !launches || !total_ms)
    return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  auto& v = h->ev_pending[kernel];
  for (auto& pr : v) {
    float ms = 0.f;
    CP_HIP(h, hipEventSynchronize(pr.second));
    CP_HIP(h, hipEventElapsedTime(&ms, pr.first, pr.second));
    h->prof_ms[kernel] += ms;
    h->prof_launches[kernel]++;
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  v.clear();
  *launches = h->prof_launches[kernel];
  *total_ms = h->prof_ms[kernel];
  return CP_OK;
}

const char* cp_last_error(const cp_handle* h) { return h ? h->err.c_str() : "null handle"; }

int cp_tensor_prepare(cp_handle* h, cp_tensor* T, hipStream_t st) {
  if (!h) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  Shape s;
  CP_TRY(check_tensor(h, T, &s));
  if (T->prepared) CP_TRY(cp_tensor_release(h, T));
  const int64_t n = T->sparse ? T->nnz : s.total();
  CP_TRY(ensure(h, h->small, 4096, st));
  double* d = static_cast<double*>(h->small.ptr);
  if (n > 0) {
    CP_TRY(sumsq_tensor(h, T->values, T->dtype, n, d, st));
    double v;
    CP_TRY(readback(h, d, 1, &v, st));
    T->norm_sq = v;
  } else {
    T->norm_sq = 0.0;
  }
  if (T->sparse) CP_TRY(sparse_prepare(h, T, s, st));
  return CP_OK;
}

int cp_tensor_release(cp_handle* h, cp_tensor* T) {
  if (!h || !T) return CP_EINVAL;
  if (T->sparse) return sparse_release(h, T);
  T->prepared = nullptr;
  return CP_OK;
}

int cp_mttkrp(cp_handle* h, const cp_tensor* T, const double* u, int32_t R, int32_t mode,
              int32_t p, double* M_out, hipStream_t st) {
  if (!h) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  Shape s;
  CP_TRY(check_mttkrp_args(h, T, u, R, mode, p, M_out, &s));
  return mttkrp_any(h, T, s, u, R, mode, p, M_out, st);
}

int cp_mttkrp_noalloc(cp_handle* h, const cp_tensor* T, const double* u, int32_t R, int32_t mode,
                      int32_t p, double* M_out, hipStream_t st) {
  if (!h) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  if (!h->scratch)
    return fail(h, CP_EDEVICE, "static scratch of device %d unavailable: %s", h->device,
                hipGetErrorString((hipError_t)h->scratch_err));
  Shape s;
  CP_TRY(check_mttkrp_args(h, T, u, R, mode, p, M_out, &s));
  // The same launches as cp_mttkrp, with every workspace slice carved from
  // the static scratch (ensure() in arena mode) instead of the handle's
  // grown buffers, which are set aside and restored untouched.  Each slice
  // is written before it is read, so nothing needs clearing; timing (which
  // creates events) is off for the call.
  DevBuf* bufs[] = {&h->part, &h->part2, &h->stage, &h->mbuf, &h->small, &h->red,
                    &h->carry, &h->otab, &h->ybuf};
  constexpr int nb = sizeof(bufs) / sizeof(bufs[0]);
  DevBuf saved[nb];
  for (int i = 0; i < nb; ++i) {
    saved[i] = *bufs[i];
    *bufs[i] = DevBuf{};
  }
  const bool prof = h->prof;
  const uint64_t gen = h->gen;
  h->prof = false;
  h->arena = static_cast<char*>(h->scratch);
  h->arena_cap = kScratchBytes;
  h->arena_used = 0;
  const int rc = mttkrp_any(h, T, s, u, R, mode, p, M_out, st);
  h->arena = nullptr;
  h->arena_cap = h->arena_used = 0;
  h->prof = prof;
  h->gen = gen;
  for (int i = 0; i < nb; ++i) *bufs[i] = saved[i];
  return rc;
}

int cp_gram(cp_handle* h, int32_t order, const int64_t* dims, const double* u, int32_t R,
            double* S_out, double* gamma_bar_out, double* gamma_out, hipStream_t st) {
  if (!h) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  if (!dims || !u || !S_out) return fail(h, CP_EINVAL, "null argument");
  Shape s;
  CP_TRY(make_shape(h, order, dims, &s));
  CP_TRY(check_rank(h, R));
  return gram_all(h, s, u, R, S_out, gamma_bar_out, gamma_out, st);
}

int cp_normalize(cp_handle* h, int32_t order, const int64_t* dims, double* u, int32_t R, double* g,
                 hipStream_t st) {
  if (!h) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  if (!dims || !u) return fail(h, CP_EINVAL, "null argument");
  Shape s;
  CP_TRY(make_shape(h, order, dims, &s));
  CP_TRY(check_rank(h, R));
  return normalize(h, s, u, R, g, st);
}

int cp_als_sweep(cp_handle* h, const cp_tensor* T, double* u, int32_t R, int32_t p,
                 int32_t normalize_after, hipStream_t st) {
  if (!h) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  Shape s;
  CP_TRY(check_tensor(h, T, &s));
  CP_TRY(check_rank(h, R));
  CP_TRY(check_prec(h, T, p));
  if (!u) return fail(h, CP_EINVAL, "null iterate");
  return als_sweep_impl(h, T, s, u, R, p, normalize_after, st);
}

int cp_mode_solve(cp_handle* h, const double* M, const double* Gbar, int64_t I, int32_t R,
                  double* A_out, int32_t* kind_out, hipStream_t st) {
  if (!h) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  CP_TRY(check_rank(h, R));
  if (I < 1 || !M || !Gbar || !A_out) return fail(h, CP_EINVAL, "bad mode-solve arguments");
  CP_HIP(h, hipMemsetAsync(h->flags, 0, sizeof(int), st));
  CP_TRY(mode_solve(h, M, Gbar, I, R, A_out, st));
  if (kind_out) {
    int v = 0;
    CP_HIP(h, hipMemcpyAsync(&h->pinned[0], h->flags, sizeof(int), hipMemcpyDeviceToHost, st));
    CP_HIP(h, hipStreamSynchronize(st));
    std::memcpy(&v, &h->pinned[0], sizeof(int));
    *kind_out = v & 3;
  }
  return CP_OK;
}

int cp_objective_grad(cp_handle* h, const cp_tensor* T, const double* u, int32_t R, int32_t p,
                      double* f_out, double* g_out, hipStream_t st) {
  if (!h) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  Shape s;
  CP_TRY(check_tensor(h, T, &s));
  CP_TRY(check_rank(h, R));
  CP_TRY(check_prec(h, T, p));
  if (!u || !f_out) return fail(h, CP_EINVAL, "null iterate or objective pointer");
  if (T->sparse && !T->prepared) return fail(h, CP_EINVAL, "sparse tensor is not prepared");
  return objective_grad_impl(h, T, s, u, R, p, f_out, g_out, st);
}

int ngmres_accelerate(cp_handle* h, int64_t L, int32_t m, const double* U, const double* G,
                      const double* u_bar, const double* g_bar, double eps, double* u_hat_out,
                      double* gTd_out, double* alpha_out, hipStream_t st) {
  if (!h) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  if (L < 1 || m < 1 || m > 64) return fail(h, CP_EINVAL, "need L >= 1 and 1 <= m <= 64");
  if (!U || !G || !u_bar || !g_bar || !u_hat_out) return fail(h, CP_EINVAL, "null argument");
  if (!(eps >= 0.0)) return fail(h, CP_EINVAL, "eps must be >= 0");
  CP_TRY(ensure(h, h->small, 64 * 1024, st));
  double* alpha = alpha_out ? alpha_out : static_cast<double*>(h->small.ptr) + 4096;
  StepPar* par = reinterpret_cast<StepPar*>(static_cast<double*>(h->small.ptr) + 4096 + 64);
  CP_TRY(set_steppar(h, par, 0.0, m, 0, st));
  CP_TRY(step2(h, L, U, G, m, par, u_bar, g_bar, eps, u_hat_out, alpha, st));
  if (gTd_out) {   // g_bar^T (u_hat - u_bar), the difference held in the mbuf slice
    CP_TRY(ensure(h, h->mbuf, sizeof(double) * (size_t)L, st));
    double* dv = static_cast<double*>(h->mbuf.ptr);
    CP_TRY(sub_to(h, u_hat_out, u_bar, dv, L, st));
    CP_TRY(dot(h, g_bar, dv, L, gTd_out, st));
  }
  return CP_OK;
}

int cp_init_uniform(cp_handle* h, int64_t L, uint64_t seed, double* u_out, hipStream_t st) {
  if (!h) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  if (L < 0 || (L > 0 && !u_out)) return fail(h, CP_EINVAL, "need L >= 0 and an output");
  return init_uniform(h, L, seed, u_out, st);
}

int cp_ngmres_create(cp_handle* h, const cp_tensor* T, int32_t R, const cp_options* opt,
                     const double* u0, hipStream_t st, cp_ngmres_state** out) {
  if (!h || !out) return CP_EINVAL;
  *out = nullptr;
  CP_HIP(h, hipSetDevice(h->device));
  Shape s;
  CP_TRY(check_tensor(h, T, &s));
  CP_TRY(check_rank(h, R));
  if (!u0 && !(opt && opt->init == CP_INIT_SEEDED))
    return fail(h, CP_EINVAL, "null initial guess");
  if (T->sparse && !T->prepared) return fail(h, CP_EINVAL, "sparse tensor is not prepared");
  if (!(T->norm_sq > 0.0)) return fail(h, CP_EINVAL, "tensor not prepared or zero (||T|| = 0)");
  cp_options o;
  if (opt) o = *opt;
  else cp_options_default(&o);
  if (o.window < 1 || o.window > 64) return fail(h, CP_EINVAL, "window must be in 1..64");
  if (o.method != CP_METHOD_NGMRES && o.method != CP_METHOD_ALS && o.method != CP_METHOD_NCG &&
      o.method != CP_METHOD_NGMRES_SD)
    return fail(h, CP_EINVAL, "unknown method %d", o.method);
  if (o.ls_maxfev < 1 || !(o.ls_stp0 > 0.0)) return fail(h, CP_EINVAL, "bad line-search options");
  if (o.init != CP_INIT_GIVEN && o.init != CP_INIT_SEEDED)
    return fail(h, CP_EINVAL, "unknown init %d", o.init);
  if (o.mttkrp_tree < 0 || o.mttkrp_tree > 2)
    return fail(h, CP_EINVAL, "mttkrp_tree must be 0, 1 or 2");
  CP_TRY(check_prec(h, T, o.precision));
  CP_TRY(check_prec(h, T, o.final_precision));
  auto* S = new (std::nothrow) cp_ngmres_state();
  if (!S) return fail(h, CP_ENOMEM, "host allocation failed");
  S->T = T;
  S->s = s;
  S->R = R;
  S->L = s.sum_dims() * R;
  S->opt = o;
  S->st = st;
  S->prec = o.precision;
  S->normT = std::sqrt(T->norm_sq);
  S->wcap = uses_window(o.method) ? o.window : 1;
  const size_t nvec = 9 + 2 * (size_t)S->wcap;
  if (hipMalloc(&S->mem, sizeof(double) * (nvec * S->L + 80)) != hipSuccess) {
    delete S;
    return fail(h, CP_ENOMEM, "state allocation failed");
  }
  double* p = S->mem;
  S->u = p; p += S->L;
  S->g = p; p += S->L;
  S->ubar = p; p += S->L;
  S->gbar = p; p += S->L;
  S->uhat = p; p += S->L;
  S->d = p; p += S->L;
  S->ut = p; p += S->L;
  S->gt = p; p += S->L;
  S->gbest = p; p += S->L;
  S->winU = p; p += (size_t)S->wcap * S->L;
  S->winG = p; p += (size_t)S->wcap * S->L;
  S->scal = p;
  S->dpar = reinterpret_cast<StepPar*>(S->scal + 72);
  if (hipHostMalloc(reinterpret_cast<void**>(&S->hpar), sizeof(StepPar)) != hipSuccess) {
    S->hpar = nullptr;
    (void)hipFree(S->mem);
    delete S;
    return fail(h, CP_ENOMEM, "pinned host allocation failed");
  }
  *S->hpar = StepPar{0.0, 0, 0};
  int rc = CP_OK;
  if (o.init == CP_INIT_SEEDED)
    rc = init_uniform(h, S->L, o.seed, S->u, st);
  else if (hipMemcpyAsync(S->u, u0, sizeof(double) * S->L, hipMemcpyDeviceToDevice, st) != hipSuccess)
    rc = fail(h, CP_EDEVICE, "copy of the initial guess failed");
  if (rc == CP_OK) rc = normalize(h, s, S->u, R, nullptr, st);
  if (rc == CP_OK) rc = eval_current(h, S);
  if (rc == CP_OK && (o.method == CP_METHOD_NGMRES || o.method == CP_METHOD_ALS) &&
      o.mttkrp_tree == 1) {
    int split = 0;
    double* XL = nullptr;
    if (tree_left_buffer(h, T, s, R, S->prec, &split, &XL)) {   // evaluated at the normalised u0
      S->xl_ok = true;
      S->xl_token = h->ywrites;
      S->xl_ptr = h->ybuf.ptr;
    }
  }
  if (rc == CP_OK) rc = window_push(h, S);
  if (rc < 0) {
    cp_ngmres_destroy(h, S);
    return rc;
  }
  *out = S;
  return CP_OK;
}

int cp_ngmres_destroy(cp_handle* h, cp_ngmres_state* S) {
  if (!S) return CP_OK;
  if (h) (void)hipSetDevice(h->device);
  if (S->st) (void)hipStreamSynchronize(S->st);
  for (auto& c : S->cap) drop_captured(c);
  if (S->hpar) (void)hipHostFree(S->hpar);
  if (S->mem) (void)hipFree(S->mem);
  delete S;
  return CP_OK;
}

int cp_ngmres_get(cp_handle* h, cp_ngmres_state* S, double* u_out, double* g_out, double* f_out,
                  double* rho_out) {
  if (!h || !S) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  if (u_out)
    CP_HIP(h, hipMemcpyAsync(u_out, S->u, sizeof(double) * S->L, hipMemcpyDeviceToDevice, S->st));
  if (g_out)
    CP_HIP(h, hipMemcpyAsync(g_out, S->g, sizeof(double) * S->L, hipMemcpyDeviceToDevice, S->st));
  if (f_out) *f_out = S->f;
  if (rho_out) *rho_out = S->rho;
  return CP_OK;
}

int cp_ngmres_save(cp_handle* h, cp_ngmres_state* S, double* U_out, double* G_out, double* u_out,
                   double* g_out, double* d_out, cp_ngmres_meta* meta) {
  if (!h || !S) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  const size_t bytes = sizeof(double) * S->L;
  const int m = uses_window(S->opt.method) ? S->wcount : 0;
  for (int j = 0; j < m; ++j) {
    if (U_out) CP_HIP(h, hipMemcpyAsync(U_out + (size_t)j * S->L, win_u(S, j), bytes, hipMemcpyDeviceToDevice, S->st));
    if (G_out) CP_HIP(h, hipMemcpyAsync(G_out + (size_t)j * S->L, win_g(S, j), bytes, hipMemcpyDeviceToDevice, S->st));
  }
  if (u_out) CP_HIP(h, hipMemcpyAsync(u_out, S->u, bytes, hipMemcpyDeviceToDevice, S->st));
  if (g_out) CP_HIP(h, hipMemcpyAsync(g_out, S->g, bytes, hipMemcpyDeviceToDevice, S->st));
  if (d_out) CP_HIP(h, hipMemcpyAsync(d_out, S->d, bytes, hipMemcpyDeviceToDevice, S->st));
  if (meta) {
    meta->it = S->it;
    meta->m = m;
    meta->precision = S->prec;
    meta->switched = S->switched;
    meta->stalled = S->stalled;
    meta->cg_fresh = S->cg_fresh;
    meta->f = S->f;
    meta->rho = S->rho;
    meta->n_fg = S->n_fg;
    meta->n_restarts = S->n_restarts;
    meta->n_ls_fallback = S->n_fallback;
    meta->switch_iter = S->switch_iter;
  }
  return CP_OK;
}

int cp_ngmres_load(cp_handle* h, cp_ngmres_state* S, const double* U, const double* G,
                   const double* u, const double* g, const double* d, const cp_ngmres_meta* meta) {
  if (!h || !S || !meta || !u || !g) return fail(h, CP_EINVAL, "null state, iterate or meta");
  CP_HIP(h, hipSetDevice(h->device));
  const bool ngm = uses_window(S->opt.method);
  if (ngm && (meta->m < 1 || meta->m > S->wcap || !U || !G))
    return fail(h, CP_EINVAL, "window of %d entries (capacity %d) needs U and G", meta->m, S->wcap);
  if (S->opt.method == CP_METHOD_NCG && !meta->cg_fresh && !d)
    return fail(h, CP_EINVAL, "an N-CG state needs its direction");
  if (meta->precision < 0 || meta->precision > 3) return fail(h, CP_EINVAL, "bad precision");
  CP_TRY(check_prec(h, S->T, meta->precision));
  const size_t bytes = sizeof(double) * S->L;
  S->whead = 0;
  S->wcount = ngm ? meta->m : 0;
  for (int j = 0; j < S->wcount; ++j)
    CP_TRY(copy2(h, U + (size_t)j * S->L, win_u(S, j), G + (size_t)j * S->L, win_g(S, j), S->L, S->st));
  CP_TRY(copy2(h, u, S->u, g, S->g, S->L, S->st));
  if (d) CP_HIP(h, hipMemcpyAsync(S->d, d, bytes, hipMemcpyDeviceToDevice, S->st));
  S->it = meta->it;
  S->prec = meta->precision;
  S->switched = meta->switched != 0;
  S->stalled = meta->stalled != 0;
  S->cg_fresh = meta->cg_fresh != 0;
  S->f = meta->f;
  S->n_fg = meta->n_fg;
  S->n_restarts = meta->n_restarts;
  S->n_fallback = meta->n_ls_fallback;
  S->switch_iter = meta->switch_iter;
  S->have_last = false;
  S->xl_ok = false;
  CP_TRY(dot(h, S->g, S->g, S->L, S->scal + 3, S->st));
  double gg;
  CP_TRY(readback(h, S->scal + 3, 1, &gg, S->st));
  S->rho = std::sqrt(std::max(0.0, gg)) / S->normT;
  return CP_OK;
}

int cp_ngmres_last_step(cp_handle* h, cp_ngmres_state* S, double* u_bar, double* g_bar,
                        double* u_hat, double* d, double* f_bar, double* slope) {
  if (!h || !S) return CP_EINVAL;
  if (!S->have_last || !uses_window(S->opt.method))
    return fail(h, CP_EINVAL, "no N-GMRES iteration taken yet");
  CP_HIP(h, hipSetDevice(h->device));
  const size_t bytes = sizeof(double) * S->L;
  if (u_bar) CP_HIP(h, hipMemcpyAsync(u_bar, S->ubar, bytes, hipMemcpyDeviceToDevice, S->st));
  if (g_bar) CP_HIP(h, hipMemcpyAsync(g_bar, S->gbar, bytes, hipMemcpyDeviceToDevice, S->st));
  if (u_hat) CP_HIP(h, hipMemcpyAsync(u_hat, S->uhat, bytes, hipMemcpyDeviceToDevice, S->st));
  if (d) CP_HIP(h, hipMemcpyAsync(d, S->d, bytes, hipMemcpyDeviceToDevice, S->st));
  if (f_bar) *f_bar = S->last_fbar;
  if (slope) *slope = S->last_slope;
  return CP_OK;
}

int ngmres_step(cp_handle* h, cp_ngmres_state* S, cp_iter_info* info) {
  if (!h || !S) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  bool sw = false;
  CP_TRY(maybe_switch(h, S, &sw));
  cp_iter_info rec{};
  rec.it = S->it;
  rec.f = S->f;
  rec.rho = S->rho;
  rec.beta = NAN;
  rec.ls_status = -1;
  rec.m = uses_window(S->opt.method) ? S->wcount : 0;
  rec.precision = S->prec;
  const int64_t passes0 = h->t_passes;
  // X_L at u kept by the previous step, unless anything has written ybuf since
  const bool xl_in = S->xl_ok && S->xl_token == h->ywrites && S->xl_ptr == h->ybuf.ptr;
  S->xl_ok = false;
  int rc = CP_OK;
  if (S->opt.method == CP_METHOD_ALS) {
    // the sweep starts from the point of the last evaluation (of the
    // normalised iterate): its left partial is that evaluation's
    CP_TRY(als_sweep_impl(h, S->T, S->s, S->u, S->R, S->prec, 1, S->st, S->opt.mttkrp_tree != 0,
                          xl_in));
    CP_TRY(eval_current(h, S));
    int split = 0;
    double* XL = nullptr;
    if (S->opt.mttkrp_tree == 1 && tree_left_buffer(h, S->T, S->s, S->R, S->prec, &split, &XL)) {
      S->xl_ok = true;
      S->xl_token = h->ywrites;
      S->xl_ptr = h->ybuf.ptr;
    }
  } else if (S->opt.method == CP_METHOD_NCG) {
    CP_TRY(ncg_step(h, S, &rec, &rc));
  } else {
    // Steps I and II: u_bar = M(u_i); f, g at u_bar; u_hat over the window
    S->hpar->m = S->wcount;
    S->hpar->whead = S->whead;
    double fbar, slope;
    if (S->opt.method == CP_METHOD_NGMRES_SD) {
      CP_TRY(sd_step1(h, S, &fbar, &rec.nfev_pre));
      CP_HIP(h, hipMemcpyAsync(S->dpar, S->hpar, sizeof(StepPar), hipMemcpyHostToDevice, S->st));
      CP_TRY(enqueue_step2(h, S));
      CP_TRY(readback(h, S->scal + 1, 1, &slope, S->st));
    } else {
      CP_TRY(run_phase(h, S, xl_in ? PHASE_STEP12_XL : PHASE_STEP12));
      S->n_fg++;
      double fs[2];   // f(u_bar) and the slope g(u_bar)^T d in one readback
      CP_TRY(readback(h, S->scal, 2, fs, S->st));
      fbar = fs[0];
      slope = fs[1];
    }
    S->have_last = true;
    S->last_fbar = fbar;
    S->last_slope = slope;
    const double* gnew = S->gbar;
    double fnew = fbar;
    double beta = 0.0;
    const bool restart = !(slope < 0.0);
    if (restart) {
      // restart: u_{i+1} = u_bar, window back to one iterate
      rec.restart = 1;
      S->n_restarts++;
      S->wcount = 0;
      S->whead = 0;
    } else {
      int nfev = 0, status = 0;
      const double* gacc = nullptr;
      CP_TRY(more_thuente(h, S, fbar, slope, &beta, &fnew, &gacc, &nfev, &status));
      rec.nfev = nfev;
      rec.ls_status = status;
      rec.beta = beta;
      if (status != LS_CONVERGED) {
        S->n_fallback++;
        rc = CP_LS_FALLBACK;
        if (!is_f64_acc(S->prec)) S->stalled = true;
      }
      if (gacc) gnew = gacc;
      else { beta = 0.0; fnew = fbar; gnew = S->gbar; }
    }
    // u_{i+1} = u_bar + beta d: the accepted trial point itself when its
    // gradient is the last trial's (the same fma on the same beta), else formed
    if (beta == 0.0) CP_TRY(copy2(h, S->ubar, S->u, gnew, S->g, S->L, S->st));
    else if (gnew == S->gt) CP_TRY(copy2(h, S->ut, S->u, gnew, S->g, S->L, S->st));
    else {
      CP_TRY(axpy_to(h, S->ubar, beta, S->d, S->u, S->L, S->st));
      CP_HIP(h, hipMemcpyAsync(S->g, gnew, sizeof(double) * S->L, hipMemcpyDeviceToDevice, S->st));
    }
    // The last evaluation was at u_{i+1} on a restart (u_bar) and when the
    // accepted point is the last trial: then the next sweep's left partial
    // is that evaluation's, carried through the normalisation
    // (tree_rescale_left) instead of a pass over T.
    int split = 0;
    double* XL = nullptr;
    const bool keep = S->opt.method == CP_METHOD_NGMRES && S->opt.mttkrp_tree == 1 &&
                      (restart || (beta != 0.0 && gnew == S->gt)) &&
                      tree_left_buffer(h, S->T, S->s, S->R, S->prec, &split, &XL);
    const double* nsc = nullptr;
    const int* nperm = nullptr;
    CP_TRY(normalize(h, S->s, S->u, S->R, S->g, S->st, keep ? &nsc : nullptr, keep ? &nperm : nullptr));
    if (keep) {
      const int rr = tree_rescale_left(h, S->s, split, S->R, XL, nsc, nperm, S->st);
      if (rr < 0) return rr;
      if (rr == CP_OK) {
        S->xl_ok = true;
        S->xl_token = h->ywrites;
        S->xl_ptr = h->ybuf.ptr;
      }
    }
    S->f = fnew;
    CP_TRY(dot(h, S->g, S->g, S->L, S->scal + 3, S->st));
    CP_TRY(window_push(h, S));   // queued before the readback below waits
    double gg;
    CP_TRY(readback(h, S->scal + 3, 1, &gg, S->st));
    S->rho = std::sqrt(std::max(0.0, gg)) / S->normT;
    if (!std::isfinite(S->f) || !std::isfinite(S->rho))
      return fail(h, CP_ENOTFINITE, "objective or gradient not finite");
  }
  S->it++;
  rec.t_passes = (int32_t)(h->t_passes - passes0);
  if (info) *info = rec;
  return rc;
}

int cp_decompose(cp_handle* h, const cp_tensor* T, int32_t R, double tol, const cp_options* opt,
                 double* u_inout, cp_report* rep, hipStream_t st) {
  if (!h) return CP_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  cp_options o;
  if (opt) o = *opt;
  else cp_options_default(&o);
  if (!(tol >= 0.0)) return fail(h, CP_EINVAL, "tol must be >= 0");
  o.stop_tol = tol;
  if (!u_inout) o.init = CP_INIT_SEEDED;   // the seeded guess; the report describes the result
  cp_ngmres_state* S = nullptr;
  // The null stream cannot be captured: run on a private stream that first
  // waits for the work the caller queued on it.
  hipStream_t own = nullptr;
  if (!st) {
    hipEvent_t ev = nullptr;
    CP_HIP(h, hipSetDevice(h->device));
    if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) == hipSuccess &&
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess &&
        hipEventRecord(ev, st) == hipSuccess && hipStreamWaitEvent(own, ev, 0) == hipSuccess) {
      st = own;
    } else if (own) {
      (void)hipStreamDestroy(own);
      own = nullptr;
    }
    if (ev) (void)hipEventDestroy(ev);
    (void)hipGetLastError();
  }
  struct OwnStream {
    hipStream_t s;
    ~OwnStream() {
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
    }
  } own_guard{own};
  CP_TRY(cp_ngmres_create(h, T, R, &o, u_inout, st, &S));
  int rc = CP_OK;
  int ntr = 0;
  for (;;) {
    // the precision schedule before the stopping test (ngmres_step applies
    // it too; here it also covers the last iterate)
    bool sw = false;
    rc = maybe_switch(h, S, &sw);
    if (rc < 0) break;
    if (S->rho <= tol || S->it >= o.max_iter) {
      if (o.trace && ntr < o.trace_cap) {
        cp_iter_info r{};
        r.it = S->it; r.f = S->f; r.rho = S->rho; r.beta = NAN; r.ls_status = -1;
        r.m = uses_window(o.method) ? S->wcount : 0;
        r.precision = S->prec;
        o.trace[ntr++] = r;
      }
      break;
    }
    cp_iter_info info{};
    rc = ngmres_step(h, S, &info);
    if (rc < 0) break;
    if (o.trace && ntr < o.trace_cap) o.trace[ntr++] = info;
  }
  if (rc >= 0) {
    if ((u_inout && hipMemcpyAsync(u_inout, S->u, sizeof(double) * S->L, hipMemcpyDeviceToDevice,
                                   st) != hipSuccess) ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = fail(h, CP_EDEVICE, "copy of the result failed");
  }
  if (rep) {
    rep->iters = S->it;
    rep->converged = S->rho <= tol;
    rep->f = S->f;
    rep->rho = S->rho;
    rep->n_fg = S->n_fg;
    rep->n_restarts = S->n_restarts;
    rep->n_ls_fallback = S->n_fallback;
    rep->switch_iter = S->switch_iter;
    rep->n_trace = ntr;
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  const bool conv = S->rho <= tol;
  cp_ngmres_destroy(h, S);
  if (rc < 0) return rc;
  return conv ? CP_OK : CP_MAXITER;
}

}  // extern "C"
