/*
 * cpng.h -- C ABI of the MI355X (gfx950) library for canonical rank-R tensor
 * decomposition by ALS accelerated with nonlinear GMRES (N-GMRES).
 *
 * The operations follow the paper "A Nonlinear GMRES Optimization Algorithm
 * for Canonical Tensor Decomposition" (H. De Sterck):
 *   - the problem: minimise f = 1/2 ||T - [[A^(1),...,A^(N)]]||_F^2 over the
 *     factor matrices (Section 1, Optimization Problem I);
 *   - the gradient G^(n) = -T_(n) Phibar^(n) + A^(n) Gammabar^(n), its MTTKRP
 *     term T_(n) Phibar^(n) and the Hadamard products of Grams Gammabar^(n)
 *     (Section 2.3);
 *   - ALS as the one-step process (Section 2.3, nonlinear block Gauss-Seidel)
 *     with the normalisation and reordering of the rank-one terms;
 *   - the three-step N-GMRES iteration (Section 2.1, Steps I-III and the
 *     algorithm box), with the window, restart and delta regularisation of the
 *     Section 2.1 remarks and the Section 2.4 parameters.
 *
 * Conventions
 *   - Every function returns an int status: CP_OK (0), a negative error code,
 *     or a positive informational code.  Nothing throws across the ABI.  The
 *     message of the last failure on a handle is cp_last_error(h).
 *   - Array arguments are DEVICE pointers owned by the caller unless stated
 *     otherwise.  Work is enqueued on the given HIP stream (stream-ordered);
 *     functions that must read a scalar back (line search, convergence test)
 *     synchronise that stream and say so.
 *   - The library owns only its handle workspace (grown on demand with
 *     hipMalloc from host calls; never inside a kernel) and the prepared
 *     structures that cp_tensor_prepare attaches to a tensor.
 *   - One handle per host thread / stream.  For fixed inputs, device and
 *     precision mode, results are bitwise reproducible: no kernel uses
 *     floating-point atomics and every reduction has a fixed order.
 *
 * Layouts
 *   - Dense tensor: C order over (I_1..I_N), last index fastest.
 *   - Sparse tensor: coordinate format, structure of arrays: coords is an
 *     order x nnz int32 array (row n holds the zero-based mode-n index of every
 *     nonzero), values has nnz entries; no repeated coordinates.
 *   - Factor A^(n): I_n x R, row-major, float64.  The iterate u is the
 *     concatenation of A^(1)..A^(N) (length L = R * sum_n I_n); a gradient g
 *     has the same layout.
 */
#ifndef CPNG_H
#define CPNG_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CP_MAX_ORDER 8

/* ---- status codes ---------------------------------------------------- */
#define CP_OK            0
#define CP_EINVAL       -1   /* bad argument (shape, rank, mode, null pointer, dtype/precision mix) */
#define CP_ENOMEM       -2   /* device or pinned allocation failed */
#define CP_EDEVICE      -3   /* a HIP runtime call or kernel launch failed */
#define CP_ESINGULAR    -4   /* a Gammabar^(n) could not be factorised even after the shift */
#define CP_EDUPLICATE   -5   /* sparse tensor has repeated coordinates */
#define CP_ENOTFINITE   -6   /* objective or gradient became NaN/Inf */
#define CP_MAXITER       1   /* cp_decompose: max_iter reached before the tolerance */
#define CP_LS_FALLBACK   2   /* ngmres_step: line search ended without a strong-Wolfe point */

typedef enum { CP_F32 = 0, CP_F64 = 1 } cp_dtype;

/* Arithmetic of the MTTKRP bulk (every small solve stays float64):
 *   CP_PREC_FP64            float64 products and sums (tensor float64, or float32 widened)
 *   CP_PREC_FP32            float32 tensor and factor copies, float32 products and
 *                           per-workgroup sums, float64 across workgroups
 *   CP_PREC_BF16X3          dense only: tensor and Khatri-Rao rows split x = hi + lo
 *                           (both bfloat16); hi*hi + hi*lo + lo*hi on MFMA with
 *                           float32 accumulation; float64 across workgroups.  MTTKRPs
 *                           whose inner mode (the last; the next-to-last for the last
 *                           mode) has a length that is not a multiple of 8 or above
 *                           512 run the CP_PREC_FP32 kernels instead (faster there,
 *                           and at least as accurate)
 *   CP_PREC_FP32IN_FP64ACC  float32 tensor widened to float64, float64 factors,
 *                           products and sums (the same kernels as CP_PREC_FP64) */
typedef enum {
  CP_PREC_FP64 = 0, CP_PREC_FP32 = 1, CP_PREC_BF16X3 = 2, CP_PREC_FP32IN_FP64ACC = 3
} cp_precision;

typedef struct cp_handle cp_handle;
typedef struct cp_ngmres_state cp_ngmres_state;

/* Data tensor descriptor.  The caller fills order..coords; prepared and
 * norm_sq are written by cp_tensor_prepare. */
typedef struct cp_tensor {
  int32_t order;                  /* N, 1 <= N <= CP_MAX_ORDER (2 or more for decompositions) */
  int64_t dims[CP_MAX_ORDER];     /* I_1..I_N, each >= 1 */
  int32_t sparse;                 /* 0 = dense, 1 = coordinate format */
  int32_t dtype;                  /* cp_dtype of values */
  const void* values;             /* device; dense: prod(dims) values; sparse: nnz values */
  int64_t nnz;                    /* sparse only (0 allowed) */
  const int32_t* coords;          /* device, sparse only: order x nnz */
  void* prepared;                 /* library-owned, from cp_tensor_prepare */
  double norm_sq;                 /* ||T||_F^2, from cp_tensor_prepare */
} cp_tensor;

/* Options of cp_decompose / cp_ngmres_create.  cp_options_default fills the
 * paper's parameters (Section 2.4): window w = 20, eps = 1e-12, line search
 * ftol = 1e-4, gtol = 1e-2, first step 1, at most 20 evaluations. */
typedef struct cp_iter_info {
  int32_t it;          /* iteration index i (state before the iteration) */
  double f;            /* objective at u_i */
  double rho;          /* ||g(u_i)||_2 / ||T||_F */
  double beta;         /* accepted line-search step (NaN if no line search ran) */
  int32_t restart;     /* 1 if this iteration restarted the window */
  int32_t nfev;        /* objective/gradient evaluations of the line search */
  int32_t ls_status;   /* 0 converged, 1 maxfev, 2 xtol, 3 stpmax, 4 stpmin, 5 rounding, -1 none */
  int32_t m;           /* window size used by Step II */
  int32_t precision;   /* cp_precision of the bulk MTTKRPs in this iteration */
  int32_t t_passes;    /* passes over the tensor's values made by this iteration's MTTKRPs */
  int32_t nfev_pre;    /* evaluations of the one-step process's own line search in Step I
                          (CP_METHOD_NGMRES_SD; 0 otherwise) */
} cp_iter_info;

#define CP_METHOD_NGMRES 0
#define CP_METHOD_ALS    1
/* Nonlinear conjugate gradients, the paper's comparison method (Section 2.4):
   Polak-Ribiere coefficient clipped at zero, the same line search, steepest
   descent when a direction is not a descent direction or after a line search
   without a Wolfe point; iterates are not normalised after the initial guess. */
#define CP_METHOD_NCG    2
/* N-GMRES with steepest descent as the one-step process M(.) of Step I in
   place of ALS (the paper's preconditioning view of N-GMRES, Section 2.2 end,
   and its Section 5 suggestion to accelerate other methods): u_bar = u_i +
   beta d with d = -g(u_i)/||g(u_i)||_2 and beta from the same line search as
   Step III (a search without a Wolfe point takes the R13 fallback), then
   u_bar normalised with its gradient carried over; f(u_bar) and g(u_bar) are
   the accepted trial's, so Step I costs its line-search evaluations only.
   Steps II and III are unchanged. */
#define CP_METHOD_NGMRES_SD 3

typedef struct cp_options {
  int32_t method;           /* CP_METHOD_NGMRES (default), CP_METHOD_ALS, CP_METHOD_NCG or
                               CP_METHOD_NGMRES_SD */
  int32_t window;           /* w, >= 1 (20) */
  double eps;               /* delta = eps * max diag(P^T P) (1e-12) */
  double ls_ftol;           /* sufficient-decrease constant (1e-4) */
  double ls_gtol;           /* curvature constant (1e-2) */
  double ls_stp0;           /* first trial step (1.0) */
  int32_t ls_maxfev;        /* evaluations per line search (20) */
  double ls_xtol;           /* relative interval width stop (1e-15) */
  double ls_stpmin;         /* (1e-15) */
  double ls_stpmax;         /* (1e15) */
  int32_t max_iter;         /* (1000) */
  int32_t precision;        /* bulk cp_precision for the first phase (CP_PREC_FP64) */
  int32_t final_precision;  /* precision after the switch (CP_PREC_FP64) */
  double switch_rho;        /* switch to final_precision (and restart the window) once
                               rho <= switch_rho (see also switch_on_stall); 0 = switch
                               only when the stopping test would fire (0) */
  int32_t normalize_accel;  /* normalise the accelerated iterate (1) */
  cp_iter_info* trace;      /* host, nullable: per-iteration records */
  int32_t trace_cap;        /* capacity of trace */
  int32_t mttkrp_tree;      /* dense tensors of order >= 3: split the modes into a left
                               and a right group, contract T once with each group's
                               complement (two partial MTTKRPs on the same kernels and
                               precision as a per-mode MTTKRP) and take every M^(n) from
                               its group's partial in float64, so a gradient evaluation
                               or ALS sweep streams T twice instead of N times.
                               1 (default): an evaluation of a float32 tensor forms
                               both partials in one pass over T where the two-sided
                               kernel covers the shape (R <= 32, the last modes of both
                               groups of length 64 or 128); the ALS sweep of an N-GMRES
                               or ALS step takes its left partial from the last evaluation
                               when that was at the sweep's starting point (rescaled
                               for the normalisation) and then makes one pass, for its
                               right partial (which needs the updated left factors);
                               2: always one pass per partial; 0: one pass per mode.
                               Other values: CP_EINVAL */
  int32_t switch_on_stall;  /* with switch_rho > 0, also switch once rho <= 1e-2 after a
                               line search in the first precision ends without a Wolfe
                               point (1) */
  double stop_tol;          /* the stopping tolerance on rho that the precision schedule
                               anticipates: a state whose bulk precision does not accumulate
                               in float64 switches to a float64-accumulating final_precision
                               once rho <= stop_tol, so the stop is certified in float64.
                               ngmres_step applies the whole schedule (switch_rho,
                               switch_on_stall, stop_tol) at the start of each iteration;
                               cp_decompose sets stop_tol to its tol (0) */
  int32_t init;             /* CP_INIT_GIVEN: the caller's array holds the initial guess;
                               CP_INIT_SEEDED: it is drawn from `seed` as cp_init_uniform
                               does, then normalised like a given one (Section 2.4: a
                               uniformly random initial guess) (CP_INIT_GIVEN) */
  uint64_t seed;            /* seed of CP_INIT_SEEDED (0) */
} cp_options;

#define CP_INIT_GIVEN  0
#define CP_INIT_SEEDED 1

typedef struct cp_report {
  int32_t iters;            /* iterations performed */
  int32_t converged;        /* 1 if rho <= tol */
  double f;                 /* final objective */
  double rho;               /* final ||g||_2 / ||T||_F (float64 gradient of the final iterate) */
  int32_t n_fg;             /* objective/gradient evaluations */
  int32_t n_restarts;
  int32_t n_ls_fallback;
  int32_t switch_iter;      /* iteration at which the precision switched (-1 none) */
  int32_t n_trace;          /* records written to options.trace */
  double seconds;           /* host wall time of the call */
} cp_report;

/* ---- handle ---------------------------------------------------------- */

/* Create a handle on HIP device `device`.  workspace_bytes is an initial
 * reservation (0 = grow on demand).  Errors: CP_EINVAL (device), CP_ENOMEM. */
int cp_create(int device, size_t workspace_bytes, cp_handle** h);
/* Destroy a handle and free its workspace (synchronises the device). */
int cp_destroy(cp_handle* h);
/* Message of the last failing call on h (static storage of the handle). */
const char* cp_last_error(const cp_handle* h);
void cp_options_default(cp_options* opt);

/* ---- tensors ----------------------------------------------------------- */

/* Validate the descriptor, compute ||T||_F^2 (float64, fixed-order
 * reduction) and, for sparse tensors, build per-mode copies of the
 * nonzeros stably sorted by that mode's index plus segment pointers, after
 * checking coordinate bounds and duplicates.  Synchronises the stream.
 * Errors: CP_EINVAL (shape, coordinate out of range), CP_EDUPLICATE, CP_ENOMEM. */
int cp_tensor_prepare(cp_handle* h, cp_tensor* T, hipStream_t stream);
/* Free what cp_tensor_prepare attached.  Synchronises the stream the tensor
 * was prepared on (not the device): work that used the tensor on any other
 * stream must be complete before the call. */
int cp_tensor_release(cp_handle* h, cp_tensor* T);

/* ---- hot-path building blocks ---------------------------------------- */

/* MTTKRP (Section 2.3, the product T_(n) Phibar^(n) of the gradient):
 *   M_out(i, r) = sum over all index tuples with i_mode = i of
 *                 T(i_1..i_N) * prod_{k != mode} A^(k)(i_k, r)
 * mode is zero-based; u holds the factors (float64, layout above); M_out is
 * I_mode x R float64 row-major.  Dense tensors need no preparation; sparse
 * ones must be prepared.  p selects the bulk arithmetic (cp_precision).
 * Errors: CP_EINVAL (R < 1, mode out of range, precision not valid for the
 * tensor: FP32/BF16X3 need a float32 tensor, BF16X3 needs a dense one). */
int cp_mttkrp(cp_handle* h, const cp_tensor* T, const double* u, int32_t R, int32_t mode,
              int32_t p, double* M_out, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * MTTKRP as cp_mttkrp, same kernels, same arguments and bitwise the same
 * M_out, but every workspace slice comes from a static array of 64 MiB per
 * device that is part of the library (placed when the library is loaded on
 * a device, held until the process ends; its device address is looked up by
 * cp_create).  The call itself makes no hipMalloc, hipFree, hipHostMalloc or
 * other allocating call and creates no timing events (cp_profile does not
 * time it).  T's arrays, u and M_out stay the caller's; a sparse T must be
 * prepared beforehand (cp_tensor_prepare allocates).  Every call on a device
 * shares that device's array: calls on the same stream are ordered, calls
 * that overlap on one device (other streams, other host threads) race and
 * give wrong results.  The array keeps the last call's contents; every slice
 * is written before it is read, so nothing needs clearing.
 * Errors: those of cp_mttkrp; CP_ENOMEM (with the sizes in cp_last_error)
 * when the call's workspace would exceed the array -- the check runs before
 * each slice's first kernel, so nothing past the array is written, and
 * M_out is then unspecified; CP_EDEVICE when the array's address could not
 * be looked up on this device. */
int cp_mttkrp_noalloc(cp_handle* h, const cp_tensor* T, const double* u, int32_t R,
                      int32_t mode, int32_t p, double* M_out, hipStream_t stream);

/* Grams and their Hadamard products (Section 2.3): S^(k) = A^(k)^T A^(k)
 * for all k (S_out: N x R x R), Gammabar^(n) = Hadamard product of S^(k)
 * over k != n (gamma_bar_out: N x R x R, nullable), Gamma = Hadamard product
 * of all S^(k) (gamma_out: R x R, nullable).  All float64. */
int cp_gram(cp_handle* h, int32_t order, const int64_t* dims, const double* u, int32_t R,
            double* S_out, double* gamma_bar_out, double* gamma_out, hipStream_t stream);

/* Normalise and reorder the rank-one terms in place (Section 2.3, last
 * paragraph): each factor column scaled to norm lambda_r^(1/N) with lambda_r
 * the product of the column norms, terms sorted by decreasing lambda_r
 * (stable; zero terms become zero and sort last).  If g_inout is non-null it
 * is mapped to the gradient at the new point (column r of G^(n) divided by
 * that column's scale, then permuted). */
int cp_normalize(cp_handle* h, int32_t order, const int64_t* dims, double* u_inout, int32_t R,
                 double* g_inout, hipStream_t stream);

/* One ALS iteration M(u) in place (Section 2.3): for n = 1..N in order,
 * A^(n) <- M^(n) (Gammabar^(n))^-1 by Cholesky, the later modes seeing the
 * updated earlier ones; then, if normalize != 0, cp_normalize.  A
 * Gammabar^(n) that is not positive definite is retried with a shift of
 * 1e-14 tr/R and then solved by a pseudo-inverse (cyclic Jacobi eigen-
 * decomposition), as the float64 reference does.  Dense tensors of order
 * >= 3 take their MTTKRPs from the two mode-group partials (two passes over
 * T, the right group's formed after the left modes are updated). */
int cp_als_sweep(cp_handle* h, const cp_tensor* T, double* u_inout, int32_t R, int32_t p,
                 int32_t normalize, hipStream_t stream);

/* The ALS mode update alone (Section 2.3: solve the optimality equation
 * G^(n) = 0 for A^(n)): A_out = M Gbar^-1 for M (I x R) and the symmetric
 * Gbar (R x R), by Cholesky; if a pivot is not positive, Cholesky of
 * Gbar + 1e-14 tr(Gbar)/R I; if that fails too, the pseudo-inverse from a
 * cyclic Jacobi eigendecomposition (eigenvalues of magnitude below
 * R eps max|w| dropped).  kind_out (host, nullable): 0, 1 or 2 for the path
 * taken; synchronises the stream when kind_out is given. */
int cp_mode_solve(cp_handle* h, const double* M, const double* Gbar, int64_t I, int32_t R,
                  double* A_out, int32_t* kind_out, hipStream_t stream);

/* Objective and gradient at u (Optimization Problem I; Section 2.3):
 *   f = 1/2 ||T||^2 - <A^(N), M^(N)> + 1/2 sum_{r,s} Gamma(r,s)
 *   G^(n) = -M^(n) + A^(n) Gammabar^(n)           for every n
 * f_out: device, 1 double; g_out: device, L doubles (nullable: f only still
 * runs every MTTKRP it needs).  T must be prepared (for ||T||^2).  Dense
 * tensors of order >= 3: the two-level evaluation, two passes over T, or one
 * for a float32 tensor whose shape the two-sided kernel covers (see
 * cp_options.mttkrp_tree = 1). */
int cp_objective_grad(cp_handle* h, const cp_tensor* T, const double* u, int32_t R, int32_t p,
                      double* f_out, double* g_out, hipStream_t stream);

/* N-GMRES Step II (Section 2.1, accelerated iterate and normal equations):
 *   p_j = g_bar - G_j, (P^T P + delta I) alpha = -P^T g_bar,
 *   delta = eps * max_j (P^T P)_jj,  u_hat = u_bar + sum_j alpha_j (u_bar - U_j)
 * U, G: m x L row-major (window iterates and gradients), 1 <= m <= 64.
 * If every p_j is zero, or P^T P + delta I has a Cholesky pivot that is not
 * positive (possible with eps = 0 or repeated gradients), alpha = 0 and
 * u_hat = u_bar.  gTd_out: device, 1 double, nullable: g_bar^T (u_hat - u_bar),
 * the slope of Step III along d = u_hat - u_bar for this (unnormalised) u_hat
 * (ngmres_step normalises u_hat first, Section 2.3 end).  alpha_out: device m
 * doubles, nullable. */
int ngmres_accelerate(cp_handle* h, int64_t L, int32_t m, const double* U, const double* G,
                      const double* u_bar, const double* g_bar, double eps, double* u_hat_out,
                      double* gTd_out, double* alpha_out, hipStream_t stream);

/* The seeded uniform initial guess (Section 2.4: uniformly random entries):
 * u_out[i] = (x_i >> 11) * 2^-53 in [0, 1), x_i the i-th 64-bit output of
 * Philox-4x64-10 (Salmon et al., SC 2011) under the key (seed, 0), outputs
 * 4b..4b+3 being the cipher of the counter (b + 1, 0, 0, 0).  u_out: device,
 * L doubles (the caller normalises it with cp_normalize if wanted). */
int cp_init_uniform(cp_handle* h, int64_t L, uint64_t seed, double* u_out, hipStream_t stream);

/* ---- the method -------------------------------------------------------- */

/* Create an N-GMRES (or ALS) state on a prepared tensor: copies u0 (device,
 * L doubles; ignored, and may be NULL, with opt->init = CP_INIT_SEEDED),
 * normalises it, evaluates f and g and starts the window.  Keeps the window
 * (w iterates and w gradients) on the device. */
int cp_ngmres_create(cp_handle* h, const cp_tensor* T, int32_t R, const cp_options* opt,
                     const double* u0, hipStream_t stream, cp_ngmres_state** st);
/* One iteration (Steps I-III of the algorithm box for N-GMRES; u <- M(u) for
 * ALS).  Synchronises the stream (scalar readbacks).  info_out: host,
 * nullable, describes the iteration just taken.  Returns CP_OK, CP_LS_FALLBACK
 * or an error. */
int ngmres_step(cp_handle* h, cp_ngmres_state* st, cp_iter_info* info_out);
/* Current iterate, gradient (device, nullable) and f, rho (host, nullable). */
int cp_ngmres_get(cp_handle* h, cp_ngmres_state* st, double* u_out, double* g_out,
                  double* f_out, double* rho_out);
int cp_ngmres_destroy(cp_handle* h, cp_ngmres_state* st);

/* Scalar part of a state's checkpoint. */
typedef struct cp_ngmres_meta {
  int32_t it;               /* iterations taken */
  int32_t m;                /* window entries (N-GMRES; 0 otherwise) */
  int32_t precision;        /* current bulk cp_precision */
  int32_t switched;         /* the precision schedule has switched */
  int32_t stalled;          /* a reduced-precision line search ended without a Wolfe point */
  int32_t cg_fresh;         /* N-CG: the next direction is -g */
  double f;                 /* objective at u */
  double rho;               /* ||g||_2 / ||T||_F (recomputed from g by cp_ngmres_load) */
  int32_t n_fg, n_restarts, n_ls_fallback, switch_iter;
} cp_ngmres_meta;

/* Checkpoint and resume of the iteration state (Algorithm box: the iterate,
 * its gradient and the window of stored iterates and gradients).
 * save: U_out, G_out (device, window x L each, nullable) receive the window
 * entries oldest first (meta->m rows), u_out, g_out (device, L, nullable) the
 * iterate and gradient, d_out (device, L, nullable) the N-CG direction;
 * meta (host) the scalars.  load: replaces all of that in a state created on
 * the same tensor, rank and options (m <= window; m >= 1 for N-GMRES), and
 * recomputes rho from g (synchronises the stream).  A loaded state steps
 * exactly as the saved one would have.  Errors: CP_EINVAL. */
int cp_ngmres_save(cp_handle* h, cp_ngmres_state* st, double* U_out, double* G_out, double* u_out,
                   double* g_out, double* d_out, cp_ngmres_meta* meta);
int cp_ngmres_load(cp_handle* h, cp_ngmres_state* st, const double* U, const double* G,
                   const double* u, const double* g, const double* d, const cp_ngmres_meta* meta);

/* Intermediate values of the last N-GMRES iteration (Steps I-II): u_bar =
 * M(u_i), g_bar = g(u_bar), the normalised accelerated iterate u_hat, the
 * direction d = u_hat - u_bar (device, L each, nullable), f(u_bar) and the
 * slope g_bar^T d (host, nullable).  CP_EINVAL before the first N-GMRES step. */
int cp_ngmres_last_step(cp_handle* h, cp_ngmres_state* st, double* u_bar, double* g_bar,
                        double* u_hat, double* d, double* f_bar, double* slope);

/* Decompose a prepared tensor: iterate until rho = ||g||_2/||T||_F <= tol or
 * max_iter.  u_inout (device, L doubles): initial guess in (unless
 * opt->init = CP_INIT_SEEDED), result out.  u_inout = NULL: the seeded guess
 * of opt->seed is used and only rep_out describes the result.  opt nullable
 * (defaults).  rep_out: host, nullable.  Returns CP_OK, CP_MAXITER or an error. */
int cp_decompose(cp_handle* h, const cp_tensor* T, int32_t R, double tol, const cp_options* opt,
                 double* u_inout, cp_report* rep_out, hipStream_t stream);

/* ---- batched N-GMRES for small dense requests ---------------------------- */

/* Largest tensor (entries) the batched path takes. */
#define CP_BATCH_MAX_ELEMS (1 << 20)

typedef struct cp_batch_request {
  const cp_tensor* T;      /* dense float32, order 3 or 4, at most CP_BATCH_MAX_ELEMS entries,
                              prepared (cp_tensor_prepare: ||T||^2) */
  int32_t R;               /* 1..32 */
  double tol;              /* stop once rho = ||g||_2 / ||T||_F <= tol */
  double* u_inout;         /* device, L doubles: initial guess in, result out */
  cp_iter_info* trace;     /* host, nullable: per-iteration records as cp_decompose writes them */
  int32_t trace_cap;
  int32_t status;          /* out: CP_OK (converged), CP_MAXITER or an error */
  cp_report report;        /* out (seconds: the whole batch) */
} cp_batch_request;

/* Decompose n small dense tensors together by N-GMRES with ALS (Section 2.1,
 * algorithm box; Section 2.3) in float64 arithmetic on the float32 values,
 * with one kernel launch per step over all unfinished requests: each launch
 * advances every request by one device phase (the start; Steps I-II; one
 * line-search trial; the end of an iteration), one workgroup per request, and
 * one readback of every request's scalars follows.  Each request's control
 * (restart test, Moré-Thuente line search with the R13 fallback, window,
 * stopping test) is its own, and every sum has a fixed order, so a request's
 * result is bitwise the same alone or in any batch.  opt (nullable):
 * method must be CP_METHOD_NGMRES, window <= 21; the precision fields are
 * ignored.  Synchronises the stream.  Errors: CP_EINVAL (a request outside
 * the batched path's limits), CP_ENOMEM; per-request errors in status. */
int cp_batch_decompose(cp_handle* h, int32_t n, cp_batch_request* reqs, const cp_options* opt,
                       hipStream_t stream);

/* ---- serving: continuous batching of decomposition requests ------------- */

typedef struct cp_server cp_server;

typedef struct cp_server_opts {
  int32_t slots;          /* decompositions running at once, each on its own stream (4; max 16) */
  size_t hbm_budget;      /* bytes the running requests may occupy (0: 80% of free memory) */
  cp_options decompose;   /* method options of every request (trace ignored) */
  int64_t batch_elems;    /* > 0 (and decompose.method = CP_METHOD_NGMRES, window <= 21):
                             dense float32 requests of order 3 or 4 with 1 <= R <= 32 and at
                             most this many entries (capped at CP_BATCH_MAX_ELEMS) run on the
                             batched path of cp_batch_decompose, admitted continuously into
                             one batch that a thread of its own advances, one launch per step
                             for all of them, in float64 arithmetic (precision fields ignored);
                             0: every request takes a slot (0) */
  int32_t batch_capacity; /* requests in the batch at once (256) */
} cp_server_opts;

typedef struct cp_result {
  int64_t req_id;         /* id returned by cp_server_submit */
  uint64_t tag;           /* caller's tag */
  int32_t status;         /* cp_decompose status (CP_OK, CP_MAXITER) or an error */
  int32_t iters;
  int32_t converged;
  int32_t n_fg;
  int32_t switch_iter;
  int32_t slot;           /* slot that ran it; -1: the batched path */
  double f;
  double rho;
  double t_submit;        /* seconds since cp_server_create */
  double t_start;         /* admitted */
  double t_end;           /* finished */
} cp_result;

/* Start a server on `device` with `slots` worker threads, each owning a
 * handle and a HIP stream (default priority), and, with batch_elems > 0, a
 * batch thread with its own handle and stream.  Requests are admitted in
 * arrival order (per path) when a slot (or batch place) is free and their
 * footprint (tensor, N-GMRES window and state, workspace estimate) fits in
 * hbm_budget beside the running ones.  o nullable (defaults). */
int cp_server_create(int device, const cp_server_opts* o, cp_server** s);
/* Queue a decomposition of T (device arrays; prepared by the server) to
 * rho <= tol from the initial guess in u_inout (device, L doubles), which
 * receives the result.  T's arrays and u_inout must stay valid until the
 * result has been polled.  A request larger than the whole budget completes
 * at once with status CP_ENOMEM. */
int cp_server_submit(cp_server* s, const cp_tensor* T, int32_t R, double tol, double* u_inout,
                     uint64_t tag, int64_t* req_id);
/* Move up to max_out finished results into out (host).  wait_for > 0 blocks
 * until that many are available or nothing is queued or running. */
int cp_server_poll(cp_server* s, int32_t wait_for, cp_result* out, int32_t max_out,
                   int32_t* n_out);
/* Queue length, running requests, bytes admitted, budget (host, nullable). */
int cp_server_stats(cp_server* s, int32_t* queued, int32_t* active, size_t* in_use,
                    size_t* budget);
/* Stop: running requests finish, queued ones are dropped; joins the workers. */
int cp_server_destroy(cp_server* s);

/* ---- kernel timing ------------------------------------------------------ */

/* Kernel ids for cp_profile_read. */
#define CP_KERNEL_DENSE_MTTKRP  0   /* main dense MTTKRP kernel, float32-accumulating
                                       precisions (CP_PREC_FP32, CP_PREC_BF16X3) */
#define CP_KERNEL_SPARSE_MTTKRP 1   /* main sparse segmented-reduction kernel */
#define CP_KERNEL_STREAM_READ   2   /* cp_stream_read */
#define CP_KERNEL_GROUP_MTTKRP  3   /* second level of the two-level evaluation: one mode's
                                       MTTKRP from its group's partial contraction */
#define CP_KERNEL_DENSE_MTTKRP_F64 4 /* main dense MTTKRP kernel, float64-accumulating
                                       precisions (CP_PREC_FP64, CP_PREC_FP32IN_FP64ACC) */
#define CP_KERNEL_SPARSE_GATHER 5   /* cp_sparse_gather_read */
#define CP_KERNEL_DENSE_TWOSIDED 6  /* both group partials of a two-level evaluation from one
                                       pass over T, float32-accumulating precisions */
#define CP_KERNEL_DENSE_TWOSIDED_F64 7 /* the same, float64-accumulating precisions */

/* Enable (1) or disable (0) HIP-event timing of the main MTTKRP kernels on
 * the stream each is launched on; enabling clears the counters. */
int cp_profile(cp_handle* h, int32_t enable);
/* Which kernel ids cp_profile times: bit k of kernel_mask selects id k
 * (default 0xFF, all eight).  Each timed launch adds two event records to its
 * stream, so timing only the kernel being measured keeps the others' launch
 * gaps out of a timed run.  CP_EINVAL for bits above 7. */
int cp_profile_select(cp_handle* h, uint32_t kernel_mask);
/* Synchronise the recorded events and return, for kernel id `kernel`, the
 * number of timed launches and their summed duration in milliseconds
 * (host pointers). */
int cp_profile_read(cp_handle* h, int32_t kernel, int64_t* launches, double* total_ms);

/* Measurement reference (not part of the method): read `bytes` of device
 * memory at `buf` once, with 16-byte loads spread over the whole chip, and
 * add them into a per-workgroup value in library workspace so the reads are
 * kept.  `buf` must be 16-byte aligned and `bytes` a multiple of 16
 * (CP_EINVAL otherwise).  Timed under CP_KERNEL_STREAM_READ while profiling
 * is on: the achievable streaming-read bandwidth that the MTTKRP rooflines
 * are also compared with. */
int cp_stream_read(cp_handle* h, const void* buf, size_t bytes, hipStream_t stream);

/* Measurement reference (not part of the method): the factor-row gathers of
 * the sparse FP32 MTTKRP of `mode` alone.  For every nonzero of the prepared
 * tensor's mode-sorted copy it reads the other modes' coordinates and the
 * corresponding rows of the padded float32 factor copy, with the MTTKRP
 * kernel's waves, lane groups and 16-byte loads, and keeps one value per
 * wave in library workspace: no values, row indices, products with the
 * tensor or segmented reduction.  Timed under CP_KERNEL_SPARSE_GATHER while
 * profiling is on: the achievable gather rate that the sparse MTTKRP is
 * compared with.  Errors: CP_EINVAL (dense or unprepared tensor, R outside
 * 1..64, mode out of range). */
int cp_sparse_gather_read(cp_handle* h, const cp_tensor* T, const double* u, int32_t R,
                          int32_t mode, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* CPNG_H */
