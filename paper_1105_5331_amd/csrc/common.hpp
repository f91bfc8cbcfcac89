// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "cpng.h"

namespace cpng {

// A device buffer owned by the handle, grown on demand from host code.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// A gradient epilogue G(i, r) = -M(i, r) + sum_q A(i, q) Gbar(q, r) that the
// next dense MTTKRP folds into its final reduction (set by the caller for one
// call; `used` tells it whether the MTTKRP took it).
struct GradEpi {
  const double* A = nullptr;
  const double* Gbar = nullptr;
  double* G = nullptr;
  bool used = false;
};

struct Status {
  int code = CP_OK;
  std::string msg;
};

}  // namespace cpng

struct cp_handle {
  int device = 0;
  int max_lds = 0;   // bytes of LDS one workgroup may use (queried on first need)
  std::string err;
  // Workspace slices, each grown on demand (host calls only).
  cpng::DevBuf part;     // MTTKRP per-workgroup partials
  cpng::DevBuf part2;    // their group sums (second reduction stage)
  cpng::DevBuf stage;    // float32 copies of the factors
  cpng::DevBuf mbuf;     // MTTKRP outputs used internally (N x maxI x R doubles)
  cpng::DevBuf small;    // Grams, Gammabar, Gamma, scales, perms, alpha, scalars
  cpng::DevBuf red;      // reduction partials
  cpng::DevBuf carry;    // sparse segment carries
  cpng::DevBuf otab;     // per-launch outer-index tables of the streaming MTTKRP
  cpng::DevBuf ybuf;     // mode-group partials of the two-level evaluation (float64)
  uint64_t gen = 0;           // bumped whenever a workspace slice is reallocated
  uint64_t ywrites = 0;       // bumped by every evaluation or sweep that writes ybuf
  cpng::GradEpi epi;          // pending gradient epilogue for the next dense MTTKRP
  double* pinned = nullptr;   // host pinned readback area (64 doubles)
  int* flags = nullptr;       // device status word (ALS solve fallbacks)
  // optional event timing of the main MTTKRP kernels
  bool prof = false;
  static constexpr int kKernelIds = 8;
  uint32_t prof_mask = 0xFFu;   // kernel ids timed while prof is on
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending[kKernelIds];
  int64_t prof_launches[kKernelIds] = {};
  double prof_ms[kKernelIds] = {};
  // passes over a tensor's values made by MTTKRP launches (always counted)
  int64_t t_passes = 0;
  // Allocation-free calls (cp_mttkrp_noalloc): while `arena` is set, ensure()
  // hands out consecutive 256-byte-aligned slices of it instead of allocating.
  char* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  // device address of this device's static scratch array (looked up by
  // cp_create), or null with the lookup's error code in scratch_err
  void* scratch = nullptr;
  int scratch_err = 0;
};

namespace cpng {

// Sets h->err and returns code.
int fail(cp_handle* h, int code, const char* fmt, ...);

// Ensure `b` holds at least `bytes`; synchronises `stream` before freeing an
// old allocation that may still be in use.
int ensure(cp_handle* h, DevBuf& b, size_t bytes, hipStream_t stream);

#define CP_HIP(h, call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::cpng::fail((h), CP_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define CP_LAUNCH_CHECK(h)                                                           \
  do {                                                                               \
    hipError_t e_ = hipGetLastError();                                               \
    if (e_ != hipSuccess)                                                            \
      return ::cpng::fail((h), CP_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e_)); \
  } while (0)

#define CP_TRY(x)            \
  do {                       \
    int s_ = (x);            \
    if (s_ < 0) return s_;   \
  } while (0)

// Shape helpers.
struct Shape {
  int N = 0;
  int64_t dims[CP_MAX_ORDER] = {};
  int64_t off[CP_MAX_ORDER + 1] = {};   // factor offsets in u, in rows (multiply by R)
  int64_t total() const {
    int64_t t = 1;
    for (int k = 0; k < N; ++k) t *= dims[k];
    return t;
  }
  int64_t sum_dims() const { return off[N]; }
  int64_t max_dim() const {
    int64_t m = 0;
    for (int k = 0; k < N; ++k) m = dims[k] > m ? dims[k] : m;
    return m;
  }
};

int make_shape(cp_handle* h, int order, const int64_t* dims, Shape* s);

// Timing id of a dense MTTKRP kernel by its accumulation type.
template <typename CT>
constexpr int dense_kernel_id() {
  return sizeof(CT) == 8 ? CP_KERNEL_DENSE_MTTKRP_F64 : CP_KERNEL_DENSE_MTTKRP;
}

// Event timing of a main kernel launch (no-op unless h->prof selects id):
// the timer holds a pair of events that CP_TIMED_LAUNCH hands to the launch
// itself (hipExtLaunchKernelGGL records the kernel's own start and end, with
// no extra packets on the stream); the destructor files the pair.
struct KernelTimer {
  cp_handle* h;
  int id;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  KernelTimer(cp_handle* h_, int id_, hipStream_t st_);
  ~KernelTimer();
};

#define CP_TIMED_LAUNCH(timer, kernel, grid, block, lds, stream, ...)                         \
  do {                                                                                         \
    if ((timer).a && (timer).b)                                                                \
      hipExtLaunchKernelGGL(kernel, grid, block, lds, stream, (timer).a, (timer).b, 0,         \
                            __VA_ARGS__);                                                      \
    else                                                                                       \
      hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);                       \
  } while (0)

// Library-owned per-mode sorted copies of a sparse tensor.
struct SparseMode {
  int32_t* coords = nullptr;   // (N-1) x nnz: the other modes' indices, sorted by this mode
  void* values = nullptr;      // nnz values sorted by this mode
  int32_t* rows = nullptr;     // nnz: this mode's index of each sorted nonzero
  int64_t* seg = nullptr;      // I_n + 1 segment pointers
};
struct SparsePrepared {
  int N = 0;
  int64_t nnz = 0;
  int dtype = CP_F32;
  hipStream_t stream = nullptr;   // the stream cp_tensor_prepare ran on
  SparseMode mode[CP_MAX_ORDER];
};

// ---- launchers (defined in the .hip files) --------------------------------
int dense_mttkrp(cp_handle* h, const cp_tensor* T, const Shape& s, const double* u, int R,
                 int mode, int prec, double* M, hipStream_t st);
int sparse_mttkrp(cp_handle* h, const cp_tensor* T, const Shape& s, const double* u, int R,
                  int mode, int prec, double* M, hipStream_t st);
int sparse_prepare(cp_handle* h, cp_tensor* T, const Shape& s, hipStream_t st);
int sparse_release(cp_handle* h, cp_tensor* T);
int sparse_gather_ref(cp_handle* h, const cp_tensor* T, const Shape& s, const double* u, int R,
                      int mode, hipStream_t st);
int stage_factors_f32(cp_handle* h, const double* u, int64_t L, float** out, hipStream_t st);
int dense_fast_bf16x3(cp_handle* h, const float* T, const double* u, const Shape& s, int R,
                      int mode, double* M, hipStream_t st);
int dense_fast_mfma_f32(cp_handle* h, const float* T, const double* u, const Shape& s, int R,
                        int mode, double* M, hipStream_t st);
int dense_fast_mfma_f64acc(cp_handle* h, const float* T, const double* u, const Shape& s, int R,
                           int mode, double* M, hipStream_t st);
// Both group partials of the two-level evaluation from one pass over a
// float32 T (dense_fast.hip); CP_OK after launching, 1 if not covered.
int dense_twosided(cp_handle* h, const float* T, const double* u, const Shape& s, int split, int R,
                   int prec, double* XL, double* XR, hipStream_t st);
template <typename TT, typename CT>
int dense_fast_vec(cp_handle* h, const TT* T, const CT* fac, const Shape& s, int R, int mode,
                   double* M, hipStream_t st);

// two-level evaluation of all modes (tree.hip): left modes [0, split), right
// modes [split, N).  tree_split returns the split, or 0 where it does not apply.
int tree_split(const cp_tensor* T, const Shape& s, int prec);
size_t tree_partial_elems(const Shape& s, int split, int R, bool left);
int tree_partial(cp_handle* h, const cp_tensor* T, const Shape& s, const double* u, int R, int prec,
                 int split, bool left, double* X, hipStream_t st);
// Every mode's MTTKRP from the two group partials in one launch (order <= 4,
// every second-level sum short), with the gradient epilogue when g is given:
// G^(n) = -M^(n) + A^(n) Gbar^(n).  Returns 1 when the shape is not covered.
// Both partials (float32 tensor, both groups of more than one mode) from one
// pass over T: CP_OK after launching, 1 where the shape is not covered.
int tree_partials_one_pass(cp_handle* h, const cp_tensor* T, const Shape& s, const double* u, int R,
                           int prec, int split, double* XL, double* XR, hipStream_t st);
int tree_all_modes(cp_handle* h, const Shape& s, int split, const double* XL, const double* XR,
                   const double* u, int R, double* M, const double* Gbar, double* g,
                   hipStream_t st);
// X_L at the iterate renormalised by the plan (scales, perm) of normalize()
int tree_rescale_left(cp_handle* h, const Shape& s, int split, int R, double* XL,
                      const double* scales, const int* perm, hipStream_t st);
int tree_mode(cp_handle* h, const Shape& s, int lo, int hi, const double* X, const double* u, int R,
              int mode, double* M, hipStream_t st);

// batched N-GMRES engine for small dense requests (batch.hip)
struct BatchEngine;
struct BatchItem;
bool batch_eligible(const cp_tensor* T, int R, int64_t max_elems);
BatchEngine* batch_engine_create(cp_handle* h, hipStream_t st, const cp_options& o, int capacity);
void batch_engine_destroy(BatchEngine* e);
int batch_engine_add(BatchEngine* e, const cp_tensor* T, int R, double tol, const double* u0,
                     double* u_out, uint64_t tag, cp_iter_info* trace, int trace_cap,
                     BatchItem** out);
// one launch over every active request; finished ones are appended to *finished
int batch_engine_tick(BatchEngine* e, std::vector<BatchItem*>* finished);
int batch_engine_active(const BatchEngine* e);
// moves every active request to *out (after a failed tick)
void batch_engine_drain(BatchEngine* e, std::vector<BatchItem*>* out);
void batch_item_report(const BatchItem* it, cp_report* rep, int* status, uint64_t* tag);
void batch_item_delete(BatchItem* it);   // frees its device memory too
int64_t batch_footprint(const cp_tensor* T, int R, int window);

// small kernels
// With factor_mode >= 0 also factorises Gammabar^(factor_mode) for the next
// mode_solve(..., Gbar = nullptr, ...).  With only_mode >= 0 only that mode's
// Gram is recomputed; S must hold the other modes' Grams of the same factors.
int gram_all(cp_handle* h, const Shape& s, const double* u, int R, double* S, double* Gbar,
             double* Gam, hipStream_t st, int factor_mode = -1, int only_mode = -1);
int normalize(cp_handle* h, const Shape& s, double* u, int R, double* g, hipStream_t st,
              const double** scales_out = nullptr, const int** perm_out = nullptr);
// A = M Gbar^-1 (Gbar nullptr: use the factor gram_all formed).
int mode_solve(cp_handle* h, const double* M, const double* Gbar, int64_t I, int R, double* A,
               hipStream_t st);
int grad_epilogue(cp_handle* h, const double* M, const double* A, const double* Gbar, int64_t I,
                  int R, double* G, hipStream_t st);
// out[0] = sum x*y (fixed-order two-stage reduction), device result
int dot(cp_handle* h, const double* x, const double* y, int64_t n, double* out, hipStream_t st);
int sumsq_tensor(cp_handle* h, const void* v, int dtype, int64_t n, double* out, hipStream_t st);
int stream_read(cp_handle* h, const void* buf, size_t bytes, hipStream_t st);
// f = 0.5*normsq - <A, M> + 0.5*sum(Gamma), the dot and the combination in
// two launches
int objective_from_dot(cp_handle* h, const double* A, const double* M, int64_t n, double normsq,
                       const double* Gam, int R, double* f, hipStream_t st);
// y1 = x1, y2 = x2 (n doubles each) in one launch
int copy2(cp_handle* h, const double* x1, double* y1, const double* x2, double* y2, int64_t n,
          hipStream_t st);
int axpy_to(cp_handle* h, const double* x, double a, const double* d, double* y, int64_t n,
            hipStream_t st);   // y = x + a*d
int sub_to(cp_handle* h, const double* a, const double* b, double* y, int64_t n,
           hipStream_t st);    // y = a - b
int cg_direction(cp_handle* h, const double* g, double gamma, double* d, int64_t n,
                 hipStream_t st);   // d = -g + gamma d
int neg_div_to(cp_handle* h, const double* x, double s, double* y, int64_t n,
               hipStream_t st);     // y = -x / s

// u[i] = i-th double of the seeded Philox-4x64-10 stream (key (seed, 0),
// block b from counter b + 1), in [0, 1)
int init_uniform(cp_handle* h, int64_t L, uint64_t seed, double* u, hipStream_t st);

// Per-call values of the N-GMRES kernels kept in device memory, so that a
// captured launch sequence can be replayed with new values: the line-search
// step and the window's current size and oldest slot.
struct StepPar {
  double beta;
  int32_t m;
  int32_t whead;
};
int set_steppar(cp_handle* h, StepPar* p, double beta, int m, int whead, hipStream_t st);
int axpy_par(cp_handle* h, const double* x, const StepPar* par, const double* d, double* y,
             int64_t n, hipStream_t st);   // y = x + par->beta * d
// Window of stored iterates: slot s at ubase + s*L (gbase + s*L); the j-th
// oldest of par->m entries is slot (par->whead + j) % wcap.
int step2(cp_handle* h, int64_t L, const double* ubase, const double* gbase, int wcap,
          const StepPar* par, const double* ubar, const double* gbar, double eps, double* uhat,
          double* alpha, hipStream_t st);

}  // namespace cpng
