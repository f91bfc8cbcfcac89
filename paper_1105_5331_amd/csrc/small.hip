// Small float64 kernels around the MTTKRP: Grams and their Hadamard
// products, normalisation/reordering, the ALS mode solve (Cholesky with the
// shift and pseudo-inverse fallbacks), the gradient epilogue, fixed-order
// reductions, and N-GMRES Step II.
#include "common.hpp"
#include "factor.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>

namespace cpng {

int fail(cp_handle* h, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h) h->err = buf;
  return code;
}

int ensure(cp_handle* h, DevBuf& b, size_t bytes, hipStream_t stream) {
  if (bytes <= b.bytes) return CP_OK;
  if (h->arena) {   // allocation-free call: the next slice of the static scratch
    const size_t off = (h->arena_used + 255) & ~size_t(255);
    if (off > h->arena_cap || bytes > h->arena_cap - off)
      return fail(h, CP_ENOMEM,
                  "this call needs more workspace than the %zu-byte static scratch "
                  "(%zu bytes used, %zu more requested)", h->arena_cap, h->arena_used, bytes);
    b.ptr = h->arena + off;
    b.bytes = bytes;
    h->arena_used = off + bytes;
    return CP_OK;
  }
  size_t want = std::max(bytes, b.bytes + b.bytes / 2);
  want = (want + 4095) & ~size_t(4095);
  if (b.ptr) {
    CP_HIP(h, hipStreamSynchronize(stream));
    CP_HIP(h, hipFree(b.ptr));
    b.ptr = nullptr;
    b.bytes = 0;
  }
  h->gen++;   // captured launch sequences that used the old slice are stale
  if (hipMalloc(&b.ptr, want) != hipSuccess) {
    b.ptr = nullptr;
    return fail(h, CP_ENOMEM, "device allocation of %zu bytes failed", want);
  }
  b.bytes = want;
  return CP_OK;
}

// A new event per timed launch boundary, destroyed once its time is read: a
// reused event (one that already timed another launch) has reported wrong
// intervals for hipExtLaunchKernelGGL launches.
static hipEvent_t new_event(cp_handle*) {
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

KernelTimer::KernelTimer(cp_handle* h_, int id_, hipStream_t st_) : h(h_), id(id_), st(st_) {
  if (!h->prof || !((h->prof_mask >> id) & 1u)) return;
  a = new_event(h);
  b = new_event(h);
  if (!a || !b) {   // no timing for this launch
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    a = b = nullptr;
  }
}

KernelTimer::~KernelTimer() {
  if (!a || !b) return;
  h->ev_pending[id].emplace_back(a, b);
  if (h->ev_pending[id].size() >= 512) {   // fold old pairs to bound the pool
    for (auto& pr : h->ev_pending[id]) {
      float ms = 0.f;
      (void)hipEventSynchronize(pr.second);
      if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
        h->prof_ms[id] += ms;
        h->prof_launches[id]++;
      }
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    h->ev_pending[id].clear();
  }
}

int make_shape(cp_handle* h, int order, const int64_t* dims, Shape* s) {
  if (order < 1 || order > CP_MAX_ORDER)
    return fail(h, CP_EINVAL, "order %d outside 1..%d", order, CP_MAX_ORDER);
  s->N = order;
  s->off[0] = 0;
  for (int k = 0; k < order; ++k) {
    if (dims[k] < 1) return fail(h, CP_EINVAL, "dims[%d] = %lld < 1", k, (long long)dims[k]);
    s->dims[k] = dims[k];
    s->off[k + 1] = s->off[k] + dims[k];
  }
  return CP_OK;
}

namespace {

constexpr int kRowsPerChunk = 64;

// sum_{q < n} p[q * stride] in q order; the loads go out 8 at a time so a
// long sum is not one memory latency per term.
__device__ inline double ordered_sum(const double* __restrict__ p, int64_t n, int64_t stride) {
  double s = 0.0;
  for (int64_t q0 = 0; q0 < n; q0 += 8) {
    double v[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) v[b] = q0 + b < n ? p[(q0 + b) * stride] : 0.0;
#pragma unroll
    for (int b = 0; b < 8; ++b) s += v[b];
  }
  return s;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

struct ModeTable {
  int N, R;
  int64_t dims[CP_MAX_ORDER];
  int64_t off[CP_MAX_ORDER + 1];     // row offsets
  int64_t coff[CP_MAX_ORDER + 1];    // chunk offsets (kRowsPerChunk rows per chunk)
};

ModeTable table(const Shape& s, int R) {
  ModeTable t{};
  t.N = s.N;
  t.R = R;
  t.coff[0] = 0;
  for (int k = 0; k < s.N; ++k) {
    t.dims[k] = s.dims[k];
    t.off[k] = s.off[k];
    t.coff[k + 1] = t.coff[k] + (s.dims[k] + kRowsPerChunk - 1) / kRowsPerChunk;
  }
  t.off[s.N] = s.off[s.N];
  return t;
}

// ---- Grams -----------------------------------------------------------------
// part[(chunk) * R * R + r * R + q] = sum_{rows in chunk} A(i, r) A(i, q); the
// chunk index ch0 + blockIdx.x runs over every mode's chunks (or one mode's).
// The chunk's rows (at most 64 x 64 values, 16 per thread) are loaded with
// every load in flight, staged in LDS, and each entry summed in row order.
__global__ __launch_bounds__(256) void gram_partial_kernel(const double* __restrict__ u,
                                                           ModeTable t, int64_t ch0,
                                                           double* __restrict__ part) {
  static_assert(kRowsPerChunk * kMaxR == 16 * 256, "16 staged values per thread");
  __shared__ double rows[kRowsPerChunk * kMaxR];
  const int R = t.R;
  const int64_t ch = ch0 + blockIdx.x;
  int k = 0;
  while (ch >= t.coff[k + 1]) ++k;
  const int64_t i_begin = (ch - t.coff[k]) * kRowsPerChunk;
  const int nr = (int)min<int64_t>(kRowsPerChunk, t.dims[k] - i_begin);
  const double* A = u + (t.off[k] + i_begin) * R;   // the chunk's rows, contiguous
  const int n = nr * R;
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + q * 256;
    v[q] = e < n ? A[e] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + q * 256;
    if (e < n) rows[e] = v[q];
  }
  __syncthreads();
  const int RR = R * R;
  if (R <= 16) {
    // R * R <= 256: one entry per thread, summed in row order from zero
    const int pr = threadIdx.x;
    if (pr < RR) {
      const int r = pr / R, c = pr - (pr / R) * R;
      double s = 0.0;
      for (int ii = 0; ii < nr; ++ii) s = fma(rows[ii * R + r], rows[ii * R + c], s);
      part[ch * RR + pr] = s;
    }
    return;
  }
  if (R <= 32) {
    // thread t: column c = t % 32, rows t / 32 + 8 q (q < 4): per row of the
    // chunk one load of column c and four loads the wave reads at two
    // addresses; each sum in row order from zero
    const int c = (int)threadIdx.x & 31;
    const int ce = c < R ? c : 0;
    int ra[4];
    bool on[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = ((int)threadIdx.x >> 5) + 8 * q;
      on[q] = r < R && c < R;
      ra[q] = on[q] ? r : 0;
    }
    double p[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int ii = 0; ii < nr; ++ii) {
      const double b = rows[ii * R + ce];
#pragma unroll
      for (int q = 0; q < 4; ++q) p[q] = fma(rows[ii * R + ra[q]], b, p[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (on[q]) part[ch * RR + ra[q] * R + c] = p[q];
    return;
  }
  // R > 32: a thread's entries in groups of four sums run side by side (each
  // still in row order from zero); entries past R * R read entry 0 and are
  // dropped
  for (int q0 = 0; q0 * 256 < RR; q0 += 4) {
    int ra[4], ca[4];
    double s[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int pr = threadIdx.x + (q0 + q) * 256;
      const int pe = pr < RR ? pr : 0;
      ra[q] = pe / R;
      ca[q] = pe - ra[q] * R;
      s[q] = 0.0;
    }
#pragma unroll 4
    for (int ii = 0; ii < nr; ++ii) {
#pragma unroll
      for (int q = 0; q < 4; ++q) s[q] = fma(rows[ii * R + ra[q]], rows[ii * R + ca[q]], s[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int pr = threadIdx.x + (q0 + q) * 256;
      if (pr < RR) part[ch * RR + pr] = s[q];
    }
  }
}

// S^(k) = sum of that mode's chunk partials (chunk order); Gammabar^(n) and
// Gamma as products over k in increasing order.
template <int RM>
__device__ __attribute__((noinline)) void factor_block(const double* __restrict__ G, int R,
                                                      double* __restrict__ F,
                                                      int* __restrict__ kind,
                                                      int* __restrict__ flags, bool try_plain);
template <int RM>
__device__ __forceinline__ bool chol_wave(const double* __restrict__ G, int R,
                                          double* __restrict__ F);

// With fmode >= 0 the same block then factorises Gammabar^(fmode) for the
// ALS mode solve (factor_block).  With only >= 0 the partials hold mode
// `only` alone and S already holds the other modes' Grams.  Two phases: the
// chunk sums into S, then (after the block barrier) the products, with the
// loads of two entries in flight at a time; Gammabar^(fmode) is also kept
// in LDS for the factorisation (RM: R rounded up to 16, 32 or 64).
template <int RM>
// With u non-null (only >= 0, R <= 32, at most 4 chunks) the block forms
// S^(only) itself from the rows in u, chunk by chunk through LDS: each
// chunk's sum in row order, the chunk sums added in chunk order, as the
// partial kernel and the chunk sum would (part is then unused).
__global__ __launch_bounds__(256) void gram_final_kernel(const double* __restrict__ part, ModeTable t,
                                  double* __restrict__ S, double* __restrict__ Gbar,
                                  double* __restrict__ Gam, int fmode, double* __restrict__ F,
                                  int* __restrict__ kind, int* __restrict__ flags, int only,
                                  const double* __restrict__ u) {
  __shared__ double gl[kMaxR * kMaxR];
  const int R = t.R;
  const int RR = R * R;
  bool direct = false;
  if constexpr (RM <= 32) {
    static_assert(kRowsPerChunk * 32 <= 8 * 256 && kMaxR * kMaxR >= kRowsPerChunk * 32, "staging");
    if (u) {
      direct = true;
      const int k = only;
      const double* A = u + t.off[k] * R;
      const int64_t I = t.dims[k];
      // R > 16: thread t takes column c = t % 32, rows t / 32 + 8 q (q < 4),
      // so a row of the chunk gives one load of column c and four loads the
      // wave reads at two addresses; entries outside R x R read entry 0 and
      // are dropped.  R <= 16: one entry per thread (tot[0]).
      const int c = (int)threadIdx.x & 31;
      int ra[4];
      bool on[4];
      double tot[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = ((int)threadIdx.x >> 5) + 8 * q;
        on[q] = r < R && c < R;
        ra[q] = on[q] ? r : 0;
      }
      const int ce = c < R ? c : 0;
      for (int64_t i0 = 0; i0 < I; i0 += kRowsPerChunk) {
        const int nr = (int)min<int64_t>(kRowsPerChunk, I - i0);
        const int n = nr * R;
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int e = threadIdx.x + q * 256;
          v[q] = e < n ? A[i0 * R + e] : 0.0;
        }
        __syncthreads();   // the previous chunk's reads of gl are done
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int e = threadIdx.x + q * 256;
          if (e < n) gl[e] = v[q];
        }
        __syncthreads();
        if (R <= 16) {
          // R * R <= 256: one entry per thread (entry threadIdx.x), its chunk
          // sum in row order from zero
          if ((int)threadIdx.x < RR) {
            const int r = (int)threadIdx.x / R, cc = (int)threadIdx.x - r * R;
            double p = 0.0;
            for (int ii = 0; ii < nr; ++ii) p = fma(gl[ii * R + r], gl[ii * R + cc], p);
            tot[0] += p;
          }
        } else {
          // the chunk's four sums, each in row order from zero
          double p[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
          for (int ii = 0; ii < nr; ++ii) {
            const double b = gl[ii * R + ce];
#pragma unroll
            for (int q = 0; q < 4; ++q) p[q] = fma(gl[ii * R + ra[q]], b, p[q]);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) tot[q] += p[q];
        }
      }
      if (R <= 16) {
        if ((int)threadIdx.x < RR) S[(int64_t)k * RR + threadIdx.x] = tot[0];
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (on[q]) S[(int64_t)k * RR + ra[q] * R + c] = tot[q];
      }
    }
  }
  if (!direct) {
    const int k0 = only >= 0 ? only : 0;
    const int k1 = only >= 0 ? only + 1 : t.N;
    for (int k = k0; k < k1; ++k) {
      const int64_t nc = t.coff[k + 1] - t.coff[k];
      const double* pk = part + t.coff[k] * RR;
      for (int pr = threadIdx.x; pr < RR; pr += 256) S[(int64_t)k * RR + pr] = ordered_sum(pk + pr, nc, RR);
    }
  }
  __syncthreads();   // S stores visible to the block; the staging in gl is done
  constexpr int kGE = 2;   // entries per thread with their loads in flight together
  for (int p0 = threadIdx.x; p0 < RR; p0 += kGE * 256) {
    double sk[kGE][CP_MAX_ORDER];
#pragma unroll
    for (int q = 0; q < kGE; ++q) {
      const int pr = p0 + q * 256;
#pragma unroll
      for (int k = 0; k < CP_MAX_ORDER; ++k)
        sk[q][k] = (pr < RR && k < t.N) ? S[(int64_t)k * RR + pr] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kGE; ++q) {
      const int pr = p0 + q * 256;
      if (pr >= RR) break;
      if (Gbar) {
#pragma unroll
        for (int n = 0; n < CP_MAX_ORDER; ++n) {
          if (n >= t.N) break;
          double gb = 1.0;
#pragma unroll
          for (int k = 0; k < CP_MAX_ORDER; ++k)
            if (k < t.N && k != n) gb *= sk[q][k];
          Gbar[(int64_t)n * RR + pr] = gb;
          if (n == fmode) gl[pr] = gb;
        }
      }
      if (Gam) {
        double g = 1.0;
#pragma unroll
        for (int k = 0; k < CP_MAX_ORDER; ++k)
          if (k < t.N) g *= sk[q][k];
        Gam[pr] = g;
      }
    }
  }
  if (fmode >= 0) {
    __syncthreads();   // Gammabar^(fmode) complete in LDS and in global memory
    // the plain factorisation from LDS by the first wave; the shifted and
    // eigenvalue paths (factor_block) read the global copy when it fails
    __shared__ int plain_ok;
    if (threadIdx.x < 64) {
      const bool good = chol_wave<RM>(gl, R, F);
      if (threadIdx.x == 0) plain_ok = good ? 1 : 0;
    }
    __syncthreads();
    if (plain_ok) {
      if (threadIdx.x == 0) *kind = 0;
    } else {
      factor_block<RM>(Gbar + (int64_t)fmode * RR, R, F, kind, flags, false);
    }
  }
}

// ---- normalisation ------------------------------------------------------------
// part[chunk * R + r] = sum over the chunk's rows of A(i, r)^2.  Thread t
// takes column t % R and rows t / R, t / R + G, ... (G = blockDim / R row
// groups, blockDim <= 256); the G group sums are added in group order.
__global__ __launch_bounds__(256) void colsq_partial_kernel(const double* __restrict__ u,
                                                            ModeTable t,
                                                            double* __restrict__ part) {
  __shared__ double sh[256];
  const int R = t.R;
  const int G = (int)blockDim.x / R;   // blockDim.x <= 256
  const int64_t ch = blockIdx.x;
  int k = 0;
  while (ch >= t.coff[k + 1]) ++k;
  const int64_t i_begin = (ch - t.coff[k]) * kRowsPerChunk;
  const int64_t i_end = min<int64_t>(t.dims[k], i_begin + kRowsPerChunk);
  const double* A = u + t.off[k] * R;
  const int r = threadIdx.x % R;
  const int grp = threadIdx.x / R;
  double s = 0.0;
  if (grp < G)
    for (int64_t i = i_begin + grp; i < i_end; i += G) s = fma(A[i * R + r], A[i * R + r], s);
  sh[threadIdx.x] = s;
  __syncthreads();
  if ((int)threadIdx.x < R) {
    double tot = 0.0;
    for (int q = 0; q < G; ++q) tot += sh[q * R + threadIdx.x];
    part[ch * R + threadIdx.x] = tot;
  }
}

// One block: nu, lambda, scales (N x R) and the stable descending order.
__global__ void norm_plan_kernel(const double* __restrict__ part, ModeTable t,
                                 double* __restrict__ scales, int* __restrict__ perm) {
  __shared__ double lam[kMaxR];
  __shared__ double nu[CP_MAX_ORDER][kMaxR];
  const int R = t.R;
  for (int r = threadIdx.x; r < R; r += blockDim.x) {
    double l = 1.0;
    for (int k = 0; k < t.N; ++k) {
      const double s = ordered_sum(part + t.coff[k] * R + r, t.coff[k + 1] - t.coff[k], R);
      nu[k][r] = sqrt(s);
      l *= nu[k][r];
    }
    lam[r] = l;
    const double root = pow(l, 1.0 / (double)t.N);
    for (int k = 0; k < t.N; ++k) scales[k * R + r] = l > 0.0 ? root / nu[k][r] : 0.0;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < R; r += blockDim.x) {
    int pos = 0;
    for (int q = 0; q < R; ++q)
      if (lam[q] > lam[r] || (lam[q] == lam[r] && q < r)) ++pos;
    perm[pos] = r;   // perm[new position] = old term index
  }
}

// In place, one lane per entry with whole rows inside a wave (64 / R rows
// per wave): lane (row, j) loads x(row, perm[j]) and that term's scale, then
// stores u(row, j) = scale * value, and for the gradient g(row, j) =
// value / scale (scale 0 -> undivided).  A row's loads are one wave
// instruction whose results every store waits for, so no lane overwrites an
// entry another lane of its row has still to read.
__global__ __launch_bounds__(256) void norm_apply_rows_kernel(double* __restrict__ u,
                                                              double* __restrict__ g, ModeTable t,
                                                              const double* __restrict__ scales,
                                                              const int* __restrict__ perm) {
  const int R = t.R;
  const int rpw = 64 / R;
  const int lane = (int)threadIdx.x & 63;
  const int sub = lane / R;
  const int j = lane - sub * R;
  const int64_t row = ((int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) * rpw + sub;
  if (sub >= rpw || row >= t.off[t.N]) return;
  int k = 0;
  while (row >= t.off[k + 1]) ++k;
  const int r = perm[j];
  const double sc = scales[k * R + r];
  const double vu = u[row * R + r];
  const double vg = g ? g[row * R + r] : 0.0;
  u[row * R + j] = sc * vu;
  if (g) g[row * R + j] = sc != 0.0 ? vg / sc : vg;
}

// ---- ALS mode solve: block factorisation in factor.hpp ---------------------------
template <int RM>
__global__ __launch_bounds__(256) void factor_kernel(const double* __restrict__ G, int R,
                                                     double* __restrict__ F,
                                                     int* __restrict__ kind,
                                                     int* __restrict__ flags) {
  factor_block<RM>(G, R, F, kind, flags, true);
}

// A(i,:) = M(i,:) Gammabar^-1 using the factor from factor_block.  One wave
// per row (grid-stride over rows), lane q holding component q (R <= 64):
// forward L y = m, then back L^T x = y, one component finished per step
// (broadcast from its lane with readlane, times the reciprocal pivot) and
// removed from the others by their lanes.
// RM <= 32: lane q holds row q and column q of L in registers (padded with
// zeros to RM), so a step reads no memory; the same operations in the same
// order.  The pseudo-inverse (kind 2) and RM = 64 read L from LDS.
template <int RM>
__global__ __launch_bounds__(256) void solve_rows_kernel(const double* __restrict__ M,
                                                         const double* __restrict__ F,
                                                         const int* __restrict__ kind, int64_t I,
                                                         int R, double* __restrict__ A) {
  if constexpr (RM <= 32) {
    if (*kind != 2) {
      const int q = threadIdx.x & 63;
      double lrow[RM], lcol[RM];
#pragma unroll
      for (int r = 0; r < RM; ++r) {
        lrow[r] = (q < R && r < R) ? F[q * R + r] : 0.0;
        lcol[r] = (q < R && r < R) ? F[r * R + q] : 0.0;
      }
      const double rd = q < R ? 1.0 / F[q * R + q] : 1.0;
      const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
      const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
      for (int64_t i = wave0; i < I; i += nwaves) {
        double y = q < R ? M[i * R + q] : 0.0;
#pragma unroll
        for (int r = 0; r < RM; ++r) {
          if (r < R) {
            const double yr = wave_bcast(y * rd, r);   // y_r / L(r, r) from lane r
            if (q == r) y = yr;
            else if (q > r && q < R) y -= lrow[r] * yr;
          }
        }
#pragma unroll
        for (int r = RM - 1; r >= 0; --r) {
          if (r < R) {
            const double xr = wave_bcast(y * rd, r);
            if (q == r) y = xr;
            else if (q < r) y -= lcol[r] * xr;
          }
        }
        if (q < R) A[i * R + q] = y;
      }
      return;
    }
  }
  __shared__ double f[kMaxR * kMaxR];
  __shared__ double rdiag[kMaxR];
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) f[e] = F[e];
  for (int r = threadIdx.x; r < R; r += blockDim.x) rdiag[r] = 1.0 / F[r * R + r];
  __syncthreads();
  const int q = threadIdx.x & 63;
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const bool pinv = *kind == 2;
  for (int64_t i = wave0; i < I; i += nwaves) {
    double y = q < R ? M[i * R + q] : 0.0;
    if (pinv) {
      double s = 0.0;
      for (int c = 0; c < R; ++c) {
        const double mc = __shfl(y, c);
        if (q < R) s = fma(mc, f[c * R + q], s);
      }
      if (q < R) A[i * R + q] = s;
      continue;
    }
    for (int r = 0; r < R; ++r) {
      const double yr = wave_bcast(y, r) * rdiag[r];
      if (q == r) y = yr;
      else if (q > r && q < R) y -= f[q * R + r] * yr;
    }
    for (int r = R - 1; r >= 0; --r) {
      const double xr = wave_bcast(y, r) * rdiag[r];
      if (q == r) y = xr;
      else if (q < r) y -= f[r * R + q] * xr;
    }
    if (q < R) A[i * R + q] = y;
  }
}

// G(i, r) = -M(i, r) + sum_s A(i, s) Gbar(s, r)
__global__ void grad_epilogue_kernel(const double* __restrict__ M, const double* __restrict__ A,
                                     const double* __restrict__ Gbar, int64_t I, int R,
                                     double* __restrict__ G) {
  __shared__ double gb[kMaxR * kMaxR];
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) gb[e] = Gbar[e];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= I * R) return;
  const int64_t i = e / R;
  const int r = (int)(e - i * R);
  double s = 0.0;
  for (int q = 0; q < R; ++q) s = fma(A[i * R + q], gb[q * R + r], s);
  G[e] = s - M[e];
}

// ---- fixed-order reductions ----------------------------------------------------
constexpr int kRedBlocks = 512;

__device__ double block_sum(double v) {
  __shared__ double sh[256];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

template <typename X, typename Y>
__global__ void dot_partial_kernel(const X* __restrict__ x, const Y* __restrict__ y, int64_t n,
                                   int64_t per, double* __restrict__ part) {
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = min<int64_t>(n, b0 + per);
  double s = 0.0;
  for (int64_t e = b0 + threadIdx.x; e < b1; e += blockDim.x)
    s = fma((double)x[e], (double)y[e], s);
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void sum_final_kernel(const double* __restrict__ part, int nb, double* __restrict__ out) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[b];
  s = block_sum(s);
  if (threadIdx.x == 0) *out = s;
}

// ---- one workgroup for short vectors ---------------------------------------------
// Iterate-length vectors (L = R sum_n I_n) are short: up to kSmallVec entries
// a dot product, the objective and the normalisation take one launch
// instead of two to four.  Thread t adds its entries t, t + 256, ... in
// order (loads 16 at a time), then the fixed-order block sum.
constexpr int64_t kSmallVec = 32768;
// The one-workgroup normalisation walks its rows tile by tile: shorter limit
// (at 16384 entries it took 50 us against about 30 for the multi-block form).
constexpr int64_t kSmallNorm = 8192;

template <typename X, typename Y>
__device__ double thread_dot(const X* __restrict__ x, const Y* __restrict__ y, int64_t n) {
  double s = 0.0;
  for (int64_t e0 = threadIdx.x; e0 < n; e0 += 16 * 256) {
    double xv[16], yv[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      const int64_t e = e0 + (int64_t)b * 256;
      xv[b] = e < n ? (double)x[e] : 0.0;
      yv[b] = e < n ? (double)y[e] : 0.0;
    }
#pragma unroll
    for (int b = 0; b < 16; ++b) s = fma(xv[b], yv[b], s);
  }
  return s;
}

template <typename X, typename Y>
__global__ __launch_bounds__(256) void dot_small_kernel(const X* __restrict__ x,
                                                        const Y* __restrict__ y, int64_t n,
                                                        double* __restrict__ out) {
  const double s = block_sum(thread_dot(x, y, n));
  if (threadIdx.x == 0) *out = s;
}

// f = 0.5 normsq - <A, M> + 0.5 sum(Gamma)
__global__ __launch_bounds__(256) void objective_small_kernel(const double* __restrict__ A,
                                                              const double* __restrict__ M,
                                                              int64_t n, double normsq,
                                                              const double* __restrict__ Gam,
                                                              int R, double* __restrict__ f) {
  const double d = block_sum(thread_dot(A, M, n));
  double sg = 0.0;
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) sg += Gam[e];
  sg = block_sum(sg);
  if (threadIdx.x == 0) *f = 0.5 * normsq - d + 0.5 * sg;
}

// Normalisation (Section 2.3 end; the same plan as norm_plan_kernel) of u and
// the gradient g at the same point, one workgroup: per mode the column norms
// nu (thread (group, r) adds rows group, group + G, ... in order, then the G
// groups in order), lambda_r = prod_n nu_r^(n), scales lambda^(1/N) / nu, the
// stable descending order of lambda, then every row rescaled and permuted in
// place through an LDS tile.
__global__ __launch_bounds__(256) void normalize_small_kernel(double* __restrict__ u,
                                                              double* __restrict__ g,
                                                              ModeTable t,
                                                              double* __restrict__ scales_out,
                                                              int* __restrict__ perm_out) {
  constexpr int kTile = 4096;
  __shared__ double nu[CP_MAX_ORDER][kMaxR];
  __shared__ double scl[CP_MAX_ORDER][kMaxR];
  __shared__ double lam[kMaxR];
  __shared__ int perm[kMaxR];
  __shared__ double red[256];
  __shared__ double tile[kTile];
  const int R = t.R;
  const int G = 256 / R;   // R <= 64
  const int c = threadIdx.x % R, grp = threadIdx.x / R;
  for (int k = 0; k < t.N; ++k) {
    const double* A = u + t.off[k] * R;
    const int64_t I = t.dims[k];
    double s = 0.0;
    if (grp < G) {
      for (int64_t i0 = grp; i0 < I; i0 += 8 * (int64_t)G) {
        double v[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const int64_t i = i0 + (int64_t)b * G;
          v[b] = i < I ? A[i * R + c] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < 8; ++b) s = fma(v[b], v[b], s);
      }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x < R) {
      double tot = 0.0;
      for (int q = 0; q < G; ++q) tot += red[q * R + threadIdx.x];
      nu[k][threadIdx.x] = sqrt(tot);
    }
    __syncthreads();
  }
  if ((int)threadIdx.x < R) {
    const int r = threadIdx.x;
    double l = 1.0;
    for (int k = 0; k < t.N; ++k) l *= nu[k][r];
    lam[r] = l;
    const double root = pow(l, 1.0 / (double)t.N);
    for (int k = 0; k < t.N; ++k) scl[k][r] = l > 0.0 ? root / nu[k][r] : 0.0;
  }
  __syncthreads();
  if ((int)threadIdx.x < R) {
    const int r = threadIdx.x;
    int pos = 0;
    for (int q = 0; q < R; ++q)
      if (lam[q] > lam[r] || (lam[q] == lam[r] && q < r)) ++pos;
    perm[pos] = r;   // perm[new position] = old term index
  }
  __syncthreads();
  if (scales_out && (int)threadIdx.x < R) {   // the plan, for callers that rescale other data
    const int r = threadIdx.x;
    for (int k = 0; k < t.N; ++k) scales_out[k * R + r] = scl[k][r];
    perm_out[r] = perm[r];
  }
  const int64_t rows = t.off[t.N];
  const int64_t tr = kTile / R;   // rows per tile
  constexpr int kPer = kTile / 256;   // tile entries per thread
  for (int pass = 0; pass < (g ? 2 : 1); ++pass) {
    double* x = pass == 0 ? u : g;
    for (int64_t r0 = 0; r0 < rows; r0 += tr) {
      const int64_t n = min<int64_t>(tr, rows - r0) * R;
      double v[kPer];   // every load of the tile in flight before the LDS stores
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int64_t e = threadIdx.x + (int64_t)q * 256;
        v[q] = e < n ? x[r0 * R + e] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < kPer; ++q) tile[threadIdx.x + q * 256] = v[q];
      __syncthreads();
      for (int64_t e = threadIdx.x; e < n; e += 256) {
        const int64_t lr = e / R;
        const int j = (int)(e - lr * R);
        const int64_t row = r0 + lr;
        int k = 0;
        while (row >= t.off[k + 1]) ++k;
        const int pj = perm[j];
        const double sc = scl[k][pj];
        const double v = tile[lr * R + pj];
        x[row * R + j] = pass ? (sc != 0.0 ? v / sc : v) : sc * v;
      }
      __syncthreads();
    }
  }
}

template <typename X, typename Y>
int dot_impl(cp_handle* h, const X* x, const Y* y, int64_t n, double* out, hipStream_t st) {
  if (n <= kSmallVec) {
    hipLaunchKernelGGL((dot_small_kernel<X, Y>), dim3(1), dim3(256), 0, st, x, y, n, out);
    CP_LAUNCH_CHECK(h);
    return CP_OK;
  }
  const int64_t per = std::max<int64_t>(256, ((n + kRedBlocks - 1) / kRedBlocks + 255) / 256 * 256);
  const int nb = (int)std::max<int64_t>(1, (n + per - 1) / per);
  CP_TRY(ensure(h, h->red, sizeof(double) * kRedBlocks, st));
  double* part = static_cast<double*>(h->red.ptr);
  hipLaunchKernelGGL((dot_partial_kernel<X, Y>), dim3(nb), dim3(256), 0, st, x, y, n, per, part);
  CP_LAUNCH_CHECK(h);
  hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(256), 0, st, part, nb, out);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}


// f = 0.5 normsq - (sum of the dot partials) + 0.5 sum(Gamma): the two sums
// in the same order as the two-launch form (dot partials summed by one block,
// then the Gamma entries).
__global__ void objective_final_kernel(const double* __restrict__ part, int nb, double normsq,
                                       const double* __restrict__ Gam, int R,
                                       double* __restrict__ f) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[b];
  const double d = block_sum(s);
  double sg = 0.0;
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) sg += Gam[e];
  sg = block_sum(sg);
  if (threadIdx.x == 0) *f = 0.5 * normsq - d + 0.5 * sg;
}

// Streaming-read reference: grid-stride 16-byte non-temporal loads, U in
// flight per thread, summed into one value per workgroup; 64 workgroups per
// CU (many short workgroups balance the end of the pass better than a few
// long ones; measured best of U in {4, 8, 16} and 8..64 workgroups per CU:
// 6.3 TB/s on 1 GiB, 6.9 TB/s on 4 GiB).
#ifndef CPNG_SR_UNROLL
#define CPNG_SR_UNROLL 8
#endif
#ifndef CPNG_SR_BPC
#define CPNG_SR_BPC 64
#endif
__global__ __launch_bounds__(256) void stream_read_kernel(const float4* __restrict__ x4, int64_t n,
                                                          double* __restrict__ out) {
  // 16-byte non-temporal loads (every component is used, so the loads stay
  // 16 bytes wide): each wave instruction reads 1 KB of whole lines
  typedef float f4v __attribute__((ext_vector_type(4)));
  const f4v* x = reinterpret_cast<const f4v*>(x4);
  constexpr int U = CPNG_SR_UNROLL;
  float s = 0.f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; e + (U - 1) * stride < n; e += U * stride) {
    f4v v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(x + e + u * stride);
#pragma unroll
    for (int u = 0; u < U; ++u) s += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  for (; e < n; e += stride) {
    const f4v v = __builtin_nontemporal_load(x + e);
    s += (v.x + v.y) + (v.z + v.w);
  }
  const double t = block_sum((double)s);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

__global__ void axpy_kernel(const double* __restrict__ x, double a, const double* __restrict__ d,
                            double* __restrict__ y, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = fma(a, d[e], x[e]);
}

// y = -x / s
__global__ void neg_div_kernel(const double* __restrict__ x, double s, double* __restrict__ y,
                               int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = -x[e] / s;
}

// d = -g + gamma d (d = -g exactly when gamma = 0)
__global__ void cg_direction_kernel(const double* __restrict__ g, double gamma,
                                    double* __restrict__ d, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) d[e] = gamma == 0.0 ? -g[e] : fma(gamma, d[e], -g[e]);
}

__global__ void sub_kernel(const double* __restrict__ a, const double* __restrict__ b,
                           double* __restrict__ y, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = a[e] - b[e];
}

// ---- N-GMRES Step II ----------------------------------------------------------
constexpr int kMaxWin = 64;
constexpr int kStepTile = 64;
struct WinDesc {
  const double* ubase;
  const double* gbase;
  int64_t L;
  int wcap;
};

__device__ inline const double* win_slot(const double* base, const WinDesc& w, int whead, int j) {
  return base + (int64_t)((whead + j) % w.wcap) * w.L;
}

__global__ void set_steppar_kernel(StepPar* p, double beta, int m, int whead) {
  p->beta = beta;
  p->m = m;
  p->whead = whead;
}

// y1 = x1 and y2 = x2 (n values each), one launch
__global__ void copy2_kernel(const double* __restrict__ x1, double* __restrict__ y1,
                             const double* __restrict__ x2, double* __restrict__ y2, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) {
    y1[e] = x1[e];
    y2[e] = x2[e];
  }
}

__global__ void axpy_par_kernel(const double* __restrict__ x, const StepPar* __restrict__ par,
                                const double* __restrict__ d, double* __restrict__ y, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = fma(par->beta, d[e], x[e]);
}

// Pair sums over a contiguous range of positions: for j <= k < m,
// B(j,k) = sum p_j p_k and rhs(j) = sum p_j gbar, with p_j = gbar - g_j.
// Partial slot layout: [pairs m(m+1)/2 in (j,k) row order][m rhs].
__global__ void step2_partial_kernel(WinDesc w, const StepPar* __restrict__ par,
                                     const double* __restrict__ gbar, int64_t L, int64_t per,
                                     double* __restrict__ part) {
  __shared__ double P[kMaxWin + 1][kStepTile];
  __shared__ const double* gp[kMaxWin];
  const int m = par->m;
  const int whead = par->whead;
  for (int j = threadIdx.x; j < m; j += blockDim.x) gp[j] = win_slot(w.gbase, w, whead, j);
  const int npairs = m * (m + 1) / 2;
  const int nval = npairs + m;
  double acc[9];
  int pj[9], pk[9];
  for (int q = 0; q < 9; ++q) {
    acc[q] = 0.0;
    const int v = threadIdx.x + q * blockDim.x;
    int j = 0, k = 0;
    if (v < npairs) {
      // invert v = (pairs of rows before j) + (k - j)
      int rem = v;
      while (rem >= m - j) {
        rem -= m - j;
        ++j;
      }
      k = j + rem;
    } else if (v < nval) {
      j = v - npairs;
      k = m;   // the gbar row
    }
    pj[q] = j;
    pk[q] = k;
  }
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = min<int64_t>(L, b0 + per);
  for (int64_t x0 = b0; x0 < b1; x0 += kStepTile) {
    const int nx = (int)min<int64_t>(kStepTile, b1 - x0);
    for (int e = threadIdx.x; e < (m + 1) * kStepTile; e += blockDim.x) {
      const int j = e / kStepTile, xx = e % kStepTile;
      double val = 0.0;
      if (xx < nx) {
        const double gb = gbar[x0 + xx];
        val = j < m ? gb - gp[j][x0 + xx] : gb;
      }
      P[j][xx] = val;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const int v = threadIdx.x + q * blockDim.x;
      if (v < nval) {
        const int j = pj[q], k = pk[q];
        double s = acc[q];
        for (int xx = 0; xx < nx; ++xx) s = fma(P[j][xx], P[k][xx], s);
        acc[q] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int v = threadIdx.x + q * blockDim.x;
    if (v < nval) part[(int64_t)blockIdx.x * nval + v] = acc[q];
  }
}

// One block: reduce partial slots in order, regularise, Cholesky-solve.
__global__ void step2_solve_kernel(const double* __restrict__ part, int nb,
                                   const StepPar* __restrict__ par, double eps,
                                   double* __restrict__ alpha_out, int* __restrict__ flags) {
  __shared__ double B[kMaxWin * kMaxWin];
  __shared__ double rhs[kMaxWin];
  __shared__ double ok;
  __shared__ double dmax;
  const int m = par->m;
  const int npairs = m * (m + 1) / 2;
  const int nval = npairs + m;
  for (int v = threadIdx.x; v < nval; v += blockDim.x) {
    const double s = ordered_sum(part + v, nb, nval);
    if (v < npairs) {
      int j = 0, rem = v;
      while (rem >= m - j) {
        rem -= m - j;
        ++j;
      }
      const int k = j + rem;
      B[j * m + k] = s;
      B[k * m + j] = s;
    } else {
      rhs[v - npairs] = -s;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double d = 0.0;
    for (int j = 0; j < m; ++j) d = fmax(d, B[j * m + j]);
    dmax = d;
  }
  __syncthreads();
  if (!(dmax > 0.0)) {
    for (int j = threadIdx.x; j < m; j += blockDim.x) alpha_out[j] = 0.0;
    return;
  }
  const double delta = eps * dmax;
  for (int j = threadIdx.x; j < m; j += blockDim.x) B[j * m + j] += delta;
  __syncthreads();
  if (!chol_lds(B, m, &ok)) {
    for (int j = threadIdx.x; j < m; j += blockDim.x) alpha_out[j] = 0.0;
    if (threadIdx.x == 0) *flags = *flags | 4;
    return;
  }
  // L y = rhs, then L^T alpha = y, by the first wave: after y(r) is known,
  // lane q > r removes its term; lane q holds row q (m <= 64).
  if (threadIdx.x < 64) {
    const int q = threadIdx.x;
    double* y = rhs;
    for (int r = 0; r < m; ++r) {
      const double yr = y[r] / B[r * m + r];
      __builtin_amdgcn_wave_barrier();
      if (q > r && q < m) y[q] -= B[q * m + r] * yr;
      if (q == r) y[q] = yr;
      __builtin_amdgcn_wave_barrier();
    }
    for (int r = m - 1; r >= 0; --r) {
      const double xr = y[r] / B[r * m + r];
      __builtin_amdgcn_wave_barrier();
      if (q < r) y[q] -= B[r * m + q] * xr;
      if (q == r) y[q] = xr;
      __builtin_amdgcn_wave_barrier();
    }
    if (q < m) alpha_out[q] = y[q];
  }
}

__global__ void step2_combine_kernel(WinDesc w, const StepPar* __restrict__ par,
                                     const double* __restrict__ ubar,
                                     const double* __restrict__ alpha, int64_t L,
                                     double* __restrict__ uhat) {
  __shared__ const double* up[kMaxWin];
  __shared__ double al[kMaxWin];
  const int m = par->m;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    up[j] = win_slot(w.ubase, w, par->whead, j);
    al[j] = alpha[j];
  }
  __syncthreads();
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= L) return;
  const double ub = ubar[x];
  double s = 0.0;
  for (int j = 0; j < m; ++j) s = fma(al[j], ub - up[j][x], s);
  uhat[x] = ub + s;
}

// ---- seeded uniform numbers -----------------------------------------------------
// Philox-4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC 2011): one round
// maps the counter block (c0, c1, c2, c3) under the key (k0, k1) to
// (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key
// advances by the Weyl constants before every round after the first.
__device__ inline void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// u[4b + q] = (x_q >> 11) 2^-53 for the cipher x of counter (b + 1, 0, 0, 0)
// under key (seed, 0): one thread per counter block.
__global__ void uniform_init_kernel(double* __restrict__ u, int64_t L, uint64_t seed) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b * 4 >= L) return;
  uint64_t c[4] = {(uint64_t)b + 1, 0, 0, 0};
  philox4x64_10(c, seed, 0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t e = b * 4 + q;
    if (e < L) u[e] = (double)(c[q] >> 11) * 0x1.0p-53;
  }
}

}  // namespace

// ---- host wrappers -----------------------------------------------------------------
static size_t small_layout(int N, int R) {
  // S, Gbar (N R R each), Gam (R R), scales (N R), perm (R ints), kind, alpha(64)
  return sizeof(double) * (size_t)(2 * N * R * R + R * R + N * R + kMaxWin + 8) +
         sizeof(int) * (size_t)(R + 8);
}

// Location of the mode-solve factor (R x R) and its kind in the small slice.
static int factor_slot(cp_handle* h, int R, double** F, int** kind, hipStream_t st) {
  CP_TRY(ensure(h, h->small, small_layout(CP_MAX_ORDER, R) + sizeof(double) * R * R + 4096, st));
  *F = static_cast<double*>(h->small.ptr) + small_layout(CP_MAX_ORDER, R) / sizeof(double);
  *kind = reinterpret_cast<int*>(*F + R * R);
  return CP_OK;
}

int gram_all(cp_handle* h, const Shape& s, const double* u, int R, double* S, double* Gbar,
             double* Gam, hipStream_t st, int factor_mode, int only_mode) {
  if (R > kMaxR) return fail(h, CP_EINVAL, "rank %d above the supported %d", R, kMaxR);
  if (!S) return fail(h, CP_EINVAL, "Gram without S");
  ModeTable t = table(s, R);
  const int64_t nch = t.coff[s.N];
  const int64_t ch0 = only_mode >= 0 ? t.coff[only_mode] : 0;
  const int64_t nrun = only_mode >= 0 ? t.coff[only_mode + 1] - ch0 : nch;
  double* F = nullptr;
  int* kind = nullptr;
  if (factor_mode >= 0) CP_TRY(factor_slot(h, R, &F, &kind, st));
  // one updated mode of at most 4 chunks at R <= 32: the final kernel forms
  // its Gram itself (no partial kernel)
  const bool direct = only_mode >= 0 && R <= 32 && nrun <= 4;
  double* part = nullptr;
  if (!direct) {
    CP_TRY(ensure(h, h->red, sizeof(double) * (size_t)(nch * R * R), st));
    part = static_cast<double*>(h->red.ptr);
    hipLaunchKernelGGL(gram_partial_kernel, dim3((unsigned)nrun), dim3(256), 0, st, u, t, ch0, part);
    CP_LAUNCH_CHECK(h);
  }
  const double* ud = direct ? u : nullptr;
  if (R <= 16)
    hipLaunchKernelGGL(gram_final_kernel<16>, dim3(1), dim3(256), 0, st, part, t, S, Gbar, Gam,
                       factor_mode, F, kind, h->flags, only_mode, ud);
  else if (R <= 32)
    hipLaunchKernelGGL(gram_final_kernel<32>, dim3(1), dim3(256), 0, st, part, t, S, Gbar, Gam,
                       factor_mode, F, kind, h->flags, only_mode, ud);
  else
    hipLaunchKernelGGL(gram_final_kernel<64>, dim3(1), dim3(256), 0, st, part, t, S, Gbar, Gam,
                       factor_mode, F, kind, h->flags, only_mode, ud);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

// With scales_out / perm_out the plan (scales[k R + r] of old term r in mode
// k, perm[new position] = old term) is left in the handle's small slice for
// the caller to apply to other data before its next call on this handle.
int normalize(cp_handle* h, const Shape& s, double* u, int R, double* g, hipStream_t st,
              const double** scales_out, const int** perm_out) {
  if (R < 1 || R > kMaxR) return fail(h, CP_EINVAL, "rank %d outside 1..%d", R, kMaxR);
  ModeTable t = table(s, R);
  if (s.sum_dims() * R <= kSmallNorm) {
    double* sc = nullptr;
    int* pm = nullptr;
    if (scales_out) {
      CP_TRY(ensure(h, h->small, small_layout(s.N, R) + 4096, st));
      sc = static_cast<double*>(h->small.ptr);
      pm = reinterpret_cast<int*>(sc + s.N * R);
      *scales_out = sc;
      *perm_out = pm;
    }
    hipLaunchKernelGGL(normalize_small_kernel, dim3(1), dim3(256), 0, st, u, g, t, sc, pm);
    CP_LAUNCH_CHECK(h);
    return CP_OK;
  }
  const int64_t nch = t.coff[s.N];
  CP_TRY(ensure(h, h->red, sizeof(double) * (size_t)(nch * R), st));
  CP_TRY(ensure(h, h->small, small_layout(s.N, R) + 4096, st));
  double* part = static_cast<double*>(h->red.ptr);
  double* scales = static_cast<double*>(h->small.ptr);
  int* perm = reinterpret_cast<int*>(scales + s.N * R);
  if (scales_out) {
    *scales_out = scales;
    *perm_out = perm;
  }
  hipLaunchKernelGGL(colsq_partial_kernel, dim3((unsigned)nch), dim3(256), 0, st, u, t, part);
  CP_LAUNCH_CHECK(h);
  hipLaunchKernelGGL(norm_plan_kernel, dim3(1), dim3(64), 0, st, part, t, scales, perm);
  CP_LAUNCH_CHECK(h);
  const int64_t rows = s.sum_dims();
  const int64_t rows_per_block = 4 * (64 / R);   // four waves of 64 / R rows (R <= 64)
  hipLaunchKernelGGL(norm_apply_rows_kernel, dim3(nblk(rows, rows_per_block)), dim3(256), 0, st, u,
                     g, t, scales, perm);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

int mode_solve(cp_handle* h, const double* M, const double* Gbar, int64_t I, int R, double* A,
               hipStream_t st) {
  if (R > kMaxR) return fail(h, CP_EINVAL, "rank %d above the supported %d", R, kMaxR);
  double* F = nullptr;
  int* kind = nullptr;
  CP_TRY(factor_slot(h, R, &F, &kind, st));
  if (Gbar) {   // else the factor was formed by gram_all(..., factor_mode)
    if (R <= 16)
      hipLaunchKernelGGL(factor_kernel<16>, dim3(1), dim3(256), 0, st, Gbar, R, F, kind, h->flags);
    else if (R <= 32)
      hipLaunchKernelGGL(factor_kernel<32>, dim3(1), dim3(256), 0, st, Gbar, R, F, kind, h->flags);
    else
      hipLaunchKernelGGL(factor_kernel<64>, dim3(1), dim3(256), 0, st, Gbar, R, F, kind, h->flags);
    CP_LAUNCH_CHECK(h);
  }
  if (I > 0) {
    const int64_t blocks = std::min<int64_t>((I + 3) / 4, 4096);   // 4 rows (waves) per block
    if (R <= 16)
      hipLaunchKernelGGL(solve_rows_kernel<16>, dim3((unsigned)blocks), dim3(256), 0, st, M, F, kind,
                         I, R, A);
    else if (R <= 32)
      hipLaunchKernelGGL(solve_rows_kernel<32>, dim3((unsigned)blocks), dim3(256), 0, st, M, F, kind,
                         I, R, A);
    else
      hipLaunchKernelGGL(solve_rows_kernel<64>, dim3((unsigned)blocks), dim3(256), 0, st, M, F, kind,
                         I, R, A);
  }
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

int grad_epilogue(cp_handle* h, const double* M, const double* A, const double* Gbar, int64_t I,
                  int R, double* G, hipStream_t st) {
  if (I * R == 0) return CP_OK;
  hipLaunchKernelGGL(grad_epilogue_kernel, dim3(nblk(I * R, 256)), dim3(256), 0, st, M, A, Gbar,
                     I, R, G);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

int stream_read(cp_handle* h, const void* buf, size_t bytes, hipStream_t st) {
  if (!buf || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(buf) % 16 != 0)
    return fail(h, CP_EINVAL, "stream_read needs a 16-byte aligned buffer of 16-byte multiples");
  int dev = 0, ncu = 0;
  CP_HIP(h, hipGetDevice(&dev));
  CP_HIP(h, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int nb = std::max(1, ncu) * CPNG_SR_BPC;
  CP_TRY(ensure(h, h->red, sizeof(double) * (size_t)nb, st));
  {
    KernelTimer timer(h, CP_KERNEL_STREAM_READ, st);
    CP_TIMED_LAUNCH(timer, stream_read_kernel, dim3(nb), dim3(256), 0, st,
                       static_cast<const float4*>(buf), (int64_t)(bytes / 16),
                       static_cast<double*>(h->red.ptr));
  }
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

int dot(cp_handle* h, const double* x, const double* y, int64_t n, double* out, hipStream_t st) {
  return dot_impl<double, double>(h, x, y, n, out, st);
}

int sumsq_tensor(cp_handle* h, const void* v, int dtype, int64_t n, double* out, hipStream_t st) {
  if (dtype == CP_F32)
    return dot_impl<float, float>(h, static_cast<const float*>(v), static_cast<const float*>(v), n,
                                  out, st);
  return dot_impl<double, double>(h, static_cast<const double*>(v), static_cast<const double*>(v),
                                  n, out, st);
}

int objective_from_dot(cp_handle* h, const double* A, const double* M, int64_t n, double normsq,
                       const double* Gam, int R, double* f, hipStream_t st) {
  if (n <= kSmallVec) {
    hipLaunchKernelGGL(objective_small_kernel, dim3(1), dim3(256), 0, st, A, M, n, normsq, Gam, R, f);
    CP_LAUNCH_CHECK(h);
    return CP_OK;
  }
  const int64_t per = std::max<int64_t>(256, ((n + kRedBlocks - 1) / kRedBlocks + 255) / 256 * 256);
  const int nb = (int)std::max<int64_t>(1, (n + per - 1) / per);
  CP_TRY(ensure(h, h->red, sizeof(double) * kRedBlocks, st));
  double* part = static_cast<double*>(h->red.ptr);
  hipLaunchKernelGGL((dot_partial_kernel<double, double>), dim3(nb), dim3(256), 0, st, A, M, n, per,
                     part);
  CP_LAUNCH_CHECK(h);
  hipLaunchKernelGGL(objective_final_kernel, dim3(1), dim3(256), 0, st, part, nb, normsq, Gam, R, f);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}


int axpy_to(cp_handle* h, const double* x, double a, const double* d, double* y, int64_t n,
            hipStream_t st) {
  if (n == 0) return CP_OK;
  hipLaunchKernelGGL(axpy_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, x, a, d, y, n);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

int copy2(cp_handle* h, const double* x1, double* y1, const double* x2, double* y2, int64_t n,
          hipStream_t st) {
  if (n == 0) return CP_OK;
  hipLaunchKernelGGL(copy2_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, x1, y1, x2, y2, n);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

int neg_div_to(cp_handle* h, const double* x, double s, double* y, int64_t n, hipStream_t st) {
  if (n == 0) return CP_OK;
  hipLaunchKernelGGL(neg_div_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, x, s, y, n);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

int cg_direction(cp_handle* h, const double* g, double gamma, double* d, int64_t n,
                 hipStream_t st) {
  hipLaunchKernelGGL(cg_direction_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, g, gamma, d, n);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

int sub_to(cp_handle* h, const double* a, const double* b, double* y, int64_t n, hipStream_t st) {
  if (n == 0) return CP_OK;
  hipLaunchKernelGGL(sub_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, a, b, y, n);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

int set_steppar(cp_handle* h, StepPar* p, double beta, int m, int whead, hipStream_t st) {
  hipLaunchKernelGGL(set_steppar_kernel, dim3(1), dim3(1), 0, st, p, beta, m, whead);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

int axpy_par(cp_handle* h, const double* x, const StepPar* par, const double* d, double* y,
             int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(axpy_par_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, x, par, d, y, n);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

int init_uniform(cp_handle* h, int64_t L, uint64_t seed, double* u, hipStream_t st) {
  if (L <= 0) return CP_OK;
  const int64_t nb4 = (L + 3) / 4;
  hipLaunchKernelGGL(uniform_init_kernel, dim3(nblk(nb4, 256)), dim3(256), 0, st, u, L, seed);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

int step2(cp_handle* h, int64_t L, const double* ubase, const double* gbase, int wcap,
          const StepPar* par, const double* ubar, const double* gbar, double eps, double* uhat,
          double* alpha, hipStream_t st) {
  if (wcap < 1 || wcap > kMaxWin) return fail(h, CP_EINVAL, "window size %d outside 1..%d", wcap, kMaxWin);
  const WinDesc w{ubase, gbase, L, wcap};
  const int nval_max = wcap * (wcap + 1) / 2 + wcap;
  const int64_t per = std::max<int64_t>(kStepTile, ((L + 255) / 256 + kStepTile - 1) / kStepTile * kStepTile);
  const int nb = (int)std::max<int64_t>(1, (L + per - 1) / per);
  CP_TRY(ensure(h, h->red, sizeof(double) * (size_t)nb * nval_max, st));
  double* part = static_cast<double*>(h->red.ptr);
  hipLaunchKernelGGL(step2_partial_kernel, dim3(nb), dim3(256), 0, st, w, par, gbar, L, per, part);
  CP_LAUNCH_CHECK(h);
  hipLaunchKernelGGL(step2_solve_kernel, dim3(1), dim3(256), 0, st, part, nb, par, eps, alpha,
                     h->flags);
  CP_LAUNCH_CHECK(h);
  hipLaunchKernelGGL(step2_combine_kernel, dim3(nblk(L, 256)), dim3(256), 0, st, w, par, ubar, alpha,
                     L, uhat);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

}  // namespace cpng
