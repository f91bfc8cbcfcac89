// Sparse (coordinate format) MTTKRP on gfx950 (Section 2.3, the product
// T_(n) Phibar^(n) restricted to the nonzeros):
//     M(i, r) = sum_{z : i_n(z) = i} v_z prod_{k != n} A^(k)(i_k(z), r).
//
// Preparation builds, for every mode n, a copy of the nonzeros stably sorted
// by i_n (other modes' coordinates and the values, structure of arrays) and
// the sorted row index of every nonzero (plus segment pointers).  The MTTKRP
// gives each wave a contiguous, equal-sized range of sorted nonzeros and
// works through it 64 nonzeros at a time.  Rows that lie strictly inside a
// wave's range are complete there and written directly; the first and the
// last row a wave meets may continue in a neighbouring wave and are written
// as two carry slots.  A fix-up kernel adds the carries of each row in slot
// order.  No atomics: the result is bitwise reproducible.
#include "common.hpp"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <type_traits>

namespace cpng {

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__global__ void bounds_kernel(const int32_t* __restrict__ coords, int64_t nnz, int N,
                              Shape s, int* __restrict__ bad) {
  const int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= nnz) return;
  for (int k = 0; k < N; ++k) {
    const int32_t c = coords[(int64_t)k * nnz + z];
    if (c < 0 || c >= s.dims[k]) bad[0] = 1;   // benign race: every writer stores 1
  }
}

__global__ void iota_kernel(int32_t* __restrict__ x, int64_t n) {
  const int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (z < n) x[z] = (int32_t)z;
}

__global__ void linear_key_kernel(const int32_t* __restrict__ coords, int64_t nnz, Shape s,
                                  uint64_t* __restrict__ key) {
  const int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= nnz) return;
  uint64_t k = 0;
  for (int m = 0; m < s.N; ++m) k = k * (uint64_t)s.dims[m] + (uint64_t)coords[(int64_t)m * nnz + z];
  key[z] = k;
}

__global__ void adjacent_equal_kernel(const uint64_t* __restrict__ key, int64_t n,
                                      int* __restrict__ dup) {
  const int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (z + 1 < n && key[z] == key[z + 1]) dup[0] = 1;
}

template <typename V>
__global__ void gather_kernel(const int32_t* __restrict__ coords, const V* __restrict__ vals,
                              const int32_t* __restrict__ perm, int64_t nnz, int N, int mode,
                              int32_t* __restrict__ out_coords, V* __restrict__ out_vals) {
  const int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= nnz) return;
  const int64_t src = perm[z];
  int kk = 0;
  for (int k = 0; k < N; ++k) {
    if (k == mode) continue;
    out_coords[(int64_t)kk * nnz + z] = coords[(int64_t)k * nnz + src];
    ++kk;
  }
  out_vals[z] = vals[src];
}

// seg[i] = number of sorted keys < i (lower bound), i = 0..I
__global__ void segment_kernel(const int32_t* __restrict__ keys, int64_t nnz, int64_t I,
                               int64_t* __restrict__ seg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > I) return;
  int64_t lo = 0, hi = nnz;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < i) lo = mid + 1;
    else hi = mid;
  }
  seg[i] = lo;
}

struct SparseParams {
  int N, mode, R, Rp;             // Rp: factor row stride (R padded)
  int64_t nnz, I_n;
  int64_t wave_nnz;               // sorted nonzeros per wave (multiple of 64)
  const int32_t* coords;          // (N-1) x nnz, other modes in increasing order
  const int64_t* seg;             // I_n + 1
  int64_t foff[CP_MAX_ORDER - 1]; // factor element offsets of the other modes
};

// Wave kernel: one wave per contiguous range of p.wave_nnz sorted nonzeros.
// The factors are read from a copy whose rows are padded to Rp = R rounded
// up to the vector width VW (4 floats or 2 doubles = 16 bytes), so a lane
// gathers VW consecutive ranks with one 16-byte load.  A wave is split into
// G = 64 / L groups of L lanes (L = Rp / VW rounded up to a power of two;
// lane c of a group holds ranks c*VW .. c*VW + VW - 1).  One step covers
// S = G * J consecutive nonzeros and group g takes J of them,
// g*J .. g*J + J - 1, in order.  The step's row indices, values and
// coordinates are loaded once, one nonzero per lane (coalesced), and handed
// to the groups by cross-lane shuffles; every gather of the step is issued
// before any product is formed.  A lane keeps one accumulator per rank it
// holds for the row being summed.  While a step continues that row, lanes
// just add; when the row changes the groups are combined (fixed butterfly
// order) and the finished row is written: directly if it lies strictly
// inside the wave's range, else into the wave's head or tail carry slot.
// KM is the number of other modes the kernel is compiled for: 2 (order 3),
// 3 (order 4) or CP_MAX_ORDER - 1 with a runtime bound (any order).
// Sorted nonzeros per wave: about CPNG_SP_WAVES waves per launch, each range
// a multiple of 64 between 512 and 4096 (longer ranges amortise a wave's
// first and last rows; fewer waves leave latency unhidden, and more than one
// round of resident waves leaves a tail: 20000^3, 2e7 nonzeros, R = 16 took
// 231 us with 4096 waves, 228 with 5120, 302 with 8192).
#ifndef CPNG_SP_WAVES
#define CPNG_SP_WAVES 5120   // one round at 5 of the 6 waves per SIMD the R <= 16 kernels allow
#endif
inline int64_t wave_range(int64_t nnz) {
  const int64_t r = ((nnz + CPNG_SP_WAVES - 1) / CPNG_SP_WAVES + 63) / 64 * 64;
  return std::min<int64_t>(4096, std::max<int64_t>(512, r));
}

template <typename CT>
struct VecOf;
template <>
struct VecOf<float> {
  static constexpr int n = 4;
  using type = float4;
};
template <>
struct VecOf<double> {
  static constexpr int n = 2;
  using type = double2;
};

template <typename CT, int VW>
__device__ inline void load_vec(const CT* __restrict__ p, CT (&x)[VW]) {
  const typename VecOf<CT>::type v = *reinterpret_cast<const typename VecOf<CT>::type*>(p);
  if constexpr (VW == 4) {
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
  } else {
    x[0] = v.x; x[1] = v.y;
  }
}

template <typename CT, int VW, int L>
__device__ inline void group_flush(CT (&acc)[VW], int R, int64_t row, int& nflush, bool final_,
                                   int lane, int64_t wid, double* __restrict__ M,
                                   int64_t* __restrict__ crow, double* __restrict__ cval) {
  CT x[VW];
#pragma unroll
  for (int v = 0; v < VW; ++v) {
    x[v] = acc[v];
#pragma unroll
    for (int m = L; m < 64; m <<= 1) x[v] += __shfl_xor(x[v], m);
    acc[v] = CT(0);
  }
  // lanes 0..L-1 (group 0) hold the totals of their ranks
  if (lane < L) {
#pragma unroll
    for (int v = 0; v < VW; ++v) {
      const int r = lane * VW + v;
      if (r >= R) break;
      if (nflush == 0) {
        cval[(2 * wid) * R + r] = (double)x[v];
        if (final_) cval[(2 * wid + 1) * R + r] = 0.0;
      } else if (final_) {
        cval[(2 * wid + 1) * R + r] = (double)x[v];
      } else {
        M[row * R + r] = (double)x[v];
      }
    }
    if (lane == 0 && (nflush == 0 || final_)) {
      if (nflush == 0) crow[2 * wid] = row;
      if (final_) crow[2 * wid + 1] = row;
    }
  }
  ++nflush;
}

template <typename TT, typename CT, int L, int KM>
__global__ __launch_bounds__(256) void sparse_wave_kernel(const TT* __restrict__ vals,
                                                          const int32_t* __restrict__ rows,
                                                          const CT* __restrict__ fac,
                                                          SparseParams p, double* __restrict__ M,
                                                          int64_t* __restrict__ crow,
                                                          double* __restrict__ cval) {
  constexpr int VW = VecOf<CT>::n;
  constexpr int G = 64 / L;
  constexpr int J = L < 8 ? L : 8;
  constexpr int S = G * J;
  const int lane = threadIdx.x & 63;
  const int g = lane / L;
  const int c = lane % L;
  const bool lane_ok = c * VW < p.Rp;
  const int cc = lane_ok ? c * VW : 0;   // idle lanes read a valid address
  const int km = KM < CP_MAX_ORDER - 1 ? KM : p.N - 1;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t z0 = wid * p.wave_nnz;
  if (z0 >= p.nnz) return;   // whole wave
  const int64_t z1 = min<int64_t>(p.nnz, z0 + p.wave_nnz);
  CT acc[VW];
#pragma unroll
  for (int v = 0; v < VW; ++v) acc[v] = CT(0);
  int64_t cur = rows[z0];
  int nflush = 0;
  for (int64_t zb = z0; zb < z1; zb += S) {
    const int nstep = (int)min<int64_t>(S, z1 - zb);
    // the step's metadata, one nonzero per lane
    const bool mine = lane < nstep;
    const int64_t zm = mine ? zb + lane : z0;
    const int32_t my_row = mine ? __builtin_nontemporal_load(rows + zm) : INT32_MAX;
    const CT my_val = mine ? (CT)__builtin_nontemporal_load(vals + zm) : CT(0);
    int32_t my_c[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k)
      my_c[k] = k < km ? __builtin_nontemporal_load(p.coords + (int64_t)k * p.nnz + zm) : 0;
    const int32_t last_row = __shfl(my_row, nstep - 1);
    // gathers of all J sub-steps, then the products
    int32_t rowj[J];
    CT contrib[J][VW];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int src = g * J + j;
      rowj[j] = __shfl(my_row, src);
      const CT vj = __shfl(my_val, src);
      CT prod[VW];
#pragma unroll
      for (int v = 0; v < VW; ++v) prod[v] = lane_ok ? vj : CT(0);
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (k < km) {
          const int32_t ck = __shfl(my_c[k], src);
          CT f[VW];
          load_vec<CT, VW>(fac + p.foff[k] + (int64_t)ck * p.Rp + cc, f);
#pragma unroll
          for (int v = 0; v < VW; ++v) prod[v] *= f[v];
        }
      }
#pragma unroll
      for (int v = 0; v < VW; ++v) contrib[j][v] = prod[v];
    }
    if (last_row == cur) {           // the whole step continues the current row
#pragma unroll
      for (int j = 0; j < J; ++j)
#pragma unroll
        for (int v = 0; v < VW; ++v) acc[v] += contrib[j][v];
      continue;
    }
    // rows change inside this step: finish each row in order
    for (;;) {
#pragma unroll
      for (int j = 0; j < J; ++j)
#pragma unroll
        for (int v = 0; v < VW; ++v) acc[v] += rowj[j] == cur ? contrib[j][v] : CT(0);
      if (cur == last_row) break;    // the last row may continue in the next step
      group_flush<CT, VW, L>(acc, p.R, cur, nflush, false, lane, wid, M, crow, cval);
      int32_t nxt = INT32_MAX;
#pragma unroll
      for (int j = 0; j < J; ++j) nxt = (rowj[j] > cur && rowj[j] < nxt) ? rowj[j] : nxt;
#pragma unroll
      for (int m = 1; m < 64; m <<= 1) nxt = min(nxt, __shfl_xor(nxt, m));
      cur = nxt;
    }
  }
  group_flush<CT, VW, L>(acc, p.R, cur, nflush, true, lane, wid, M, crow, cval);
}

// Measurement reference: the factor-row gathers of sparse_wave_kernel alone.
// The same waves, ranges, lane groups, coordinate stream (non-temporal, one
// nonzero per lane, handed out by shuffles) and 16-byte row loads; the rows of
// a nonzero are multiplied into a running per-lane product (so every load is
// used) instead of being weighted by the value and reduced by row.  Each wave
// writes one float.  What it measures is the rate at which these random
// factor-row reads can be served, the bound the MTTKRP cannot beat.
template <typename CT, int L, int KM>
__global__ __launch_bounds__(256) void sparse_gather_ref_kernel(const CT* __restrict__ fac,
                                                                SparseParams p,
                                                                float* __restrict__ out) {
  constexpr int VW = VecOf<CT>::n;
  constexpr int G = 64 / L;
  constexpr int J = L < 8 ? L : 8;
  constexpr int S = G * J;
  const int lane = threadIdx.x & 63;
  const int g = lane / L;
  const int c = lane % L;
  const bool lane_ok = c * VW < p.Rp;
  const int cc = lane_ok ? c * VW : 0;
  const int km = KM < CP_MAX_ORDER - 1 ? KM : p.N - 1;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t z0 = wid * p.wave_nnz;
  if (z0 >= p.nnz) return;
  const int64_t z1 = min<int64_t>(p.nnz, z0 + p.wave_nnz);
  CT acc = CT(0);
  for (int64_t zb = z0; zb < z1; zb += S) {
    const int nstep = (int)min<int64_t>(S, z1 - zb);
    const bool mine = lane < nstep;
    const int64_t zm = mine ? zb + lane : z0;
    int32_t my_c[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k)
      my_c[k] = k < km ? __builtin_nontemporal_load(p.coords + (int64_t)k * p.nnz + zm) : 0;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int src = g * J + j;
      CT prod[VW];
#pragma unroll
      for (int v = 0; v < VW; ++v) prod[v] = CT(1);
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (k < km) {
          const int32_t ck = __shfl(my_c[k], src);
          CT f[VW];
          load_vec<CT, VW>(fac + p.foff[k] + (int64_t)ck * p.Rp + cc, f);
#pragma unroll
          for (int v = 0; v < VW; ++v) prod[v] *= f[v];
        }
      }
#pragma unroll
      for (int v = 0; v < VW; ++v) acc += src < nstep ? prod[v] : CT(0);
    }
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) acc += __shfl_xor(acc, m);
  if (lane == 0) out[wid] = (float)acc;
}

template <typename CT, int L>
int launch_gather_ref(cp_handle* h, const CT* fac, const SparseParams& p, hipStream_t st) {
  const int64_t nwaves = (p.nnz + p.wave_nnz - 1) / p.wave_nnz;
  CP_TRY(ensure(h, h->carry, sizeof(float) * (size_t)std::max<int64_t>(1, nwaves), st));
  float* out = static_cast<float*>(h->carry.ptr);
  KernelTimer timer(h, CP_KERNEL_SPARSE_GATHER, st);
  if (p.N == 3)
    CP_TIMED_LAUNCH(timer, (sparse_gather_ref_kernel<CT, L, 2>), dim3(nblk(nwaves * 64, 256)), dim3(256), 0, st, fac, p, out);
  else if (p.N == 4)
    CP_TIMED_LAUNCH(timer, (sparse_gather_ref_kernel<CT, L, 3>), dim3(nblk(nwaves * 64, 256)), dim3(256), 0, st, fac, p, out);
  else
    CP_TIMED_LAUNCH(timer, (sparse_gather_ref_kernel<CT, L, CP_MAX_ORDER - 1>), dim3(nblk(nwaves * 64, 256)), dim3(256), 0, st, fac, p, out);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

// For each run of equal rows among the carry slots, the first slot of the run
// sums the run in slot order and writes the row.
__global__ void carry_fixup_kernel(const int64_t* __restrict__ carry_row,
                                   const double* __restrict__ carry_val, int64_t nslots, int R,
                                   double* __restrict__ M) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nslots * R) return;
  const int64_t s = e / R;
  const int r = (int)(e - s * R);
  const int64_t row = carry_row[s];
  if (s > 0 && carry_row[s - 1] == row) return;
  double sum = 0.0;
  for (int64_t q = s; q < nslots && carry_row[q] == row; ++q) sum += carry_val[q * R + r];
  M[row * R + r] = sum;
}

__global__ void zero_kernel(double* __restrict__ x, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] = 0.0;
}

// y(i, r) = x(i, r) for r < R, 0 for R <= r < Rp (rows padded to Rp)
template <typename CT>
__global__ void pad_factors_kernel(const double* __restrict__ x, int64_t rows, int R, int Rp,
                                   CT* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * Rp) return;
  const int64_t i = e / Rp;
  const int r = (int)(e - i * Rp);
  y[e] = r < R ? (CT)x[i * R + r] : CT(0);
}

template <typename TT, typename CT, int L, int KM>
int launch_sparse_wave(cp_handle* h, const TT* vals, const int32_t* rows, const CT* fac,
                       SparseParams p, double* M, hipStream_t st) {
  const int64_t nwaves = (p.nnz + p.wave_nnz - 1) / p.wave_nnz;
  const int64_t nslots = 2 * nwaves;
  CP_TRY(ensure(h, h->carry, (sizeof(int64_t) + sizeof(double) * p.R) * (size_t)std::max<int64_t>(1, nslots), st));
  int64_t* crow = static_cast<int64_t*>(h->carry.ptr);
  double* cval = reinterpret_cast<double*>(crow + nslots);
  {
    KernelTimer timer(h, CP_KERNEL_SPARSE_MTTKRP, st);
    CP_TIMED_LAUNCH(timer, (sparse_wave_kernel<TT, CT, L, KM>), dim3(nblk(nwaves * 64, 256)),
                       dim3(256), 0, st, vals, rows, fac, p, M, crow, cval);
  }
  CP_LAUNCH_CHECK(h);
  hipLaunchKernelGGL(carry_fixup_kernel, dim3(nblk(nslots * p.R, 256)), dim3(256), 0, st, crow,
                     cval, nslots, p.R, M);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

template <typename TT, typename CT, int L>
int dispatch_order(cp_handle* h, const TT* vals, const int32_t* rows, const CT* fac,
                   const SparseParams& p, double* M, hipStream_t st) {
  if (p.N == 3) return launch_sparse_wave<TT, CT, L, 2>(h, vals, rows, fac, p, M, st);
  if (p.N == 4) return launch_sparse_wave<TT, CT, L, 3>(h, vals, rows, fac, p, M, st);
  return launch_sparse_wave<TT, CT, L, CP_MAX_ORDER - 1>(h, vals, rows, fac, p, M, st);
}

template <typename TT, typename CT>
int dispatch_wave(cp_handle* h, const TT* vals, const int32_t* rows, const CT* fac,
                  const SparseParams& p, double* M, hipStream_t st) {
  const int lanes = p.Rp / VecOf<CT>::n;
  if (lanes <= 1) return dispatch_order<TT, CT, 1>(h, vals, rows, fac, p, M, st);
  if (lanes <= 2) return dispatch_order<TT, CT, 2>(h, vals, rows, fac, p, M, st);
  if (lanes <= 4) return dispatch_order<TT, CT, 4>(h, vals, rows, fac, p, M, st);
  if (lanes <= 8) return dispatch_order<TT, CT, 8>(h, vals, rows, fac, p, M, st);
  if (lanes <= 16) return dispatch_order<TT, CT, 16>(h, vals, rows, fac, p, M, st);
  if constexpr (VecOf<CT>::n == 2) {
    if (lanes <= 32) return dispatch_order<TT, CT, 32>(h, vals, rows, fac, p, M, st);
  }
  return fail(h, CP_EINVAL, "sparse MTTKRP supports R <= 64 (got %d)", p.R);
}

// The factors as CT with rows padded to Rp; the FP64 factors are used in
// place when no padding is needed.
template <typename CT>
int padded_factors(cp_handle* h, const double* u, int64_t rows, int R, int Rp, const CT** out,
                   hipStream_t st) {
  if constexpr (std::is_same<CT, double>::value) {
    if (Rp == R && reinterpret_cast<uintptr_t>(u) % 16 == 0) {
      *out = u;
      return CP_OK;
    }
  }
  CP_TRY(ensure(h, h->stage, sizeof(CT) * (size_t)(rows * Rp), st));
  CT* y = static_cast<CT*>(h->stage.ptr);
  if (rows > 0) {
    hipLaunchKernelGGL(pad_factors_kernel<CT>, dim3(nblk(rows * Rp, 256)), dim3(256), 0, st, u,
                       rows, R, Rp, y);
    CP_LAUNCH_CHECK(h);
  }
  *out = y;
  return CP_OK;
}

template <typename V>
int prepare_typed(cp_handle* h, cp_tensor* T, const Shape& s, hipStream_t st, SparsePrepared* sp) {
  const int64_t nnz = T->nnz;
  const int N = s.N;
  const int32_t* coords = T->coords;
  const V* vals = static_cast<const V*>(T->values);
  int32_t *keys_out = nullptr, *perm_in = nullptr, *perm_out = nullptr;
  void* temp = nullptr;
  size_t temp_bytes = 0;
  int rc = CP_OK;
  auto cleanup = [&]() {
    if (keys_out) (void)hipFree(keys_out);
    if (perm_in) (void)hipFree(perm_in);
    if (perm_out) (void)hipFree(perm_out);
    if (temp) (void)hipFree(temp);
  };
  if (hipMalloc(&keys_out, sizeof(int32_t) * nnz) != hipSuccess ||
      hipMalloc(&perm_in, sizeof(int32_t) * nnz) != hipSuccess ||
      hipMalloc(&perm_out, sizeof(int32_t) * nnz) != hipSuccess) {
    cleanup();
    return fail(h, CP_ENOMEM, "sparse prepare: allocation failed");
  }
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, coords, keys_out, perm_in, perm_out,
                                         (int)nnz, 0, 32, st) != hipSuccess) {
    cleanup();
    return fail(h, CP_EDEVICE, "sparse prepare: sort workspace query failed");
  }
  if (hipMalloc(&temp, temp_bytes + 16) != hipSuccess) {
    cleanup();
    return fail(h, CP_ENOMEM, "sparse prepare: sort workspace allocation failed");
  }
  for (int n = 0; n < N && rc == CP_OK; ++n) {
    SparseMode& md = sp->mode[n];
    if (hipMalloc(&md.coords, sizeof(int32_t) * std::max<int64_t>(1, (N - 1) * nnz)) != hipSuccess ||
        hipMalloc(&md.values, sizeof(V) * nnz) != hipSuccess ||
        hipMalloc(&md.seg, sizeof(int64_t) * (s.dims[n] + 1)) != hipSuccess ||
        hipMalloc(&md.rows, sizeof(int32_t) * nnz) != hipSuccess) {
      rc = fail(h, CP_ENOMEM, "sparse prepare: allocation failed");
      break;
    }
    hipLaunchKernelGGL(iota_kernel, dim3(nblk(nnz, 256)), dim3(256), 0, st, perm_in, nnz);
    int bits = 1;
    while (bits < 31 && (int64_t(1) << bits) < s.dims[n]) ++bits;
    size_t tb = temp_bytes;
    // stable LSD radix sort of (i_n, original position)
    if (hipcub::DeviceRadixSort::SortPairs(temp, tb, coords + (int64_t)n * nnz, keys_out, perm_in,
                                           perm_out, (int)nnz, 0, bits, st) != hipSuccess) {
      rc = fail(h, CP_EDEVICE, "sparse prepare: radix sort failed");
      break;
    }
    hipLaunchKernelGGL((gather_kernel<V>), dim3(nblk(nnz, 256)), dim3(256), 0, st, coords, vals,
                       perm_out, nnz, N, n, md.coords, static_cast<V*>(md.values));
    hipLaunchKernelGGL(segment_kernel, dim3(nblk(s.dims[n] + 1, 256)), dim3(256), 0, st, keys_out,
                       nnz, s.dims[n], md.seg);
    if (hipMemcpyAsync(md.rows, keys_out, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, st) !=
        hipSuccess)
      rc = fail(h, CP_EDEVICE, "sparse prepare: copy of the sorted indices failed");
    if (hipGetLastError() != hipSuccess) rc = fail(h, CP_EDEVICE, "sparse prepare: launch failed");
  }
  if (hipStreamSynchronize(st) != hipSuccess && rc == CP_OK)
    rc = fail(h, CP_EDEVICE, "sparse prepare: synchronisation failed");
  cleanup();
  return rc;
}

}  // namespace

int sparse_prepare(cp_handle* h, cp_tensor* T, const Shape& s, hipStream_t st) {
  const int64_t nnz = T->nnz;
  if (nnz < 0 || nnz > INT32_MAX - 1)
    return fail(h, CP_EINVAL, "nnz %lld outside 0..2^31-2", (long long)nnz);
  if (nnz > 0 && (!T->coords || !T->values))
    return fail(h, CP_EINVAL, "sparse tensor without coords/values");
  auto* sp = new SparsePrepared();
  sp->N = s.N;
  sp->nnz = nnz;
  sp->dtype = T->dtype;
  sp->stream = st;
  int rc = CP_OK;
  if (nnz > 0) {
    int* dflag = nullptr;
    uint64_t *key = nullptr, *key2 = nullptr;
    void* temp = nullptr;
    int flags[2] = {0, 0};
    // records the first failing HIP call; later steps are skipped
    auto ok = [&](hipError_t e, const char* what) {
      if (e != hipSuccess && rc == CP_OK)
        rc = fail(h, CP_EDEVICE, "sparse prepare: %s failed (%s)", what, hipGetErrorString(e));
      return rc == CP_OK;
    };
    if (hipMalloc(&dflag, 2 * sizeof(int)) != hipSuccess)
      rc = fail(h, CP_ENOMEM, "sparse prepare: allocation failed");
    if (rc == CP_OK && ok(hipMemsetAsync(dflag, 0, 2 * sizeof(int), st), "flag clear")) {
      hipLaunchKernelGGL(bounds_kernel, dim3(nblk(nnz, 256)), dim3(256), 0, st, T->coords, nnz,
                         s.N, s, dflag);
      // duplicate check on the full linear index when it fits in 64 bits
      double lim = 1.0;
      for (int k = 0; k < s.N; ++k) lim *= (double)s.dims[k];
      if (lim < 1.8e19) {
        size_t tb = 0;
        if (hipMalloc(&key, sizeof(uint64_t) * nnz) != hipSuccess ||
            hipMalloc(&key2, sizeof(uint64_t) * nnz) != hipSuccess) {
          rc = fail(h, CP_ENOMEM, "sparse prepare: duplicate-check allocation failed");
        } else if (ok(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, key, key2, (int)nnz, 0, 64, st),
                      "duplicate-check sort query")) {
          int bad = 0;
          if (hipMalloc(&temp, tb + 16) != hipSuccess) {
            rc = fail(h, CP_ENOMEM, "sparse prepare: duplicate-check workspace allocation failed");
          } else if (ok(hipStreamSynchronize(st), "synchronisation") &&
                     ok(hipMemcpy(&bad, dflag, sizeof(int), hipMemcpyDeviceToHost), "flag readback") &&
                     !bad) {   // keys are only meaningful with in-range coordinates
            hipLaunchKernelGGL(linear_key_kernel, dim3(nblk(nnz, 256)), dim3(256), 0, st, T->coords,
                               nnz, s, key);
            if (ok(hipcub::DeviceRadixSort::SortKeys(temp, tb, key, key2, (int)nnz, 0, 64, st),
                   "duplicate-check sort"))
              hipLaunchKernelGGL(adjacent_equal_kernel, dim3(nblk(nnz, 256)), dim3(256), 0, st, key2,
                                 nnz, dflag + 1);
          }
        }
      }
      if (ok(hipGetLastError(), "launch") && ok(hipStreamSynchronize(st), "synchronisation"))
        ok(hipMemcpy(flags, dflag, 2 * sizeof(int), hipMemcpyDeviceToHost), "flag readback");
    }
    if (key) (void)hipFree(key);
    if (key2) (void)hipFree(key2);
    if (temp) (void)hipFree(temp);
    if (dflag) (void)hipFree(dflag);
    if (rc == CP_OK && flags[0]) rc = fail(h, CP_EINVAL, "sparse tensor has a coordinate out of range");
    if (rc == CP_OK && flags[1]) rc = fail(h, CP_EDUPLICATE, "sparse tensor has repeated coordinates");
  }
  if (rc == CP_OK && nnz > 0) {
    if (T->dtype == CP_F32) rc = prepare_typed<float>(h, T, s, st, sp);
    else rc = prepare_typed<double>(h, T, s, st, sp);
  }
  if (rc == CP_OK && nnz == 0) {
    for (int n = 0; n < s.N; ++n) {
      SparseMode& md = sp->mode[n];
      if (hipMalloc(&md.seg, sizeof(int64_t) * (s.dims[n] + 1)) != hipSuccess) {
        rc = fail(h, CP_ENOMEM, "sparse prepare: allocation failed");
        break;
      }
      if (hipMemsetAsync(md.seg, 0, sizeof(int64_t) * (s.dims[n] + 1), st) != hipSuccess) {
        rc = fail(h, CP_EDEVICE, "sparse prepare: clearing the segment pointers failed");
        break;
      }
    }
    if (rc == CP_OK && hipStreamSynchronize(st) != hipSuccess)
      rc = fail(h, CP_EDEVICE, "sparse prepare: synchronisation failed");
  }
  T->prepared = sp;
  if (rc != CP_OK) {
    sparse_release(h, T);
  }
  return rc;
}

int sparse_release(cp_handle* h, cp_tensor* T) {
  auto* sp = static_cast<SparsePrepared*>(T->prepared);
  if (!sp) return CP_OK;
  // only the stream the tensor was prepared on (a serving slot's own): a
  // device-wide synchronisation would wait for every other slot's work
  (void)hipStreamSynchronize(sp->stream);
  for (int n = 0; n < sp->N; ++n) {
    if (sp->mode[n].coords) (void)hipFree(sp->mode[n].coords);
    if (sp->mode[n].values) (void)hipFree(sp->mode[n].values);
    if (sp->mode[n].seg) (void)hipFree(sp->mode[n].seg);
    if (sp->mode[n].rows) (void)hipFree(sp->mode[n].rows);
  }
  delete sp;
  T->prepared = nullptr;
  (void)h;
  return CP_OK;
}

namespace {
void set_offsets(const Shape& s, int mode, SparseParams& p) {
  int kk = 0;
  for (int k = 0; k < s.N; ++k)
    if (k != mode) p.foff[kk++] = s.off[k] * p.Rp;
}
}  // namespace

int sparse_mttkrp(cp_handle* h, const cp_tensor* T, const Shape& s, const double* u, int R,
                  int mode, int prec, double* M, hipStream_t st) {
  h->t_passes++;
  auto* sp = static_cast<const SparsePrepared*>(T->prepared);
  if (!sp) return fail(h, CP_EINVAL, "sparse tensor is not prepared (cp_tensor_prepare)");
  if (prec == CP_PREC_BF16X3) return fail(h, CP_EINVAL, "BF16X3 applies to dense tensors only");
  const int64_t I = s.dims[mode];
  hipLaunchKernelGGL(zero_kernel, dim3(nblk(I * R, 256)), dim3(256), 0, st, M, I * R);
  CP_LAUNCH_CHECK(h);
  if (sp->nnz == 0) return CP_OK;
  SparseParams p{};
  p.N = s.N;
  p.mode = mode;
  p.R = R;
  p.nnz = sp->nnz;
  p.wave_nnz = wave_range(sp->nnz);
  p.I_n = I;
  p.coords = sp->mode[mode].coords;
  p.seg = sp->mode[mode].seg;
  const void* vals = sp->mode[mode].values;
  const int32_t* rws = sp->mode[mode].rows;
  const int64_t frows = s.sum_dims();
  if (prec == CP_PREC_FP32) {
    if (sp->dtype != CP_F32) return fail(h, CP_EINVAL, "precision FP32 needs float32 values");
    p.Rp = (R + 3) / 4 * 4;
    set_offsets(s, mode, p);
    const float* fac = nullptr;
    CP_TRY(padded_factors<float>(h, u, frows, R, p.Rp, &fac, st));
    return dispatch_wave<float, float>(h, static_cast<const float*>(vals), rws, fac, p, M, st);
  }
  p.Rp = (R + 1) / 2 * 2;
  set_offsets(s, mode, p);
  const double* fac = nullptr;
  CP_TRY(padded_factors<double>(h, u, frows, R, p.Rp, &fac, st));
  if (sp->dtype == CP_F32)
    return dispatch_wave<float, double>(h, static_cast<const float*>(vals), rws, fac, p, M, st);
  return dispatch_wave<double, double>(h, static_cast<const double*>(vals), rws, fac, p, M, st);
}

// The gather reference of sparse_mttkrp(.., mode, CP_PREC_FP32, ..): the same
// padded float32 factor copy and wave layout, the gathers alone.
int sparse_gather_ref(cp_handle* h, const cp_tensor* T, const Shape& s, const double* u, int R,
                      int mode, hipStream_t st) {
  auto* sp = static_cast<const SparsePrepared*>(T->prepared);
  if (!sp) return fail(h, CP_EINVAL, "sparse tensor is not prepared (cp_tensor_prepare)");
  if (sp->nnz == 0) return CP_OK;
  SparseParams p{};
  p.N = s.N;
  p.mode = mode;
  p.R = R;
  p.nnz = sp->nnz;
  p.wave_nnz = wave_range(sp->nnz);
  p.I_n = s.dims[mode];
  p.coords = sp->mode[mode].coords;
  p.seg = sp->mode[mode].seg;
  p.Rp = (R + 3) / 4 * 4;
  set_offsets(s, mode, p);
  const float* fac = nullptr;
  CP_TRY(padded_factors<float>(h, u, s.sum_dims(), R, p.Rp, &fac, st));
  const int lanes = p.Rp / 4;
  if (lanes <= 1) return launch_gather_ref<float, 1>(h, fac, p, st);
  if (lanes <= 2) return launch_gather_ref<float, 2>(h, fac, p, st);
  if (lanes <= 4) return launch_gather_ref<float, 4>(h, fac, p, st);
  if (lanes <= 8) return launch_gather_ref<float, 8>(h, fac, p, st);
  return launch_gather_ref<float, 16>(h, fac, p, st);
}

}  // namespace cpng
