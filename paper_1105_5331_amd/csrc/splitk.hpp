// Fixed-order reduction of split-K partial slots, shared by the dense MTTKRP
// kernels.  part holds nsplit slots of n values (slot-major).  Output e is
//     M(e) = sum over contiguous slot ranges, in range order, of the
//            in-order sum of that range,
// so the result depends only on nsplit and n, never on timing.  Up to 16
// slots, and up to 256 when there are at least 2^16 outputs, one thread per
// output adds all slots in order (256 consecutive outputs per block, 16
// slots' loads in flight at a time; a wave reads 256 contiguous bytes of a
// slot).  Otherwise up to 256 slots, a block covers 16 consecutive outputs
// with 16 threads per output; each thread issues its range's loads 8 at a
// time before adding.  Many slots go through a first stage over groups of
// 64 slots (see launch_splitk_reduce).
// With a pending gradient epilogue on the handle (M is an I x R MTTKRP) the
// same kernel also writes G(i, r) = -M(i, r) + sum_q A(i, q) Gbar(q, r), with
// the sum in q order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace cpng {
namespace {

constexpr int kSplitThreads = 256;

// OUT outputs per block, RANGES slot ranges per output (OUT * RANGES = 256).
template <typename PT, int OUT, int RANGES>
__global__ __launch_bounds__(kSplitThreads) void splitk_reduce_kernel(
    const PT* __restrict__ part, int64_t nsplit, int64_t n, double* __restrict__ M,
    const double* __restrict__ eA, const double* __restrict__ eGbar, double* __restrict__ eG,
    int eR) {
  static_assert(OUT * RANGES == kSplitThreads, "block shape");
  __shared__ double sh[RANGES][OUT + 1];
  const int tx = threadIdx.x % OUT;
  const int ty = threadIdx.x / OUT;
  const int64_t e = (int64_t)blockIdx.x * OUT + tx;
  const int64_t chunk = (nsplit + RANGES - 1) / RANGES;
  const int64_t s0 = ty * chunk;
  const int64_t s1 = min<int64_t>(nsplit, s0 + chunk);
  double s = 0.0;
  if (e < n) {
    for (int64_t q0 = s0; q0 < s1; q0 += 8) {
      PT v[8];
#pragma unroll
      for (int b = 0; b < 8; ++b) v[b] = q0 + b < s1 ? part[(q0 + b) * n + e] : PT(0);
#pragma unroll
      for (int b = 0; b < 8; ++b) s += (double)v[b];
    }
  }
  sh[ty][tx] = s;
  __syncthreads();
  if (ty == 0 && e < n) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < RANGES; ++q) t += sh[q][tx];
    M[e] = t;
    if (eG) {
      const int64_t i = e / eR;
      const int r = (int)(e - i * eR);
      double g = 0.0;
      for (int q = 0; q < eR; ++q) g = fma(eA[i * eR + q], eGbar[q * eR + r], g);
      eG[e] = g - t;
    }
  }
}

// Thread e adds slots 0..nsplit-1 of output e in order, 16 loads at a time.
// With the epilogue, Gbar (R x R) is staged in LDS (dynamic, R * R doubles).
template <typename PT>
__global__ __launch_bounds__(kSplitThreads) void splitk_flat_kernel(
    const PT* __restrict__ part, int nsplit, int64_t n, double* __restrict__ M,
    const double* __restrict__ eA, const double* __restrict__ eGbar, double* __restrict__ eG,
    int eR) {
  extern __shared__ double gsh[];
  const int64_t e = (int64_t)blockIdx.x * kSplitThreads + threadIdx.x;
  if (eG) {
    for (int t = threadIdx.x; t < eR * eR; t += kSplitThreads) gsh[t] = eGbar[t];
    __syncthreads();
  }
  if (e >= n) return;
  double t = 0.0;
  for (int q0 = 0; q0 < nsplit; q0 += 16) {
    PT v[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) v[b] = q0 + b < nsplit ? part[(int64_t)(q0 + b) * n + e] : PT(0);
#pragma unroll
    for (int b = 0; b < 16; ++b) t += (double)v[b];
  }
  M[e] = t;
  if (eG) {
    const int64_t i = e / eR;
    const int r = (int)(e - i * eR);
    const double* a = eA + i * eR;
    double g = 0.0;
    for (int q = 0; q < eR; ++q) g = fma(a[q], gsh[q * eR + r], g);
    eG[e] = g - t;
  }
}

// First stage for many slots: block (x, g) adds slots 64g .. 64g + 63 for the
// 64 outputs 64x .. 64x + 63 (a wave reads 64 consecutive outputs of one slot
// row), four quarter-ranges of 16 slots in order, into part2[g][e].
template <typename PT>
__global__ __launch_bounds__(kSplitThreads) void splitk_group_kernel(const PT* __restrict__ part,
                                                                     int64_t nsplit, int64_t n,
                                                                     double* __restrict__ part2) {
  __shared__ double sh[4][64];
  const int tx = threadIdx.x & 63;
  const int ty = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + tx;
  const int64_t q0 = (int64_t)blockIdx.y * 64 + ty * 16;
  const int64_t q1 = min<int64_t>(nsplit, q0 + 16);
  double s = 0.0;
  if (e < n) {
    PT v[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) v[b] = q0 + b < q1 ? part[(q0 + b) * n + e] : PT(0);
#pragma unroll
    for (int b = 0; b < 16; ++b) s += (double)v[b];
  }
  sh[ty][tx] = s;
  __syncthreads();
  if (ty == 0 && e < n) part2[(int64_t)blockIdx.y * n + e] = (sh[0][tx] + sh[1][tx]) + (sh[2][tx] + sh[3][tx]);
}

// Slots in MFMA fragment order (the two-sided kernel's partials): slot s
// holds nrows / 16 row tiles by 2 rank tiles of 16 x 16, tile t = 2 (row
// tile) + (rank tile) at t * 256, value q of lane l at 4 l + q, which is row
// 16 (row tile) + drow(l / 16, q) (4 (l / 16) + q, or l / 16 + 4 q for
// float64 MFMA results) and rank 16 (rank tile) + l % 16.  Thread e adds
// value e of every slot in slot order (16 loads in flight) and writes
// M(row, rank) for rank < R.
template <typename PT, bool F64ROWS>
__global__ __launch_bounds__(kSplitThreads) void splitk_frag_kernel(const PT* __restrict__ part,
                                                                    int nsplit, int64_t nfrag,
                                                                    int64_t nrows, int R,
                                                                    double* __restrict__ M) {
  const int64_t e = (int64_t)blockIdx.x * kSplitThreads + threadIdx.x;
  if (e >= nfrag) return;
  double t = 0.0;
  for (int q0 = 0; q0 < nsplit; q0 += 16) {
    PT v[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) v[b] = q0 + b < nsplit ? part[(int64_t)(q0 + b) * nfrag + e] : PT(0);
#pragma unroll
    for (int b = 0; b < 16; ++b) t += (double)v[b];
  }
  const int64_t tile = e >> 8;
  const int lane = (int)(e >> 2) & 63, q = (int)(e & 3), g = lane >> 4;
  const int64_t row = (tile >> 1) * 16 + (F64ROWS ? g + 4 * q : 4 * g + q);
  const int col = (int)(tile & 1) * 16 + (lane & 15);
  if (col < R && row < nrows) M[row * R + col] = t;
}

// nrows x R output from nsplit fragment-order slots of nrows x 32 values
template <typename PT>
inline int launch_splitk_frag(cp_handle* h, const PT* part, int64_t nsplit, int64_t nrows, int R,
                              bool f64rows, double* M, hipStream_t st) {
  (void)h;
  const int64_t nfrag = nrows * 32;
  const dim3 grid((unsigned)((nfrag + kSplitThreads - 1) / kSplitThreads));
  if (f64rows)
    hipLaunchKernelGGL((splitk_frag_kernel<PT, true>), grid, dim3(kSplitThreads), 0, st, part,
                       (int)nsplit, nfrag, nrows, R, M);
  else
    hipLaunchKernelGGL((splitk_frag_kernel<PT, false>), grid, dim3(kSplitThreads), 0, st, part,
                       (int)nsplit, nfrag, nrows, R, M);
  return CP_OK;
}

// R: columns of M (for the epilogue).  Up to 256 slots: one pass with 16
// ranges per output.  More: groups of 64 slots first (coalesced), then the
// group sums.  The shape depends only on nsplit and n, so the order of the
// additions is fixed for given sizes.
template <typename PT>
inline int launch_splitk_reduce(cp_handle* h, const PT* part, int64_t nsplit, int64_t n, int R,
                                double* M, hipStream_t st) {
  GradEpi& ep = h->epi;
  const bool epi = ep.G != nullptr && !ep.used;
  const double* eA = epi ? ep.A : nullptr;
  const double* eGb = epi ? ep.Gbar : nullptr;
  double* eG = epi ? ep.G : nullptr;
  if (nsplit <= 16 || (nsplit <= 256 && n >= (int64_t(1) << 16))) {
    const size_t lds = epi ? sizeof(double) * (size_t)R * R : 0;
    hipLaunchKernelGGL((splitk_flat_kernel<PT>), dim3((unsigned)((n + kSplitThreads - 1) / kSplitThreads)),
                       dim3(kSplitThreads), lds, st, part, (int)nsplit, n, M, eA, eGb, eG, R);
  } else if (nsplit <= 256) {
    hipLaunchKernelGGL((splitk_reduce_kernel<PT, 16, 16>), dim3((unsigned)((n + 15) / 16)),
                       dim3(kSplitThreads), 0, st, part, nsplit, n, M, eA, eGb, eG, R);
  } else {
    const int64_t groups = (nsplit + 63) / 64;
    CP_TRY(ensure(h, h->part2, sizeof(double) * (size_t)(groups * n), st));
    double* part2 = static_cast<double*>(h->part2.ptr);
    hipLaunchKernelGGL((splitk_group_kernel<PT>), dim3((unsigned)((n + 63) / 64), (unsigned)groups),
                       dim3(kSplitThreads), 0, st, part, nsplit, n, part2);
    hipLaunchKernelGGL((splitk_reduce_kernel<double, 16, 16>), dim3((unsigned)((n + 15) / 16)),
                       dim3(kSplitThreads), 0, st, part2, groups, n, M, eA, eGb, eG, R);
  }
  if (epi) ep.used = true;
  return CP_OK;
}

}  // namespace
}  // namespace cpng
