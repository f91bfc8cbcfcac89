// Fixed-order reduction of split-K partial slots, shared by the dense MTTKRP
// kernels.  part holds nsplit slots of n values (slot-major).  Output e is
//     M(e) = sum over 16 contiguous slot ranges, in range order, of the
//            in-order sum of that range,
// so the result depends only on nsplit and n, never on timing.  A block
// covers 16 outputs (16 x 8 B contiguous per slot row) with 16 threads per
// output; each thread issues its range's loads 8 at a time before adding.
// With a pending gradient epilogue on the handle (M is an I x R MTTKRP) the
// same kernel also writes G(i, r) = -M(i, r) + sum_q A(i, q) Gbar(q, r), with
// the sum in q order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace cpng {
namespace {

constexpr int kSplitOut = 16;     // outputs per block
constexpr int kSplitRanges = 16;  // slot ranges per output

template <typename PT>
__global__ __launch_bounds__(kSplitOut * kSplitRanges) void splitk_reduce_kernel(
    const PT* __restrict__ part, int64_t nsplit, int64_t n, double* __restrict__ M,
    const double* __restrict__ eA, const double* __restrict__ eGbar, double* __restrict__ eG,
    int eR) {
  __shared__ double sh[kSplitRanges][kSplitOut + 1];
  const int tx = threadIdx.x % kSplitOut;
  const int ty = threadIdx.x / kSplitOut;
  const int64_t e = (int64_t)blockIdx.x * kSplitOut + tx;
  const int64_t chunk = (nsplit + kSplitRanges - 1) / kSplitRanges;
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
    for (int q = 0; q < kSplitRanges; ++q) t += sh[q][tx];
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

// R: columns of M (for the epilogue).
template <typename PT>
inline void launch_splitk_reduce(cp_handle* h, const PT* part, int64_t nsplit, int64_t n, int R,
                                 double* M, hipStream_t st) {
  GradEpi& ep = h->epi;
  const bool epi = ep.G != nullptr && !ep.used;
  hipLaunchKernelGGL((splitk_reduce_kernel<PT>), dim3((unsigned)((n + kSplitOut - 1) / kSplitOut)),
                     dim3(kSplitOut * kSplitRanges), 0, st, part, nsplit, n, M,
                     epi ? ep.A : nullptr, epi ? ep.Gbar : nullptr, epi ? ep.G : nullptr, R);
  if (epi) ep.used = true;
}

}  // namespace
}  // namespace cpng
