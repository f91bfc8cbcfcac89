// Factorisation of the symmetric R x R matrix Gammabar^(n) of the ALS mode
// solve (Section 2.3: A^(n) = M^(n) Gammabar^(n)^-1) by one workgroup, shared
// by the per-call kernels (small.hip) and the batched serving kernels
// (batch.hip): Cholesky by one wave in registers; if a pivot is not positive,
// Cholesky of Gammabar + 1e-14 tr/R I in LDS; if that fails too, the
// pseudo-inverse from a cyclic Jacobi eigendecomposition (eigenvalues below
// R eps max|w| dropped).
#pragma once

#include <hip/hip_runtime.h>

namespace cpng {
namespace {

constexpr int kMaxR = 64;

// ---- ALS mode solve -----------------------------------------------------------
// One block factorises Gammabar (R x R): Cholesky; if a pivot is not positive,
// Cholesky of Gammabar + 1e-14 tr/R I; if that fails too, the pseudo-inverse
// from a cyclic Jacobi eigendecomposition (eigenvalues below R eps max|w|
// dropped).  out: kind (0 chol, 1 shifted chol, 2 pinv) in *kind, the lower
// factor L or the pseudo-inverse P in F (R x R).
__device__ bool chol_lds(double* a, int R, double* piv_ok) {
  // right-looking Cholesky on a[R][R] in LDS, lower triangle
  for (int j = 0; j < R; ++j) {
    if (threadIdx.x == 0) {
      const double d = a[j * R + j];
      *piv_ok = (d > 0.0 && isfinite(d)) ? 1.0 : 0.0;
      a[j * R + j] = d > 0.0 ? sqrt(d) : d;
    }
    __syncthreads();
    if (*piv_ok == 0.0) return false;
    const double djj = a[j * R + j];
    for (int i = j + 1 + threadIdx.x; i < R; i += blockDim.x) a[i * R + j] /= djj;
    __syncthreads();
    const int n = R - j - 1;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int i = j + 1 + e / n, c = j + 1 + e % n;
      if (c <= i) a[i * R + c] -= a[i * R + j] * a[c * R + j];
    }
    __syncthreads();
  }
  return true;
}

// Value of v in lane `lane` (a constant), for the whole wave.
__device__ inline double wave_bcast(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, lane);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Cholesky of the symmetric R x R matrix G (R <= RM <= 64) by the first wave,
// in registers: lane c holds column c of the trailing matrix, both
// triangles, padded to RM x RM with the identity (so no step needs a bound
// test and the padding leaves the R x R factor unchanged).  Step j: the pivot
// d = a(j, j) from lane j; every lane forms its multiplier L(c, j) =
// a(j, c) / sqrt(d) (its own register j, since the trailing matrix is
// symmetric) and removes L(i, j) L(c, j) from a(i, c) for i > j, L(i, j)
// taken from lane i.  The same operations in the same order as the
// right-looking block factorisation (chol_lds), without barriers.  Lane c
// writes row c of L into F (zero above the diagonal).  Returns false at a
// pivot that is not positive and finite (the later steps still run, on
// values that are then discarded, and F is partly garbage).
template <int RM>
__device__ __forceinline__ bool chol_wave(const double* __restrict__ G, int R, double* __restrict__ F) {
  const int c = threadIdx.x & 63;
  double a[RM];
#pragma unroll
  for (int i = 0; i < RM; ++i) a[i] = (c < R && i < R) ? G[i * R + c] : (i == c ? 1.0 : 0.0);
  bool ok = true;   // uniform across the wave
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    const double d = wave_bcast(a[j], j);
    ok = ok && d > 0.0 && isfinite(d);
    const double djj = sqrt(d);
    const double m = a[j] / djj;   // L(c, j) for c > j
    if (j < R && c < R) F[c * R + j] = c > j ? m : (c == j ? djj : 0.0);
#pragma unroll
    for (int i = j + 1; i < RM; ++i) a[i] -= wave_bcast(m, i) * m;
  }
  return ok;
}

// try_plain: start with the one-wave factorisation (callers that already
// tried it pass false).  RM: R rounded up to 16, 32 or 64.
template <int RM>
__device__ __attribute__((noinline)) void factor_block(const double* __restrict__ G, int R,
                                                      double* __restrict__ F,
                                                      int* __restrict__ kind,
                                                      int* __restrict__ flags, bool try_plain) {
  __shared__ double a[RM * RM];   // R x R, R <= RM
  __shared__ double v[RM * RM];
  __shared__ double ok;
  __shared__ double shift;
  __shared__ int plain_ok;
  // plain Cholesky by the first wave
  if (threadIdx.x < 64) {
    const bool good = try_plain && chol_wave<RM>(G, R, F);
    if (threadIdx.x == 0) plain_ok = good ? 1 : 0;
  }
  __syncthreads();
  if (plain_ok) {
    if (threadIdx.x == 0) *kind = 0;
    return;
  }
  int k = 0;
  bool good = false;
  {
    if (threadIdx.x == 0) {
      double tr = 0.0;
      for (int i = 0; i < R; ++i) tr += G[i * R + i];
      shift = 1e-14 * tr / R;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < R * R; e += blockDim.x)
      a[e] = G[e] + ((e / R) == (e % R) ? shift : 0.0);
    __syncthreads();
    k = 1;
    good = chol_lds(a, R, &ok);
  }
  if (good) {
    for (int e = threadIdx.x; e < R * R; e += blockDim.x)
      F[e] = ((e % R) <= (e / R)) ? a[e] : 0.0;
    if (threadIdx.x == 0) {
      *kind = k;
      if (k > *flags) *flags = k;   // single-block kernel: plain store, stream-ordered
    }
    return;
  }
  // cyclic Jacobi: a <- G, v <- I; rotate until off-diagonal mass is negligible
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    a[e] = G[e];
    v[e] = ((e / R) == (e % R)) ? 1.0 : 0.0;
  }
  __syncthreads();
  __shared__ double cs[2];
  for (int sweep = 0; sweep < 60; ++sweep) {
    __shared__ double off;
    if (threadIdx.x == 0) {
      double o = 0.0, d = 0.0;
      for (int i = 0; i < R; ++i)
        for (int j = 0; j < R; ++j) (i == j ? d : o) += a[i * R + j] * a[i * R + j];
      off = (o <= 1e-30 * d || o == 0.0) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (off != 0.0) break;
    for (int p = 0; p < R - 1; ++p) {
      for (int q = p + 1; q < R; ++q) {
        if (threadIdx.x == 0) {
          const double apq = a[p * R + q];
          double c = 1.0, s = 0.0;
          if (apq != 0.0) {
            const double tau = (a[q * R + q] - a[p * R + p]) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
          cs[0] = c;
          cs[1] = s;
        }
        __syncthreads();
        const double c = cs[0], s = cs[1];
        if (s != 0.0) {
          // columns p, q
          for (int i = threadIdx.x; i < R; i += blockDim.x) {
            const double aip = a[i * R + p], aiq = a[i * R + q];
            a[i * R + p] = c * aip - s * aiq;
            a[i * R + q] = s * aip + c * aiq;
            const double vip = v[i * R + p], viq = v[i * R + q];
            v[i * R + p] = c * vip - s * viq;
            v[i * R + q] = s * vip + c * viq;
          }
          __syncthreads();
          // rows p, q
          for (int i = threadIdx.x; i < R; i += blockDim.x) {
            const double api = a[p * R + i], aqi = a[q * R + i];
            a[p * R + i] = c * api - s * aqi;
            a[q * R + i] = s * api + c * aqi;
          }
        }
        __syncthreads();
      }
    }
  }
  __shared__ double wmax;
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int i = 0; i < R; ++i) m = fmax(m, fabs(a[i * R + i]));
    wmax = m;
  }
  __syncthreads();
  const double tol = R * 2.220446049250313e-16 * fmax(wmax, 1e-300);
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    const int i = e / R, j = e % R;
    double s = 0.0;
    for (int q = 0; q < R; ++q) {
      const double w = a[q * R + q];
      if (fabs(w) > tol) s += v[i * R + q] * v[j * R + q] / w;
    }
    F[e] = s;
  }
  if (threadIdx.x == 0) {
    *kind = 2;
    if (2 > *flags) *flags = 2;
  }
}

}  // namespace
}  // namespace cpng
