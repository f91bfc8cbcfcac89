// Batched N-GMRES for small dense decomposition requests: the serving loop's
// persistent batched launches.
//
// A batch holds small dense requests (float32 tensor of order 3 or 4, at most
// CP_BATCH_MAX_ELEMS entries, R <= 32), each decomposed by N-GMRES with ALS as
// the one-step process (Section 2.1, algorithm box; Section 2.3), in float64
// arithmetic on the float32 values (the CP_PREC_FP32IN_FP64ACC arithmetic).
// Every tick is ONE kernel launch over all active requests: workgroup b runs
// request b's next device phase from start to end by itself --
//   START   normalise u_0, f and g at u_0, start the window;
//   STEP12  Step I (one ALS sweep, normalised) and Step II (f, g at u_bar,
//           the window's normal equations, u_hat normalised, d, the slope);
//   TRIAL   one line-search trial: u_t = u_bar + beta d, f, g and g^T d;
//   FINAL   the accepted iterate, normalised with its gradient, ||g||^2 and
//           the window push --
// with every sum in a fixed order, so a request's results depend only on its
// own data: the same bits alone or in any mix.  Between ticks the host reads
// every request's scalars back at once and advances each request's own
// control (restart test, Moré–Thuente search, window, stopping test).
#include "common.hpp"
#include "factor.hpp"
#include "linesearch.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

namespace cpng {

namespace {

constexpr int kBT = 256;
constexpr int kBatchMaxR = 32;
constexpr int kBatchMaxOrder = 4;
// the Gram of the window's differences and g_bar has (w + 1)(w + 2) / 2
// pairs, one per thread
constexpr int kBatchMaxWindow = 21;
static_assert((kBatchMaxWindow + 1) * (kBatchMaxWindow + 2) / 2 <= kBT, "one pair per thread");

enum BPhase { BP_START = 0, BP_STEP12 = 1, BP_TRIAL = 2, BP_FINAL = 3 };

// Device descriptor of one request for one tick.
struct BReq {
  const float* T;
  int N, R;
  int64_t dims[kBatchMaxOrder];
  int64_t off[kBatchMaxOrder + 1];   // factor row offsets (multiply by R)
  int64_t L;
  double normsq;
  double *u, *g, *ubar, *gbar, *uhat, *d, *ut, *gt, *gbest, *winU, *winG;
  double *M, *S, *Gb, *F;           // M: L doubles; S, Gb: N x R x R; F: R x R
  int wcap;
  int phase;
  int m, whead;      // STEP12: window entries and the oldest slot
  int push;          // START, FINAL: window slot written
  double beta;       // TRIAL: the step; FINAL: the accepted step
  int keep_best;     // TRIAL: copy g_t to g_best first (the previous trial is the best so far)
  int accept;        // FINAL: 0 u_bar, 1 the last trial's point, 2 u_bar + beta d with g_best
  double eps;
  int normalize_accel;
};

__device__ inline void wg_sync() { __syncthreads(); }

// Fixed-order sum over the workgroup: a butterfly inside each wave, then the
// four wave sums (0 + 1) + (2 + 3).  Every thread gets the result.
__device__ double wg_sum(double v) {
  __shared__ double part[kBT / 64];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  wg_sync();
  const double r = (part[0] + part[1]) + (part[2] + part[3]);
  wg_sync();
  return r;
}

__device__ double wg_dot(const double* __restrict__ x, const double* __restrict__ y, int64_t n) {
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += kBT) s = fma(x[e], y[e], s);
  return wg_sum(s);
}

__device__ void wg_copy(const double* __restrict__ x, double* __restrict__ y, int64_t n) {
  for (int64_t e = threadIdx.x; e < n; e += kBT) y[e] = x[e];
  wg_sync();
}

// S^(k) = A^(k)^T A^(k) (row order), for mode `only` or for all modes (-1)
__device__ void wg_grams(const BReq& q, const double* __restrict__ u, int only) {
  const int R = q.R, RR = R * R;
  const int k0 = only < 0 ? 0 : only, k1 = only < 0 ? q.N : only + 1;
  for (int e = threadIdx.x; e < (k1 - k0) * RR; e += kBT) {
    const int k = k0 + e / RR, rq = e % RR, r = rq / R, c = rq % R;
    const double* A = u + q.off[k] * R;
    const int64_t I = q.dims[k];
    double s = 0.0;
    for (int64_t i0 = 0; i0 < I; i0 += 8) {   // 8 loads in flight, row order kept
      double x[8], y[8];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool ok = i0 + b < I;
        x[b] = ok ? A[(i0 + b) * R + r] : 0.0;
        y[b] = ok ? A[(i0 + b) * R + c] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < 8; ++b)
        if (i0 + b < I) s = fma(x[b], y[b], s);
    }
    q.S[k * RR + rq] = s;
  }
  wg_sync();
}

// Gammabar^(n) = Hadamard product of S^(k) over k != n (mode order); all n
__device__ void wg_gammabars(const BReq& q) {
  const int RR = q.R * q.R;
  for (int e = threadIdx.x; e < q.N * RR; e += kBT) {
    const int n = e / RR, rq = e % RR;
    double p = 1.0;
    for (int k = 0; k < q.N; ++k)
      if (k != n) p *= q.S[k * RR + rq];
    q.Gb[n * RR + rq] = p;
  }
  wg_sync();
}

// M^(n)(i, r) = sum over the other indices (C order) of T(...) prod_{k != n}
// A^(k)(i_k, r): the innermost other mode summed first and scaled by the
// product of the outer modes' values.  Output entries go to threads; when
// there are fewer than 256 of them, G groups of threads split the outermost
// other mode (group g takes its indices g, g + G, ...) and the G partial sums
// are added in group order.
__device__ void wg_mttkrp(const BReq& q, const double* __restrict__ u, int n,
                          double* __restrict__ Mn) {
  __shared__ double gpart[kBT];
  const int R = q.R, N = q.N;
  int64_t stride[kBatchMaxOrder];
  stride[N - 1] = 1;
  for (int k = N - 2; k >= 0; --k) stride[k] = stride[k + 1] * q.dims[k + 1];
  int om[kBatchMaxOrder - 1];
  int no = 0;
  for (int k = 0; k < N; ++k)
    if (k != n) om[no++] = k;
  const int kc = om[no - 1];                 // innermost other mode
  const int64_t Ic = q.dims[kc], sc = stride[kc];
  const double* Ac = u + q.off[kc] * R;
  const int ka = om[0], kb = no == 3 ? om[1] : -1;
  const int64_t Ia = q.dims[ka], sa = stride[ka];
  const int64_t Ib = kb >= 0 ? q.dims[kb] : 1, sb = kb >= 0 ? stride[kb] : 0;
  const double* Aa = u + q.off[ka] * R;
  const double* Ab = kb >= 0 ? u + q.off[kb] * R : nullptr;
  const int64_t In = q.dims[n];
  const int64_t ne = In * R;
  const int G = (int)std::max<int64_t>(1, std::min<int64_t>(kBT / std::max<int64_t>(1, ne), Ia));
  const int grp = G > 1 ? (int)(threadIdx.x / ne) : 0;
  const int64_t e0 = G > 1 ? (int64_t)threadIdx.x - grp * ne : threadIdx.x;
  for (int64_t e = e0; e < ne && grp < G; e += G > 1 ? ne : kBT) {
    const int64_t i = e / R;
    const int r = (int)(e - i * R);
    const float* Ti = q.T + i * stride[n];
    double acc = 0.0;
    for (int64_t ia = grp; ia < Ia; ia += G) {
      const double pa = Aa[ia * R + r];
      for (int64_t ib = 0; ib < Ib; ++ib) {
        const double p = kb >= 0 ? pa * Ab[ib * R + r] : pa;
        const float* Tab = Ti + ia * sa + ib * sb;
        double s = 0.0;
        // the loads of 8 terms go out together; the sum keeps ic order
        for (int64_t i0 = 0; i0 < Ic; i0 += 8) {
          float tv[8];
          double av[8];
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            const bool ok = i0 + b < Ic;
            tv[b] = ok ? Tab[(i0 + b) * sc] : 0.f;
            av[b] = ok ? Ac[(i0 + b) * R + r] : 0.0;
          }
#pragma unroll
          for (int b = 0; b < 8; ++b)
            if (i0 + b < Ic) s = fma((double)tv[b], av[b], s);
        }
        acc = fma(p, s, acc);
      }
    }
    if (G > 1) gpart[threadIdx.x] = acc;
    else Mn[e] = acc;
  }
  if (G > 1) {
    wg_sync();
    for (int64_t e = threadIdx.x; e < ne; e += kBT) {
      double s = gpart[e];
      for (int g = 1; g < G; ++g) s += gpart[g * ne + e];
      Mn[e] = s;
    }
  }
  wg_sync();
}

// A(i,:) = M(i,:) Gammabar^-1 from the factor in q.F (kind 0, 1: the Cholesky
// factor L, forward then back substitution with reciprocal pivots, column by
// column; kind 2: the pseudo-inverse), one row per thread.
__device__ void wg_solve_rows(const BReq& q, const double* __restrict__ M, int64_t I, int kind,
                              double* __restrict__ A) {
  const int R = q.R;
  const double* F = q.F;
  for (int64_t i = threadIdx.x; i < I; i += kBT) {
    double y[kBatchMaxR];
#pragma unroll
    for (int c = 0; c < kBatchMaxR; ++c) y[c] = c < R ? M[i * R + c] : 0.0;
    if (kind == 2) {
      double x[kBatchMaxR];
#pragma unroll
      for (int c = 0; c < kBatchMaxR; ++c) {
        double s = 0.0;
        if (c < R) {
#pragma unroll
          for (int j = 0; j < kBatchMaxR; ++j)
            if (j < R) s = fma(y[j], F[j * R + c], s);
        }
        x[c] = s;
      }
#pragma unroll
      for (int c = 0; c < kBatchMaxR; ++c)
        if (c < R) A[i * R + c] = x[c];
      continue;
    }
#pragma unroll
    for (int r = 0; r < kBatchMaxR; ++r) {
      if (r < R) {
        y[r] = y[r] * (1.0 / F[r * R + r]);
#pragma unroll
        for (int c = 0; c < kBatchMaxR; ++c)
          if (c > r && c < R) y[c] -= F[c * R + r] * y[r];
      }
    }
#pragma unroll
    for (int r = kBatchMaxR - 1; r >= 0; --r) {
      if (r < R) {
        y[r] = y[r] * (1.0 / F[r * R + r]);
#pragma unroll
        for (int c = 0; c < kBatchMaxR; ++c)
          if (c < r) y[c] -= F[r * R + c] * y[r];
      }
    }
#pragma unroll
    for (int c = 0; c < kBatchMaxR; ++c)
      if (c < R) A[i * R + c] = y[c];
  }
  wg_sync();
}

// Normalise and reorder the rank-one terms of u in place (Section 2.3, end):
// column norms nu, lambda_r = prod_k nu_r^(k), scale lambda_r^(1/N) / nu_r^(k)
// (0 for a zero term), stable descending order of lambda; g (nullable) is
// mapped to the new point (column divided by its scale, undivided for a
// zero term, then permuted).
__device__ void wg_normalize(const BReq& q, double* __restrict__ u, double* __restrict__ g) {
  __shared__ double nu[kBatchMaxOrder][kBatchMaxR];
  __shared__ double scl[kBatchMaxOrder][kBatchMaxR];
  __shared__ double lam[kBatchMaxR];
  __shared__ int perm[kBatchMaxR];
  const int R = q.R, N = q.N;
  for (int e = threadIdx.x; e < N * R; e += kBT) {
    const int k = e / R, r = e % R;
    const double* A = u + q.off[k] * R;
    const int64_t I = q.dims[k];
    double s = 0.0;
    for (int64_t i0 = 0; i0 < I; i0 += 8) {
      double x[8];
#pragma unroll
      for (int b = 0; b < 8; ++b) x[b] = i0 + b < I ? A[(i0 + b) * R + r] : 0.0;
#pragma unroll
      for (int b = 0; b < 8; ++b)
        if (i0 + b < I) s = fma(x[b], x[b], s);
    }
    nu[k][r] = sqrt(s);
  }
  wg_sync();
  if ((int)threadIdx.x < R) {
    const int r = threadIdx.x;
    double l = 1.0;
    for (int k = 0; k < N; ++k) l *= nu[k][r];
    lam[r] = l;
    const double root = pow(l, 1.0 / (double)N);
    for (int k = 0; k < N; ++k) scl[k][r] = l > 0.0 ? root / nu[k][r] : 0.0;
  }
  wg_sync();
  if ((int)threadIdx.x < R) {
    const int r = threadIdx.x;
    int pos = 0;
    for (int c = 0; c < R; ++c)
      if (lam[c] > lam[r] || (lam[c] == lam[r] && c < r)) ++pos;
    perm[pos] = r;   // perm[new position] = old term index
  }
  wg_sync();
  // one thread per row: read the whole row, then write it permuted
  const int64_t rows = q.off[N];
  for (int64_t row = threadIdx.x; row < rows; row += kBT) {
    int k = 0;
    while (row >= q.off[k + 1]) ++k;
    double x[kBatchMaxR], y[kBatchMaxR];
#pragma unroll
    for (int c = 0; c < kBatchMaxR; ++c) {
      x[c] = c < R ? u[row * R + c] : 0.0;
      y[c] = (g && c < R) ? g[row * R + c] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kBatchMaxR; ++j) {
      if (j < R) {
        const int pj = perm[j];
        double xv = 0.0, yv = 0.0;
#pragma unroll
        for (int c = 0; c < kBatchMaxR; ++c)
          if (c == pj) { xv = x[c]; yv = y[c]; }
        const double sc = scl[k][pj];
        u[row * R + j] = sc * xv;
        if (g) g[row * R + j] = sc != 0.0 ? yv / sc : yv;
      }
    }
  }
  wg_sync();
}

// f and g at x (Optimization Problem I; Section 2.3): every M^(n), G^(n) =
// -M^(n) + A^(n) Gammabar^(n), f = 1/2 ||T||^2 - <A^(N), M^(N)> + 1/2 sum Gamma.
__device__ double wg_objgrad(const BReq& q, const double* __restrict__ x, double* __restrict__ gout) {
  const int R = q.R, N = q.N, RR = R * R;
  wg_grams(q, x, -1);
  wg_gammabars(q);
  for (int n = 0; n < N; ++n) wg_mttkrp(q, x, n, q.M + q.off[n] * R);
  // gradient
  for (int64_t e = threadIdx.x; e < q.L; e += kBT) {
    const int64_t row = e / R;
    const int r = (int)(e - row * R);
    int n = 0;
    while (row >= q.off[n + 1]) ++n;
    const double* Gb = q.Gb + n * RR;
    double s = 0.0;
    for (int c = 0; c < R; ++c) s = fma(x[row * R + c], Gb[c * R + r], s);
    gout[e] = s - q.M[e];
  }
  wg_sync();
  // sum of Gamma = Hadamard product of all Grams, in entry order
  double sg = 0.0;
  for (int e = threadIdx.x; e < RR; e += kBT) {
    double p = 1.0;
    for (int k = 0; k < N; ++k) p *= q.S[k * RR + e];
    sg += p;
  }
  sg = wg_sum(sg);
  const int64_t oN = q.off[N - 1] * R, nN = q.dims[N - 1] * R;
  const double am = wg_dot(x + oN, q.M + oN, nN);
  return 0.5 * q.normsq - am + 0.5 * sg;
}

// One ALS sweep in place (Section 2.3): for n in order, Gammabar^(n) from the
// current Grams, its factorisation (with the shift and pseudo-inverse
// fallbacks), M^(n) from the current factors, A^(n) = M^(n) Gammabar^(n)^-1.
__device__ void wg_als_sweep(const BReq& q, double* __restrict__ u) {
  __shared__ int kind, flags;
  const int R = q.R, RR = R * R;
  wg_grams(q, u, -1);
  for (int n = 0; n < q.N; ++n) {
    if (n > 0) wg_grams(q, u, n - 1);
    double* Gb = q.Gb + n * RR;
    for (int e = threadIdx.x; e < RR; e += kBT) {
      double p = 1.0;
      for (int k = 0; k < q.N; ++k)
        if (k != n) p *= q.S[k * RR + e];
      Gb[e] = p;
    }
    if (threadIdx.x == 0) flags = 0;
    wg_sync();
    factor_block<kBatchMaxR>(Gb, R, q.F, &kind, &flags, true);
    wg_sync();
    const int kd = kind;
    double* Mn = q.M + q.off[n] * R;
    wg_mttkrp(q, u, n, Mn);
    wg_solve_rows(q, Mn, q.dims[n], kd, u + q.off[n] * R);
  }
}

// N-GMRES Step II (Section 2.1): p_j = g_bar - g_j over the window,
// (P^T P + delta I) alpha = -P^T g_bar with delta = eps max diag, by Cholesky;
// alpha = 0 when every p_j is zero or the matrix has a pivot that is not
// positive; u_hat = u_bar + sum_j alpha_j (u_bar - u_j).  The Gram of the m
// differences and g_bar is formed over 256-entry chunks staged in LDS, each
// pair summed by one thread in entry order.
__device__ void wg_step2(const BReq& q) {
  constexpr int kC = 128;   // entries per staged chunk
  __shared__ double chunk[(kBatchMaxWindow + 1) * kC];
  __shared__ double gram[(kBatchMaxWindow + 1) * (kBatchMaxWindow + 2) / 2];
  __shared__ double alpha[kBatchMaxWindow];
  __shared__ double Lf[kBatchMaxWindow * kBatchMaxWindow];
  __shared__ double y[kBatchMaxWindow];
  const int m = q.m;
  const int nv = m + 1;   // p_0..p_{m-1}, g_bar
  const int npairs = nv * (nv + 1) / 2;
  double acc = 0.0;
  int pj = 0, pk = 0;
  if ((int)threadIdx.x < npairs) {   // pair index -> (j, k), j <= k
    int t = threadIdx.x;
    while (t >= nv - pj) { t -= nv - pj; ++pj; }
    pk = pj + t;
  }
  for (int64_t e0 = 0; e0 < q.L; e0 += kC) {
    for (int idx = threadIdx.x; idx < nv * kC; idx += kBT) {
      const int j = idx / kC, c = idx % kC;
      const int64_t e = e0 + c;
      double v = 0.0;
      if (e < q.L) {
        v = q.gbar[e];
        if (j < m) v -= q.winG[(int64_t)((q.whead + j) % q.wcap) * q.L + e];
      }
      chunk[idx] = v;
    }
    wg_sync();
    if ((int)threadIdx.x < npairs) {
      const int n = (int)std::min<int64_t>(kC, q.L - e0);
      for (int c = 0; c < n; ++c) acc = fma(chunk[pj * kC + c], chunk[pk * kC + c], acc);
    }
    wg_sync();
  }
  if ((int)threadIdx.x < npairs) gram[threadIdx.x] = acc;
  wg_sync();
  if (threadIdx.x == 0) {
    // gram index of (j, k), j <= k
    auto gi = [&](int j, int k) { return j * nv - j * (j - 1) / 2 + (k - j); };
    double dmax = 0.0;
    for (int j = 0; j < m; ++j) dmax = fmax(dmax, gram[gi(j, j)]);
    bool ok = dmax > 0.0;
    if (ok) {
      const double delta = q.eps * dmax;
      for (int j = 0; j < m; ++j)
        for (int k = 0; k <= j; ++k) Lf[j * m + k] = gram[gi(k, j)] + (j == k ? delta : 0.0);
      for (int j = 0; j < m && ok; ++j) {   // right-looking Cholesky, lower triangle
        const double d = Lf[j * m + j];
        if (!(d > 0.0) || !isfinite(d)) { ok = false; break; }
        const double s = sqrt(d);
        Lf[j * m + j] = s;
        for (int i = j + 1; i < m; ++i) Lf[i * m + j] /= s;
        for (int i = j + 1; i < m; ++i)
          for (int k = j + 1; k <= i; ++k) Lf[i * m + k] -= Lf[i * m + j] * Lf[k * m + j];
      }
    }
    if (ok) {
      for (int j = 0; j < m; ++j) y[j] = -gram[gi(j, m)];
      for (int j = 0; j < m; ++j) {   // L y = rhs
        for (int k = 0; k < j; ++k) y[j] -= Lf[j * m + k] * y[k];
        y[j] /= Lf[j * m + j];
      }
      for (int j = m - 1; j >= 0; --j) {   // L^T alpha = y
        for (int k = j + 1; k < m; ++k) y[j] -= Lf[k * m + j] * y[k];
        y[j] /= Lf[j * m + j];
      }
    }
    for (int j = 0; j < m; ++j) alpha[j] = ok ? y[j] : 0.0;
  }
  wg_sync();
  for (int64_t e = threadIdx.x; e < q.L; e += kBT) {
    const double ub = q.ubar[e];
    double s = ub;
    for (int j = 0; j < m; ++j) {
      const int slot = (q.whead + j) % q.wcap;
      s = fma(alpha[j], ub - q.winU[(int64_t)slot * q.L + e], s);
    }
    q.uhat[e] = s;
  }
  wg_sync();
}

__global__ __launch_bounds__(kBT) void batch_phase_kernel(const BReq* __restrict__ reqs,
                                                          double* __restrict__ outs) {
  const BReq q = reqs[blockIdx.x];
  double* out = outs + 4 * (int64_t)blockIdx.x;
  const int64_t L = q.L;
  if (q.phase == BP_START) {
    wg_normalize(q, q.u, nullptr);
    const double f = wg_objgrad(q, q.u, q.g);
    const double gg = wg_dot(q.g, q.g, L);
    for (int64_t e = threadIdx.x; e < L; e += kBT) {
      q.winU[(int64_t)q.push * L + e] = q.u[e];
      q.winG[(int64_t)q.push * L + e] = q.g[e];
    }
    if (threadIdx.x == 0) { out[0] = f; out[1] = gg; }
  } else if (q.phase == BP_STEP12) {
    wg_copy(q.u, q.ubar, L);
    wg_als_sweep(q, q.ubar);
    wg_normalize(q, q.ubar, nullptr);
    const double fbar = wg_objgrad(q, q.ubar, q.gbar);
    wg_step2(q);
    if (q.normalize_accel) wg_normalize(q, q.uhat, nullptr);
    for (int64_t e = threadIdx.x; e < L; e += kBT) q.d[e] = q.uhat[e] - q.ubar[e];
    wg_sync();
    const double slope = wg_dot(q.gbar, q.d, L);
    if (threadIdx.x == 0) { out[0] = fbar; out[1] = slope; }
  } else if (q.phase == BP_TRIAL) {
    if (q.keep_best) wg_copy(q.gt, q.gbest, L);
    for (int64_t e = threadIdx.x; e < L; e += kBT) q.ut[e] = fma(q.beta, q.d[e], q.ubar[e]);
    wg_sync();
    const double f = wg_objgrad(q, q.ut, q.gt);
    const double dphi = wg_dot(q.gt, q.d, L);
    if (threadIdx.x == 0) { out[0] = f; out[1] = dphi; }
  } else {   // BP_FINAL
    const double* us = q.accept == 1 ? q.ut : q.ubar;
    const double* gs = q.accept == 0 ? q.gbar : (q.accept == 1 ? q.gt : q.gbest);
    for (int64_t e = threadIdx.x; e < L; e += kBT) {
      q.u[e] = q.accept == 2 ? fma(q.beta, q.d[e], us[e]) : us[e];
      q.g[e] = gs[e];
    }
    wg_sync();
    wg_normalize(q, q.u, q.g);
    const double gg = wg_dot(q.g, q.g, L);
    for (int64_t e = threadIdx.x; e < L; e += kBT) {
      q.winU[(int64_t)q.push * L + e] = q.u[e];
      q.winG[(int64_t)q.push * L + e] = q.g[e];
    }
    if (threadIdx.x == 0) out[0] = gg;
  }
}

}  // namespace

// ---------------------------------------------------------------- host side ---

bool batch_eligible(const cp_tensor* T, int R, int64_t max_elems) {
  if (!T || T->sparse || T->dtype != CP_F32 || T->order < 3 || T->order > kBatchMaxOrder)
    return false;
  if (R < 1 || R > kBatchMaxR) return false;
  int64_t n = 1;
  for (int k = 0; k < T->order; ++k) {
    if (T->dims[k] < 1) return false;
    n *= T->dims[k];
    if (n > max_elems) return false;
  }
  return true;
}

struct BatchItem {
  cp_tensor T{};
  int R = 0;
  double tol = 0.0;
  double* u_out = nullptr;
  cp_iter_info* trace = nullptr;
  int trace_cap = 0;
  uint64_t tag = 0;
  // device memory and descriptor
  double* mem = nullptr;
  BReq d{};
  // control
  int stage = BP_START;
  int it = 0;
  double f = 0.0, rho = 0.0, normT = 0.0;
  int wcount = 0, whead = 0;
  int n_fg = 0, n_restarts = 0, n_fallback = 0;
  ls::MoreThuente mt;
  double fbar = 0.0, fnew = 0.0;
  cp_iter_info rec{};
  int n_trace = 0;
  bool done = false;
  int status = CP_OK;
  double t_start = 0.0;
};

struct BatchEngine {
  cp_handle* h = nullptr;
  hipStream_t st = nullptr;
  cp_options opt{};
  std::vector<BatchItem*> items;   // active
  BReq* hdesc = nullptr;           // pinned, capacity entries
  double* hout = nullptr;          // pinned, 4 per entry
  BReq* ddesc = nullptr;
  double* dout = nullptr;
  int cap = 0;
  int64_t ticks = 0;

  int init(cp_handle* hh, hipStream_t s, const cp_options& o, int capacity) {
    h = hh;
    st = s;
    opt = o;
    cap = capacity;
    if (hipHostMalloc(reinterpret_cast<void**>(&hdesc), sizeof(BReq) * cap) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&hout), sizeof(double) * 4 * cap) != hipSuccess ||
        hipMalloc(&ddesc, sizeof(BReq) * cap) != hipSuccess ||
        hipMalloc(&dout, sizeof(double) * 4 * cap) != hipSuccess) {
      release();
      return fail(h, CP_ENOMEM, "batch engine allocation failed");
    }
    return CP_OK;
  }

  void release() {
    if (hdesc) (void)hipHostFree(hdesc);
    if (hout) (void)hipHostFree(hout);
    if (ddesc) (void)hipFree(ddesc);
    if (dout) (void)hipFree(dout);
    hdesc = nullptr;
    hout = nullptr;
    ddesc = nullptr;
    dout = nullptr;
  }

  // Admit a request (T prepared for norm_sq); its initial guess is copied.
  int add(BatchItem* it, const double* u0) {
    if ((int)items.size() >= cap) return fail(h, CP_EINVAL, "batch is full");
    const int N = it->T.order, R = it->R;
    BReq& q = it->d;
    q = BReq{};
    q.T = static_cast<const float*>(it->T.values);
    q.N = N;
    q.R = R;
    q.off[0] = 0;
    for (int k = 0; k < N; ++k) {
      q.dims[k] = it->T.dims[k];
      q.off[k + 1] = q.off[k] + q.dims[k];
    }
    q.L = q.off[N] * R;
    q.normsq = it->T.norm_sq;
    q.wcap = std::max(1, std::min(opt.window, kBatchMaxWindow));
    q.eps = opt.eps;
    q.normalize_accel = opt.normalize_accel;
    const size_t L = (size_t)q.L, RR = (size_t)R * R;
    const size_t nd = L * (10 + 2 * (size_t)q.wcap) + RR * (2 * (size_t)N + 1);
    if (hipMalloc(&it->mem, sizeof(double) * nd) != hipSuccess) {
      it->mem = nullptr;
      return fail(h, CP_ENOMEM, "batch request allocation failed");
    }
    double* p = it->mem;
    q.u = p; p += L;
    q.g = p; p += L;
    q.ubar = p; p += L;
    q.gbar = p; p += L;
    q.uhat = p; p += L;
    q.d = p; p += L;
    q.ut = p; p += L;
    q.gt = p; p += L;
    q.gbest = p; p += L;
    q.M = p; p += L;
    q.winU = p; p += L * q.wcap;
    q.winG = p; p += L * q.wcap;
    q.S = p; p += RR * N;
    q.Gb = p; p += RR * N;
    q.F = p;
    CP_HIP(h, hipMemcpyAsync(q.u, u0, sizeof(double) * L, hipMemcpyDeviceToDevice, st));
    it->normT = std::sqrt(it->T.norm_sq);
    it->stage = BP_START;
    q.phase = BP_START;
    q.push = 0;
    items.push_back(it);
    return CP_OK;
  }

  void trace_push(BatchItem* it) {
    if (it->trace && it->n_trace < it->trace_cap) it->trace[it->n_trace++] = it->rec;
  }

  // Set the record of iteration it->it and decide: stop, or the next STEP12.
  void begin_iteration(BatchItem* it) {
    it->rec = cp_iter_info{};
    it->rec.it = it->it;
    it->rec.f = it->f;
    it->rec.rho = it->rho;
    it->rec.beta = NAN;
    it->rec.ls_status = -1;
    it->rec.m = it->wcount;
    it->rec.precision = CP_PREC_FP32IN_FP64ACC;
    if (!std::isfinite(it->f) || !std::isfinite(it->rho)) {
      trace_push(it);
      it->status = fail(h, CP_ENOTFINITE, "objective or gradient not finite");
      it->done = true;
      return;
    }
    if (it->rho <= it->tol || it->it >= opt.max_iter) {
      trace_push(it);
      it->status = it->rho <= it->tol ? CP_OK : CP_MAXITER;
      it->done = true;
      return;
    }
    it->stage = BP_STEP12;
    it->d.phase = BP_STEP12;
    it->d.m = it->wcount;
    it->d.whead = it->whead;
  }

  // The window push of the driver: drop the oldest when full, then the slot.
  int push_slot(BatchItem* it) {
    const int wcap = it->d.wcap;
    if (it->wcount == wcap) {
      it->whead = (it->whead + 1) % wcap;
      it->wcount--;
    }
    const int j = (it->whead + it->wcount) % wcap;
    it->wcount++;
    return j;
  }

  void go_final(BatchItem* it, int accept, double beta, double fnew) {
    it->stage = BP_FINAL;
    it->d.phase = BP_FINAL;
    it->d.accept = accept;
    it->d.beta = beta;
    it->fnew = fnew;
    it->d.push = push_slot(it);
  }

  // Consume the scalars of the phase a request just ran and set its next one.
  void advance(BatchItem* it, const double* o) {
    switch (it->stage) {
      case BP_START:
        it->n_fg++;
        it->f = o[0];
        it->rho = std::sqrt(std::max(0.0, o[1])) / it->normT;
        it->wcount = 1;
        it->whead = 0;
        it->it = 0;
        begin_iteration(it);
        break;
      case BP_STEP12: {
        it->n_fg++;
        it->fbar = o[0];
        const double slope = o[1];
        if (!std::isfinite(it->fbar) || !std::isfinite(slope)) {
          trace_push(it);
          it->status = fail(h, CP_ENOTFINITE, "objective or slope not finite");
          it->done = true;
          break;
        }
        if (!(slope < 0.0)) {   // restart: u_{i+1} = u_bar, window from u_{i+1}
          it->rec.restart = 1;
          it->n_restarts++;
          it->wcount = 0;
          it->whead = 0;
          go_final(it, 0, 0.0, it->fbar);
        } else {
          it->stage = BP_TRIAL;
          it->d.phase = BP_TRIAL;
          it->d.beta = it->mt.start(opt, it->fbar, slope);
          it->d.keep_best = 0;
        }
        break;
      }
      case BP_TRIAL: {
        it->n_fg++;
        if (!std::isfinite(o[0]) || !std::isfinite(o[1])) {
          trace_push(it);
          it->status = fail(h, CP_ENOTFINITE, "objective or slope not finite in the line search");
          it->done = true;
          break;
        }
        bool keep = false;
        const int status = it->mt.feed(o[0], o[1], &keep);
        if (status < 0) {
          it->d.beta = it->mt.stp;
          it->d.keep_best = keep ? 1 : 0;
          break;
        }
        it->rec.nfev = it->mt.nfev;
        it->rec.ls_status = status;
        it->rec.beta = it->mt.acc_beta;
        if (status != ls::LS_CONVERGED) it->n_fallback++;
        const int acc = it->mt.acc_grad;
        if (acc == ls::MoreThuente::ACC_NONE) go_final(it, 0, 0.0, it->fbar);
        else if (acc == ls::MoreThuente::ACC_LAST) go_final(it, 1, it->mt.acc_beta, it->mt.acc_f);
        else go_final(it, 2, it->mt.acc_beta, it->mt.acc_f);
        break;
      }
      default: {   // BP_FINAL
        it->f = it->fnew;
        it->rho = std::sqrt(std::max(0.0, o[0])) / it->normT;
        trace_push(it);
        it->it++;
        begin_iteration(it);
        break;
      }
    }
  }

  // One tick: one launch over every active request, one readback.  Finished
  // requests are moved to *finished (their result copied to u_out).
  int tick(std::vector<BatchItem*>* finished) {
    const int n = (int)items.size();
    if (n == 0) return CP_OK;
    for (int b = 0; b < n; ++b) hdesc[b] = items[b]->d;
    CP_HIP(h, hipMemcpyAsync(ddesc, hdesc, sizeof(BReq) * n, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(batch_phase_kernel, dim3((unsigned)n), dim3(kBT), 0, st, ddesc, dout);
    CP_LAUNCH_CHECK(h);
    CP_HIP(h, hipMemcpyAsync(hout, dout, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, st));
    CP_HIP(h, hipStreamSynchronize(st));
    ++ticks;
    std::vector<BatchItem*> keep;
    keep.reserve(n);
    for (int b = 0; b < n; ++b) {
      BatchItem* it = items[b];
      advance(it, hout + 4 * b);
      if (it->done) {
        if (it->u_out)
          CP_HIP(h, hipMemcpyAsync(it->u_out, it->d.u, sizeof(double) * it->d.L,
                                   hipMemcpyDeviceToDevice, st));
        finished->push_back(it);
      } else {
        keep.push_back(it);
      }
    }
    items.swap(keep);
    if (!finished->empty()) CP_HIP(h, hipStreamSynchronize(st));
    return CP_OK;
  }
};

// Frees a finished item's device memory (its stream work is complete).
void batch_item_free(BatchItem* it) {
  if (it->mem) (void)hipFree(it->mem);
  it->mem = nullptr;
}

BatchEngine* batch_engine_create(cp_handle* h, hipStream_t st, const cp_options& o, int capacity) {
  auto* e = new (std::nothrow) BatchEngine();
  if (!e) return nullptr;
  if (e->init(h, st, o, capacity) != CP_OK) {
    delete e;
    return nullptr;
  }
  return e;
}

void batch_engine_destroy(BatchEngine* e) {
  if (!e) return;
  (void)hipStreamSynchronize(e->st);
  for (BatchItem* it : e->items) {
    batch_item_free(it);
    delete it;
  }
  e->release();
  delete e;
}

int batch_engine_add(BatchEngine* e, const cp_tensor* T, int R, double tol, const double* u0,
                     double* u_out, uint64_t tag, cp_iter_info* trace, int trace_cap,
                     BatchItem** out) {
  auto* it = new (std::nothrow) BatchItem();
  if (!it) return fail(e->h, CP_ENOMEM, "host allocation failed");
  it->T = *T;
  it->R = R;
  it->tol = tol;
  it->u_out = u_out;
  it->tag = tag;
  it->trace = trace;
  it->trace_cap = trace_cap;
  const int rc = e->add(it, u0);
  if (rc != CP_OK) {
    delete it;
    return rc;
  }
  if (out) *out = it;
  return CP_OK;
}

int batch_engine_tick(BatchEngine* e, std::vector<BatchItem*>* finished) { return e->tick(finished); }
int batch_engine_active(const BatchEngine* e) { return (int)e->items.size(); }

void batch_engine_drain(BatchEngine* e, std::vector<BatchItem*>* out) {
  (void)hipStreamSynchronize(e->st);
  for (BatchItem* it : e->items) {
    if (it->status == CP_OK) it->status = CP_EDEVICE;
    out->push_back(it);
  }
  e->items.clear();
}

void batch_item_delete(BatchItem* it) {
  batch_item_free(it);
  delete it;
}

// Device bytes of a request on the batched path: the tensor, 10 + 2 w
// iterate-length vectors and the Grams, Gammabars and factor.
int64_t batch_footprint(const cp_tensor* T, int R, int window) {
  int64_t total = 1, sum = 0;
  for (int k = 0; k < T->order; ++k) {
    total *= T->dims[k];
    sum += T->dims[k];
  }
  const int64_t w = std::max(1, std::min(window, kBatchMaxWindow));
  return total * 4 + 8 * sum * R * (10 + 2 * w) + 8 * (int64_t)R * R * (2 * T->order + 1);
}

void batch_item_report(const BatchItem* it, cp_report* rep, int* status, uint64_t* tag) {
  if (rep) {
    *rep = cp_report{};
    rep->iters = it->it;
    rep->converged = it->status == CP_OK && it->rho <= it->tol;
    rep->f = it->f;
    rep->rho = it->rho;
    rep->n_fg = it->n_fg;
    rep->n_restarts = it->n_restarts;
    rep->n_ls_fallback = it->n_fallback;
    rep->switch_iter = -1;
    rep->n_trace = it->n_trace;
  }
  if (status) *status = it->status;
  if (tag) *tag = it->tag;
}

}  // namespace cpng

using namespace cpng;

extern "C" int cp_batch_decompose(cp_handle* h, int32_t n, cp_batch_request* reqs,
                                  const cp_options* opt, hipStream_t st) {
  if (!h || n < 0 || (n > 0 && !reqs)) return CP_EINVAL;
  CP_HIP(h, hipSetDevice(h->device));
  const auto t0 = std::chrono::steady_clock::now();
  cp_options o;
  if (opt) o = *opt;
  else cp_options_default(&o);
  if (o.method != CP_METHOD_NGMRES) return fail(h, CP_EINVAL, "the batched path runs N-GMRES with ALS");
  if (o.window < 1 || o.window > kBatchMaxWindow)
    return fail(h, CP_EINVAL, "window must be in 1..%d for the batched path", kBatchMaxWindow);
  if (o.ls_maxfev < 1 || !(o.ls_stp0 > 0.0)) return fail(h, CP_EINVAL, "bad line-search options");
  for (int i = 0; i < n; ++i) {
    cp_batch_request& r = reqs[i];
    if (!batch_eligible(r.T, r.R, CP_BATCH_MAX_ELEMS))
      return fail(h, CP_EINVAL, "request %d: the batched path takes dense float32 tensors of "
                  "order 3 or 4 with at most %lld entries and 1 <= R <= %d", i,
                  (long long)CP_BATCH_MAX_ELEMS, kBatchMaxR);
    if (!r.u_inout || !r.T->values) return fail(h, CP_EINVAL, "request %d: null array", i);
    if (!(r.T->norm_sq > 0.0)) return fail(h, CP_EINVAL, "request %d: tensor not prepared", i);
    if (!(r.tol >= 0.0)) return fail(h, CP_EINVAL, "request %d: tol must be >= 0", i);
  }
  hipStream_t s = st;
  bool own = false;
  if (!s) {
    CP_HIP(h, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    own = true;
  }
  int rc = CP_OK;
  BatchEngine* e = batch_engine_create(h, s, o, std::max(1, n));
  if (!e) rc = fail(h, CP_ENOMEM, "batch engine allocation failed");
  std::vector<BatchItem*> all;
  for (int i = 0; i < n && rc == CP_OK; ++i) {
    BatchItem* it = nullptr;
    rc = batch_engine_add(e, reqs[i].T, reqs[i].R, reqs[i].tol, reqs[i].u_inout, reqs[i].u_inout,
                          (uint64_t)i, reqs[i].trace, reqs[i].trace_cap, &it);
    if (rc == CP_OK) all.push_back(it);
  }
  std::vector<BatchItem*> fin;
  while (rc == CP_OK && batch_engine_active(e) > 0) rc = batch_engine_tick(e, &fin);
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (e) (void)hipStreamSynchronize(s);
  for (BatchItem* it : fin) {
    cp_batch_request& r = reqs[it->tag];
    batch_item_report(it, &r.report, &r.status, nullptr);
    r.report.seconds = secs;
    batch_item_free(it);
    delete it;
  }
  if (e) batch_engine_destroy(e);   // frees what a failed run left active
  if (own) (void)hipStreamDestroy(s);
  return rc;
}
