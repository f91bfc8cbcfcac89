// Two-level evaluation of all N MTTKRPs of a dense tensor at one point
// (Section 2.3, M^(n) = T_(n) Phibar^(n) for every n), and the same split for
// the ALS sweep.  The modes are cut into a left group [0, s) and a right
// group [s, N).  Two partial contractions stream T once each:
//     X_L(i_0..i_{s-1}, r) = sum_{i_s..i_{N-1}} T(i) prod_{m >= s} A^(m)(i_m, r),
//     X_R(i_s..i_{N-1}, r) = sum_{i_0..i_{s-1}} T(i) prod_{m < s}  A^(m)(i_m, r).
// Each is an ordinary MTTKRP of T seen with one group merged into a single
// mode: X_L is mode 0 of T as (I_0 ... I_{s-1}, I_s, .., I_{N-1}), X_R the
// last mode of T as (I_0, .., I_{s-1}, I_s ... I_{N-1}), so they run on the
// same streaming kernels (and precisions) as the per-mode MTTKRPs.  Every
// M^(n) is then an MTTKRP of its group's partial that is elementwise in r:
//     M^(n)(i, r) = sum_{i_m, m in group, m != n} X(.., i, .., r) prod_{m in group, m != n} A^(m)(i_m, r),
// computed in float64 from the float64 partial.  A group of one mode needs no
// second level: its partial is M^(n) itself.  T is streamed twice instead of
// N times.  In the ALS sweep X_L is formed before the updates of the left
// modes (which leave the right factors alone) and X_R after them, so each
// M^(n) sees the factors exactly as the sequential update does.
//
// For the split before the last mode in the float32 and float64 vector-ALU
// precisions, X_L is formed by contract_last_kernel: 64 rows of T (as a
// rows x I_N matrix) per workgroup, inner chunks of 64 through LDS
// (transposed) with the factor chunk next to them, the next chunk's loads in
// flight while the current one is multiplied; lane = row, the four waves
// take every fourth k and are added in a fixed order at the end.
//
// Second level: thread (i, r) walks a contiguous range of the other indices
// (outer o, inner k) of the group for mode n, loads issued 8 at a time.
// Short sums take one launch (group_fused_kernel: four waves per 64 outputs,
// the quarters added in a fixed order, the gradient epilogue fused); long
// ones are split over workgroups (group_mttkrp_kernel) and the slots added by
// the fixed-order split-K reduction.  No atomics anywhere: results are
// reproducible.
#include "common.hpp"
#include "splitk.hpp"

#include <algorithm>

namespace cpng {

namespace {

constexpr int kThr = 256;

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

constexpr int kTB = 64;   // rows and inner chunk per tile of the last-mode contraction

struct LastParams {
  int64_t rows;    // prod_{m < N-1} I_m
  int64_t K;       // I_{N-1}
  int R;
  int64_t qfoff;   // element offset of A^(N-1) in the factors
  int vec_ok;      // rows start on 16-byte boundaries
};

// Left partial of the split before the last mode on the vector ALUs:
// X(row, r) = sum_k T(row, k) A^(N-1)(k, r) for T as a rows x I_{N-1} matrix.
template <typename TT, typename CT, int RB>
__global__ __launch_bounds__(kThr) void contract_last_kernel(const TT* __restrict__ T,
                                                             const CT* __restrict__ fac,
                                                             LastParams p, double* __restrict__ Y) {
  constexpr int TB = kTB;
  constexpr int TS = TB + 1;
  constexpr int VE = 16 / sizeof(TT);
  constexpr int NL = TB * TB / VE / kThr;
  constexpr int NB = TB * RB / kThr;
  static_assert(NB >= 1, "RB too small for the factor tile split");
  __shared__ CT Ts[TB * TS];   // [k][row]
  __shared__ CT Bs[TB * RB];   // [k][r]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int g = tid >> 6;
  const int r0 = blockIdx.y * RB;
  const int64_t row0 = (int64_t)blockIdx.x * TB;
  const int nkc = (int)((p.K + TB - 1) / TB);

  CT acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = CT(0);
  TT v[NL][VE];
  CT b[NB];

  auto load_chunk = [&](int kc) {
    const int64_t k0 = (int64_t)kc * TB;
#pragma unroll
    for (int t = 0; t < NL; ++t) {
      const int e = tid + t * kThr;
      const int ii = e / (TB / VE), kk = (e % (TB / VE)) * VE;
      const int64_t row = row0 + ii, k = k0 + kk;
      if (p.vec_ok && row < p.rows && k + VE <= p.K) {
        const TT* src = T + row * p.K + k;
        if constexpr (VE == 4) {
          const float4 x = *reinterpret_cast<const float4*>(src);
          v[t][0] = x.x; v[t][1] = x.y; v[t][2] = x.z; v[t][3] = x.w;
        } else {
          const double2 x = *reinterpret_cast<const double2*>(src);
          v[t][0] = x.x; v[t][1] = x.y;
        }
      } else {
#pragma unroll
        for (int q = 0; q < VE; ++q)
          v[t][q] = (row < p.rows && k + q < p.K) ? T[row * p.K + k + q] : TT(0);
      }
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int e = tid + t * kThr;
      const int kk = e / RB, rr = e - (e / RB) * RB;
      const int64_t k = k0 + kk;
      b[t] = (k < p.K && r0 + rr < p.R) ? fac[p.qfoff + k * p.R + r0 + rr] : CT(0);
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int t = 0; t < NL; ++t) {
      const int e = tid + t * kThr;
      const int ii = e / (TB / VE), kk = (e % (TB / VE)) * VE;
#pragma unroll
      for (int q = 0; q < VE; ++q) Ts[(kk + q) * TS + ii] = (CT)v[t][q];
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) Bs[tid + t * kThr] = b[t];
  };

  load_chunk(0);
  for (int kc = 0; kc < nkc; ++kc) {
    __syncthreads();   // every wave is done with the previous chunk
    store_chunk();
    __syncthreads();
    if (kc + 1 < nkc) load_chunk(kc + 1);
    const int kv = (int)min<int64_t>(TB, p.K - (int64_t)kc * TB);
    for (int kk = g; kk < kv; kk += 4) {
      const CT x = Ts[kk * TS + lane];
#pragma unroll
      for (int r = 0; r < RB; ++r) acc[r] = fma(x, Bs[kk * RB + r], acc[r]);
    }
  }
  // fixed-order sum of the four waves: (0 + 2) + (1 + 3), then 0 + 1
  __syncthreads();
  CT* red = Ts;
  if (g >= 2)
#pragma unroll
    for (int r = 0; r < RB; ++r) red[((g - 2) * RB + r) * TS + lane] = acc[r];
  __syncthreads();
  if (g < 2)
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] += red[(g * RB + r) * TS + lane];
  __syncthreads();
  if (g == 1)
#pragma unroll
    for (int r = 0; r < RB; ++r) red[r * TS + lane] = acc[r];
  __syncthreads();
  if (g == 0) {
    const int64_t row = row0 + lane;
    if (row < p.rows) {
#pragma unroll
      for (int r = 0; r < RB; ++r)
        if (r0 + r < p.R) Y[row * p.R + r0 + r] = (double)(acc[r] + red[r * TS + lane]);
    }
  }
}

template <typename TT, typename CT>
int launch_contract_last(cp_handle* h, const TT* T, const CT* fac, const LastParams& p, double* X,
                         hipStream_t st) {
  const int RB = p.R <= 8 ? 8 : (p.R <= 16 ? 16 : 32);
  const dim3 grid(nblk(p.rows, kTB), (unsigned)((p.R + RB - 1) / RB));
  KernelTimer timer(h, dense_kernel_id<CT>(), st);
  if (RB == 8) CP_TIMED_LAUNCH(timer, (contract_last_kernel<TT, CT, 8>), grid, dim3(kThr), 0, st, T, fac, p, X);
  else if (RB == 16) CP_TIMED_LAUNCH(timer, (contract_last_kernel<TT, CT, 16>), grid, dim3(kThr), 0, st, T, fac, p, X);
  else CP_TIMED_LAUNCH(timer, (contract_last_kernel<TT, CT, 32>), grid, dim3(kThr), 0, st, T, fac, p, X);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

struct GroupParams {
  int R;
  int nlo, nhi;                      // group modes before / after the target mode
  int64_t lodims[CP_MAX_ORDER];      // their sizes (in mode order)
  int64_t hidims[CP_MAX_ORDER];
  int64_t lofoff[CP_MAX_ORDER];      // their factors' element offsets
  int64_t hifoff[CP_MAX_ORDER];
  int64_t O, I, K;                   // prod lodims, target size, prod hidims
  int64_t per;                       // (o, k) pairs per range
};

// prod over the nm modes of the multi-index x (last mode fastest) of
// A^(m)(x_m, r).  Group sizes fit in 32 bits.
__device__ inline double idx_product(int64_t x, int nm, const int64_t* dims, const int64_t* foff,
                                     const double* __restrict__ fac, int R, int r) {
  if (nm == 0) return 1.0;
  if (nm == 1) return fac[foff[0] + x * R + r];
  double s = 1.0;
  uint32_t xx = (uint32_t)x;
  for (int m = nm - 1; m >= 0; --m) {
    const uint32_t d = (uint32_t)dims[m];
    const uint32_t q = xx / d;
    s *= fac[foff[m] + (int64_t)(xx - q * d) * R + r];
    xx = q;
  }
  return s;
}

// Sum over the (o, k) pairs f0 .. f1-1 (o major) of X(o, i, k, r) P(o, r) Q(k, r),
// in pair order, loads issued 8 at a time.
__device__ inline double group_range(const double* __restrict__ X, const double* __restrict__ fac,
                                     const GroupParams& p, int64_t i, int r, int64_t f0,
                                     int64_t f1) {
  double acc = 0.0;
  if (p.K == 1) {   // target is the group's last mode: the pairs are the outer indices o
    const double* x = X + i * p.R + r;
    const int64_t ostep = p.I * p.R;
    for (int64_t o = f0; o < f1; o += 8) {
      double xv[8], pv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const bool ok = o + j < f1;
        xv[j] = ok ? x[(o + j) * ostep] : 0.0;
        pv[j] = ok ? idx_product(o + j, p.nlo, p.lodims, p.lofoff, fac, p.R, r) : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) acc = fma(xv[j], pv[j], acc);
    }
    return acc;
  }
  int64_t f = f0;
  while (f < f1) {
    const int64_t o = f / p.K;
    const int64_t k0 = f - o * p.K;
    const int64_t k1 = min<int64_t>(p.K, k0 + (f1 - f));
    const double P = idx_product(o, p.nlo, p.lodims, p.lofoff, fac, p.R, r);
    const double* x = X + ((o * p.I + i) * p.K) * p.R + r;
    double s = 0.0;
    for (int64_t k = k0; k < k1; k += 8) {
      double xv[8], qv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const bool ok = k + j < k1;
        xv[j] = ok ? x[(k + j) * p.R] : 0.0;
        qv[j] = ok ? idx_product(k + j, p.nhi, p.hidims, p.hifoff, fac, p.R, r) : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) s = fma(xv[j], qv[j], s);
    }
    acc = fma(P, s, acc);
    f += k1 - k0;
  }
  return acc;
}

// part[c][i * R + r] = the c-th range of (o, k) pairs (group_range).
__global__ __launch_bounds__(kThr) void group_mttkrp_kernel(const double* __restrict__ X,
                                                            const double* __restrict__ fac,
                                                            GroupParams p,
                                                            double* __restrict__ part) {
  const int64_t e = (int64_t)blockIdx.x * kThr + threadIdx.x;
  if (e >= p.I * p.R) return;
  const int64_t i = e / p.R;
  const int r = (int)(e - i * p.R);
  const int64_t f0 = (int64_t)blockIdx.y * p.per;
  const int64_t f1 = min<int64_t>(p.O * p.K, f0 + p.per);
  part[(int64_t)blockIdx.y * p.I * p.R + e] = group_range(X, fac, p, i, r, f0, f1);
}

// Short sums (O K <= kFusedPairs) in one launch: block b covers outputs
// 64 b .. 64 b + 63 (lane = output), wave w adds the w-th quarter of the pairs,
// the quarters are added in a fixed order, and with a pending gradient
// epilogue G(i, r) = -M(i, r) + sum_q A(i, q) Gbar(q, r) (Gbar staged in LDS).
constexpr int64_t kFusedPairs = 2048;

__device__ __forceinline__ void group_fused_body(const double* __restrict__ X,
                                                 const double* __restrict__ fac,
                                                 const GroupParams& p, double* __restrict__ M,
                                                 const double* __restrict__ eA,
                                                 const double* __restrict__ eGbar,
                                                 double* __restrict__ eG, int64_t bx) {
  extern __shared__ double gsh[];
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t e = bx * 64 + lane;
  const int64_t n = p.I * p.R;
  if (eG)
    for (int t = threadIdx.x; t < p.R * p.R; t += kThr) gsh[t] = eGbar[t];
  double s = 0.0;
  const int64_t i = e / p.R;
  const int r = (int)(e - i * p.R);
  if (e < n) {
    const int64_t work = p.O * p.K, q4 = (work + 3) / 4;
    const int64_t f0 = w * q4, f1 = min<int64_t>(work, f0 + q4);
    if (f0 < f1) s = group_range(X, fac, p, i, r, f0, f1);
  }
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && e < n) {
    const double t = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    M[e] = t;
    if (eG) {
      const double* a = eA + i * p.R;
      double g = 0.0;
      for (int q = 0; q < p.R; ++q) g = fma(a[q], gsh[q * p.R + r], g);
      eG[e] = g - t;
    }
  }
}

__global__ __launch_bounds__(kThr) void group_fused_kernel(const double* __restrict__ X,
                                                           const double* __restrict__ fac,
                                                           GroupParams p, double* __restrict__ M,
                                                           const double* __restrict__ eA,
                                                           const double* __restrict__ eGbar,
                                                           double* __restrict__ eG) {
  group_fused_body(X, fac, p, M, eA, eGbar, eG, blockIdx.x);
}

// Every mode of a low-order tensor in one launch: the blocks of mode m are
// bstart[m] .. bstart[m + 1] - 1, each running the single-mode body.
constexpr int kMultiModes = 4;
struct MultiGroup {
  int nm;
  int64_t bstart[kMultiModes + 1];
  GroupParams p[kMultiModes];
  const double* X[kMultiModes];
  double* M[kMultiModes];
  const double* eA[kMultiModes];
  const double* eGbar[kMultiModes];
  double* eG[kMultiModes];
};

static_assert(sizeof(MultiGroup) <= 2048, "kernel argument size");

__global__ __launch_bounds__(kThr) void group_fused_multi_kernel(const double* __restrict__ fac,
                                                                 MultiGroup mg) {
  int m = 0;
  while (m + 1 < mg.nm && (int64_t)blockIdx.x >= mg.bstart[m + 1]) ++m;
  group_fused_body(mg.X[m], fac, mg.p[m], mg.M[m], mg.eA[m], mg.eGbar[m], mg.eG[m],
                   (int64_t)blockIdx.x - mg.bstart[m]);
}


int64_t group_size(const Shape& s, int lo, int hi) {
  int64_t t = 1;
  for (int m = lo; m < hi; ++m) t *= s.dims[m];
  return t;
}

}  // namespace

int tree_split(const cp_tensor* T, const Shape& s, int prec) {
  if (T->sparse || s.N < 3) return 0;
  if ((prec == CP_PREC_FP32 || prec == CP_PREC_BF16X3) && T->dtype != CP_F32) return 0;
  // the split whose second-level partials are smallest (ties to the larger
  // s), among those whose partials have at most 2^22 rows (the partial
  // MTTKRP puts its output rows on the second grid dimension)
  constexpr int64_t kMaxRows = int64_t(1) << 22;
  int best = 0;
  int64_t cost = 0;
  for (int k = 1; k < s.N; ++k) {
    const int64_t l = k > 1 ? group_size(s, 0, k) : 0;
    const int64_t r = s.N - k > 1 ? group_size(s, k, s.N) : 0;
    if (l > kMaxRows || r > kMaxRows) continue;
    if (best == 0 || l + r <= cost) {
      best = k;
      cost = l + r;
    }
  }
  return best;
}

size_t tree_partial_elems(const Shape& s, int split, int R, bool left) {
  const int64_t n = left ? (split > 1 ? group_size(s, 0, split) : 0)
                         : (s.N - split > 1 ? group_size(s, split, s.N) : 0);
  return (size_t)n * (size_t)R;
}

int tree_partial(cp_handle* h, const cp_tensor* T, const Shape& s, const double* u, int R, int prec,
                 int split, bool left, double* X, hipStream_t st) {
  if (left && split == s.N - 1 && prec != CP_PREC_BF16X3) {
    // T as a rows x I_{N-1} matrix times the last factor, on the vector ALUs
    LastParams p{};
    p.K = s.dims[s.N - 1];
    p.rows = s.total() / p.K;
    p.R = R;
    p.qfoff = s.off[s.N - 1] * R;
    const size_t tb = T->dtype == CP_F32 ? 4 : 8;
    p.vec_ok = (p.K * tb) % 16 == 0 && reinterpret_cast<uintptr_t>(T->values) % 16 == 0;
    h->t_passes++;
    if (prec == CP_PREC_FP32) {
      float* f32 = nullptr;
      CP_TRY(stage_factors_f32(h, u, s.sum_dims() * R, &f32, st));
      return launch_contract_last<float, float>(h, static_cast<const float*>(T->values), f32, p, X, st);
    }
    if (T->dtype == CP_F32)
      return launch_contract_last<float, double>(h, static_cast<const float*>(T->values), u, p, X, st);
    return launch_contract_last<double, double>(h, static_cast<const double*>(T->values), u, p, X, st);
  }
  // T seen with the other group merged into one mode; the merged mode's
  // factor offset is never read (it is the output mode).
  Shape v{};
  int mode;
  if (left) {
    v.N = s.N - split + 1;
    v.dims[0] = group_size(s, 0, split);
    v.off[0] = 0;
    for (int m = split; m < s.N; ++m) {
      v.dims[m - split + 1] = s.dims[m];
      v.off[m - split + 1] = s.off[m];
    }
    mode = 0;
  } else {
    v.N = split + 1;
    for (int m = 0; m < split; ++m) {
      v.dims[m] = s.dims[m];
      v.off[m] = s.off[m];
    }
    v.dims[split] = group_size(s, split, s.N);
    v.off[split] = 0;
    mode = split;
  }
  v.off[v.N] = s.off[s.N];   // all factor rows (precision staging converts them all)
  return dense_mttkrp(h, T, v, u, R, mode, prec, X, st);
}

int tree_partials_one_pass(cp_handle* h, const cp_tensor* T, const Shape& s, const double* u, int R,
                           int prec, int split, double* XL, double* XR, hipStream_t st) {
  if (T->sparse || T->dtype != CP_F32 || !XL || !XR) return 1;
  return dense_twosided(h, static_cast<const float*>(T->values), u, s, split, R, prec, XL, XR, st);
}

namespace {
// The second-level description of `mode` within the group [lo, hi).
GroupParams group_params(const Shape& s, int lo, int hi, int mode, int R) {
  GroupParams p{};
  p.R = R;
  p.O = 1;
  p.K = 1;
  for (int m = lo; m < hi; ++m) {
    if (m < mode) {
      p.lodims[p.nlo] = s.dims[m];
      p.lofoff[p.nlo] = s.off[m] * R;
      p.O *= s.dims[m];
      p.nlo++;
    } else if (m > mode) {
      p.hidims[p.nhi] = s.dims[m];
      p.hifoff[p.nhi] = s.off[m] * R;
      p.K *= s.dims[m];
      p.nhi++;
    }
  }
  p.I = s.dims[mode];
  return p;
}
}  // namespace

int tree_all_modes(cp_handle* h, const Shape& s, int split, const double* XL, const double* XR,
                   const double* u, int R, double* M, const double* Gbar, double* g,
                   hipStream_t st) {
  if (s.N > kMultiModes || !XL || !XR || split < 1 || split >= s.N) return 1;
  MultiGroup mg{};
  mg.nm = s.N;
  int64_t blocks = 0;
  for (int n = 0; n < s.N; ++n) {
    const bool left = n < split;
    const GroupParams p = group_params(s, left ? 0 : split, left ? split : s.N, n, R);
    if (p.O * p.K > kFusedPairs) return 1;
    mg.p[n] = p;
    mg.bstart[n] = blocks;
    blocks += nblk(p.I * R, 64);
    mg.X[n] = left ? XL : XR;
    mg.M[n] = M + s.off[n] * R;
    mg.eA[n] = g ? u + s.off[n] * R : nullptr;
    mg.eGbar[n] = g ? Gbar + (int64_t)n * R * R : nullptr;
    mg.eG[n] = g ? g + s.off[n] * R : nullptr;
  }
  mg.bstart[s.N] = blocks;
  {
    KernelTimer timer(h, CP_KERNEL_GROUP_MTTKRP, st);
    CP_TIMED_LAUNCH(timer, group_fused_multi_kernel, dim3((unsigned)blocks), dim3(kThr),
                    g ? sizeof(double) * (size_t)R * R : 0, st, u, mg);
  }
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

int tree_mode(cp_handle* h, const Shape& s, int lo, int hi, const double* X, const double* u, int R,
              int mode, double* M, hipStream_t st) {
  GroupParams p = group_params(s, lo, hi, mode, R);
  const int64_t n_out = p.I * R;
  const int64_t work = p.O * p.K;
  if (work <= kFusedPairs) {
    GradEpi& ep = h->epi;
    const bool epi = ep.G != nullptr && !ep.used;
    {
      KernelTimer timer(h, CP_KERNEL_GROUP_MTTKRP, st);
      CP_TIMED_LAUNCH(timer, group_fused_kernel, dim3(nblk(n_out, 64)), dim3(kThr),
                         epi ? sizeof(double) * (size_t)R * R : 0, st, X, u, p, M,
                         epi ? ep.A : nullptr, epi ? ep.Gbar : nullptr, epi ? ep.G : nullptr);
    }
    CP_LAUNCH_CHECK(h);
    if (epi) ep.used = true;
    return CP_OK;
  }
  // about 2^19 threads, at least 8 (o, k) pairs each (one batch of loads),
  // at most 32768 ranges
  const int64_t want = std::min<int64_t>(32768, std::max<int64_t>(1, (int64_t(1) << 19) / n_out));
  p.per = std::max<int64_t>(8, (work + want - 1) / want);
  const int64_t nch = (work + p.per - 1) / p.per;
  const dim3 grid(nblk(n_out, kThr), (unsigned)nch);
  CP_TRY(ensure(h, h->part, sizeof(double) * (size_t)(nch * n_out), st));
  double* part = static_cast<double*>(h->part.ptr);
  {
    KernelTimer timer(h, CP_KERNEL_GROUP_MTTKRP, st);
    CP_TIMED_LAUNCH(timer, group_mttkrp_kernel, grid, dim3(kThr), 0, st, X, u, p, part);
  }
  CP_LAUNCH_CHECK(h);
  CP_TRY(launch_splitk_reduce(h, part, nch, n_out, R, M, st));
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

// The left partial at a renormalised iterate.  Normalising moves term
// perm[j] to position j and scales its factor column in mode k by
// scales[k R + perm[j]]; K_R's column of a term is the Khatri-Rao product of
// the right group's factor columns, so X_L = T K_R becomes
//     X_L'(p, j) = X_L(p, perm[j]) prod_{k >= split} scales[k R + perm[j]].
// In place, 64 / R rows per wave: a row's lanes all read (one load
// instruction, whose results every store waits for) before any lane stores.
__global__ __launch_bounds__(256) void rescale_left_kernel(double* __restrict__ X, int64_t P, int R,
                                                           int split, int N,
                                                           const double* __restrict__ scales,
                                                           const int* __restrict__ perm) {
  const int lane = threadIdx.x & 63;
  const int rpw = 64 / R;
  const int j = lane % R, sub = lane / R;
  const int64_t p = (((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6) * rpw + sub;
  if (sub >= rpw || p >= P) return;
  const int pj = perm[j];
  double fac = 1.0;
  for (int k = split; k < N; ++k) fac *= scales[k * R + pj];
  const double v = X[p * R + pj];
  X[p * R + j] = v * fac;
}

int tree_rescale_left(cp_handle* h, const Shape& s, int split, int R, double* XL,
                      const double* scales, const int* perm, hipStream_t st) {
  const int64_t P = group_size(s, 0, split);
  if (P <= 0 || R < 1 || R > 64) return 1;
  const int64_t waves = (P + 64 / R - 1) / (64 / R);
  hipLaunchKernelGGL(rescale_left_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, XL, P,
                     R, split, s.N, scales, perm);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

}  // namespace cpng
