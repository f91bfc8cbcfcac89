// Dense MTTKRP on gfx950: M^(n) = T_(n) Phibar^(n)  (Section 2.3).
//
// Every mode uses one view of the C-order tensor as a 3-way array
// T[l][i][j] with l the C-order index of the modes before n (I_left values),
// i = i_n (I_n values) and j the C-order index of the modes after n (I_right
// values).  The contraction index is c = l * I_right + j, and
//     M(i, r) = sum_c T[l][i][j] * B[c][r],   B[c][r] = prod_{k != n} A^(k)(i_k(c), r),
// i.e. B is the Khatri-Rao row of the other modes (Phibar^(n) row c).  B is
// never materialised: each workgroup builds the rows of its current tile in
// LDS from the (float32 or float64) factor copies.
//
// Split-K over workgroups: blockIdx.x owns a contiguous range of tiles of the
// contraction, blockIdx.y a chunk of rows i, blockIdx.z a chunk of ranks r.
// Each workgroup writes its partial I-chunk x R-chunk sums to its own slot of
// a partial buffer; a second kernel adds the slots in slot order in float64.
// No atomics anywhere: results are bitwise reproducible.
#include "common.hpp"
#include "splitk.hpp"

#include <algorithm>

namespace cpng {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 64;   // contraction indices per tile

struct DenseParams {
  int N, mode, R;
  int64_t dims[CP_MAX_ORDER];
  int64_t foff[CP_MAX_ORDER];   // element offset of A^(k) in the factor buffer
  int64_t I_left, I_n, I_right, C;
  int64_t ntiles, tiles_per_block;
  int64_t ksplit;
};

// Decompose contraction index c into (l, j) and the mode indices of every
// other mode; writes idx[k * kTile + cc] (k != mode) and the element offset
// of T[l][0][j].
__device__ inline void decompose(const DenseParams& p, int64_t c, int cc, int32_t* idx,
                                 int64_t* base) {
  int64_t l = c / p.I_right;
  int64_t j = c - l * p.I_right;
  base[cc] = l * p.I_n * p.I_right + j;
  for (int k = p.N - 1; k > p.mode; --k) {
    int64_t q = j / p.dims[k];
    idx[k * kTile + cc] = (int32_t)(j - q * p.dims[k]);
    j = q;
  }
  for (int k = p.mode - 1; k >= 0; --k) {
    int64_t q = l / p.dims[k];
    idx[k * kTile + cc] = (int32_t)(l - q * p.dims[k]);
    l = q;
  }
}

// Generic vector kernel.  Threads: lane = tid & 63 owns rows i0 + lane + 64 s
// (s < S); wave g = tid >> 6 handles tile columns cc = g, g + 4, ...  RB ranks
// per workgroup (blockIdx.z chunk), CT the arithmetic type, TT the tensor type.
template <typename TT, typename CT, int RB, int S>
__global__ __launch_bounds__(kThreads) void mttkrp_vec_kernel(const TT* __restrict__ T,
                                                              const CT* __restrict__ fac,
                                                              DenseParams p,
                                                              double* __restrict__ part) {
  constexpr int IC = 64 * S;          // rows per workgroup
  constexpr int TS = IC + 1;          // padded LDS row stride of the tensor tile
  constexpr size_t kTileBytes = sizeof(CT) * (size_t)kTile * TS + sizeof(CT) * kTile * RB;
  constexpr size_t kRedBytes = 2 * sizeof(CT) * (size_t)IC * RB;
  constexpr size_t kLds = kTileBytes > kRedBytes ? kTileBytes : kRedBytes;
  __shared__ __align__(16) unsigned char lds[kLds];
  __shared__ int32_t idx[CP_MAX_ORDER * kTile];
  __shared__ int64_t base[kTile];
  CT* Ts = reinterpret_cast<CT*>(lds);                 // [kTile][TS]
  CT* Bs = Ts + (size_t)kTile * TS;                    // [kTile][RB]

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int g = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.y * IC;
  const int rows = (int)min<int64_t>(IC, p.I_n - i0);
  const int r0 = blockIdx.z * RB;

  CT acc[S][RB];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[s][r] = CT(0);

  const int64_t t_begin = (int64_t)blockIdx.x * p.tiles_per_block;
  const int64_t t_end = min<int64_t>(p.ntiles, t_begin + p.tiles_per_block);
  for (int64_t t = t_begin; t < t_end; ++t) {
    const int64_t c0 = t * kTile;
    const int len = (int)min<int64_t>(kTile, p.C - c0);
    if (tid < len) decompose(p, c0 + tid, tid, idx, base);
    __syncthreads();
    // Khatri-Rao rows of this tile (zero beyond R)
    for (int e = tid; e < kTile * RB; e += kThreads) {
      const int cc = e / RB, rr = e - (e / RB) * RB;
      const int r = r0 + rr;
      CT prod = CT(0);
      if (cc < len && r < p.R) {
        prod = CT(1);
        for (int k = 0; k < p.N; ++k)
          if (k != p.mode) prod *= fac[p.foff[k] + (int64_t)idx[k * kTile + cc] * p.R + r];
      }
      Bs[cc * RB + rr] = prod;
    }
    // tensor tile, transposed to [cc][i]
    if (p.I_right == 1) {
      for (int e = tid; e < kTile * IC; e += kThreads) {
        const int ii = e % IC, cc = e / IC;
        CT v = CT(0);
        if (cc < len && ii < rows) v = (CT)T[base[cc] + (i0 + ii)];
        Ts[cc * TS + ii] = v;
      }
    } else {
      for (int e = tid; e < kTile * IC; e += kThreads) {
        const int cc = e % kTile, ii = e / kTile;
        CT v = CT(0);
        if (cc < len && ii < rows) v = (CT)T[base[cc] + (i0 + ii) * p.I_right];
        Ts[cc * TS + ii] = v;
      }
    }
    __syncthreads();
    for (int cc = g; cc < len; cc += 4) {
      CT b[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) b[r] = Bs[cc * RB + r];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const CT x = Ts[cc * TS + lane + 64 * s];
#pragma unroll
        for (int r = 0; r < RB; ++r) acc[s][r] = fma(x, b[r], acc[s][r]);
      }
    }
    __syncthreads();
  }

  // Reduce the four column groups in a fixed order: (0+2) + (1+3), then 0 + 1.
  CT* red = reinterpret_cast<CT*>(lds);   // 2 x [IC][RB]
  if (g >= 2) {
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int r = 0; r < RB; ++r) red[((g - 2) * IC + lane + 64 * s) * RB + r] = acc[s][r];
  }
  __syncthreads();
  if (g < 2) {
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int r = 0; r < RB; ++r) acc[s][r] += red[(g * IC + lane + 64 * s) * RB + r];
  }
  __syncthreads();
  if (g == 1) {
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int r = 0; r < RB; ++r) red[(lane + 64 * s) * RB + r] = acc[s][r];
  }
  __syncthreads();
  if (g == 0) {
    double* out = part + (int64_t)blockIdx.x * p.I_n * p.R;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int ii = lane + 64 * s;
      if (ii < rows) {
#pragma unroll
        for (int r = 0; r < RB; ++r)
          if (r0 + r < p.R)
            out[(i0 + ii) * p.R + r0 + r] = (double)(acc[s][r] + red[ii * RB + r]);
      }
    }
  }
}

__global__ void to_f32_kernel(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = (float)x[e];
}

template <typename TT, typename CT, int RB, int S>
int launch_vec(cp_handle* h, const TT* T, const CT* fac, DenseParams p, double* M,
               hipStream_t st) {
  constexpr int IC = 64 * S;
  const int64_t ichunks = (p.I_n + IC - 1) / IC;
  const int64_t rchunks = (p.R + RB - 1) / RB;
  const int64_t target = 1024;
  int64_t ks = (target + ichunks * rchunks - 1) / (ichunks * rchunks);
  ks = std::max<int64_t>(1, std::min<int64_t>(ks, p.ntiles));
  p.tiles_per_block = (p.ntiles + ks - 1) / ks;
  ks = (p.ntiles + p.tiles_per_block - 1) / p.tiles_per_block;
  p.ksplit = ks;
  const int64_t n_out = p.I_n * p.R;
  CP_TRY(ensure(h, h->part, sizeof(double) * (size_t)(ks * n_out), st));
  double* part = static_cast<double*>(h->part.ptr);
  dim3 grid((unsigned)ks, (unsigned)ichunks, (unsigned)rchunks);
  {
    KernelTimer timer(h, dense_kernel_id<CT>(), st);
    CP_TIMED_LAUNCH(timer, (mttkrp_vec_kernel<TT, CT, RB, S>), grid, dim3(kThreads), 0, st, T, fac, p,
                       part);
  }
  CP_LAUNCH_CHECK(h);
  CP_TRY(launch_splitk_reduce(h, part, ks, n_out, p.R, M, st));
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

template <typename TT, typename CT>
int dispatch_rank(cp_handle* h, const TT* T, const CT* fac, const DenseParams& p, double* M,
                  hipStream_t st) {
  const bool two = p.I_n > 64;
  if (p.R <= 8) return two ? launch_vec<TT, CT, 8, 2>(h, T, fac, p, M, st)
                           : launch_vec<TT, CT, 8, 1>(h, T, fac, p, M, st);
  if (p.R <= 16) return two ? launch_vec<TT, CT, 16, 2>(h, T, fac, p, M, st)
                            : launch_vec<TT, CT, 16, 1>(h, T, fac, p, M, st);
  if (sizeof(CT) == 8) return launch_vec<TT, CT, 32, 1>(h, T, fac, p, M, st);
  return two ? launch_vec<TT, CT, 32, 2>(h, T, fac, p, M, st)
             : launch_vec<TT, CT, 32, 1>(h, T, fac, p, M, st);
}


// ---- BF16x3 on MFMA ----------------------------------------------------------
// x = hi + lo with hi = bf16(x) (round to nearest even) and lo = bf16(x - hi);
// x*y ~ hi_x hi_y + hi_x lo_y + lo_x hi_y, each product exact in float32 on the
// matrix cores, float32 accumulation.  The dropped lo*lo term and the rounding
// of lo are below 2^-16 relative per product.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline void split_bf16(float x, uint16_t& hi, uint16_t& lo) {
  hi = bf16_rne(x);
  const float rem = x - __uint_as_float((uint32_t)hi << 16);   // exact
  lo = bf16_rne(rem);
}

constexpr int kKS = 72;   // padded LDS row length (bf16) of a 64-wide tile row

// Workgroup: 4 waves, 64*S rows x 32 ranks.  Wave w owns row tiles
// {S*w .. S*w+S-1} (16 rows each) and both 16-rank column tiles.
// v_mfma_f32_16x16x32_bf16 operand layout: A lane l holds row l%16, k =
// 8*(l/16)..+7; B lane l holds column l%16, same k; D lane l holds rows
// 4*(l/16)..+3 of column l%16.
template <int S>
__global__ __launch_bounds__(kThreads) void mttkrp_bf16x3_kernel(const float* __restrict__ T,
                                                                 const float* __restrict__ fac,
                                                                 DenseParams p,
                                                                 double* __restrict__ part) {
  constexpr int IC = 64 * S;
  __shared__ __align__(16) uint16_t Thi[IC * kKS];
  __shared__ __align__(16) uint16_t Tlo[IC * kKS];
  __shared__ __align__(16) uint16_t Bhi[32 * kKS];
  __shared__ __align__(16) uint16_t Blo[32 * kKS];
  __shared__ int32_t idx[CP_MAX_ORDER * kTile];
  __shared__ int64_t base[kTile];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.y * IC;
  const int rows = (int)min<int64_t>(IC, p.I_n - i0);
  const int r0 = blockIdx.z * 32;

  floatx4 acc[S][2];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[s][c] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int64_t t_begin = (int64_t)blockIdx.x * p.tiles_per_block;
  const int64_t t_end = min<int64_t>(p.ntiles, t_begin + p.tiles_per_block);
  for (int64_t t = t_begin; t < t_end; ++t) {
    const int64_t c0 = t * kTile;
    const int len = (int)min<int64_t>(kTile, p.C - c0);
    if (tid < len) decompose(p, c0 + tid, tid, idx, base);
    __syncthreads();
    for (int e = tid; e < kTile * 32; e += kThreads) {
      const int cc = e & (kTile - 1), rr = e >> 6;
      const int r = r0 + rr;
      float prod = 0.f;
      if (cc < len && r < p.R) {
        prod = 1.f;
        for (int k = 0; k < p.N; ++k)
          if (k != p.mode) prod *= fac[p.foff[k] + (int64_t)idx[k * kTile + cc] * p.R + r];
      }
      uint16_t hi, lo;
      split_bf16(prod, hi, lo);
      Bhi[rr * kKS + cc] = hi;
      Blo[rr * kKS + cc] = lo;
    }
    if (p.I_right == 1) {
      for (int e = tid; e < kTile * IC; e += kThreads) {
        const int ii = e % IC, cc = e / IC;
        float v = 0.f;
        if (cc < len && ii < rows) v = T[base[cc] + (i0 + ii)];
        uint16_t hi, lo;
        split_bf16(v, hi, lo);
        Thi[ii * kKS + cc] = hi;
        Tlo[ii * kKS + cc] = lo;
      }
    } else {
      for (int e = tid; e < kTile * IC; e += kThreads) {
        const int cc = e % kTile, ii = e / kTile;
        float v = 0.f;
        if (cc < len && ii < rows) v = T[base[cc] + (i0 + ii) * p.I_right];
        uint16_t hi, lo;
        split_bf16(v, hi, lo);
        Thi[ii * kKS + cc] = hi;
        Tlo[ii * kKS + cc] = lo;
      }
    }
    __syncthreads();
    const int lrow = lane & 15;
    const int kb = (lane >> 4) * 8;
#pragma unroll
    for (int k0 = 0; k0 < kTile; k0 += 32) {
      bf16x8 bh[2], bl[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int off = (c * 16 + lrow) * kKS + k0 + kb;
        bh[c] = *reinterpret_cast<const bf16x8*>(&Bhi[off]);
        bl[c] = *reinterpret_cast<const bf16x8*>(&Blo[off]);
      }
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int off = ((w * S + s) * 16 + lrow) * kKS + k0 + kb;
        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&Thi[off]);
        const bf16x8 al = *reinterpret_cast<const bf16x8*>(&Tlo[off]);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          acc[s][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[c], acc[s][c], 0, 0, 0);
          acc[s][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[c], acc[s][c], 0, 0, 0);
          acc[s][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[c], acc[s][c], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  double* out = part + (int64_t)blockIdx.x * p.I_n * p.R;
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int r = r0 + c * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ii = (w * S + s) * 16 + (lane >> 4) * 4 + q;
        if (ii < rows && r < p.R) out[(i0 + ii) * p.R + r] = (double)acc[s][c][q];
      }
    }
}

template <int S>
int launch_bf16x3(cp_handle* h, const float* T, const float* fac, DenseParams p, double* M,
                  hipStream_t st) {
  constexpr int IC = 64 * S;
  const int64_t ichunks = (p.I_n + IC - 1) / IC;
  const int64_t rchunks = (p.R + 31) / 32;
  const int64_t target = 1024;
  int64_t ks = (target + ichunks * rchunks - 1) / (ichunks * rchunks);
  ks = std::max<int64_t>(1, std::min<int64_t>(ks, p.ntiles));
  p.tiles_per_block = (p.ntiles + ks - 1) / ks;
  ks = (p.ntiles + p.tiles_per_block - 1) / p.tiles_per_block;
  p.ksplit = ks;
  const int64_t n_out = p.I_n * p.R;
  CP_TRY(ensure(h, h->part, sizeof(double) * (size_t)(ks * n_out), st));
  double* part = static_cast<double*>(h->part.ptr);
  dim3 grid((unsigned)ks, (unsigned)ichunks, (unsigned)rchunks);
  {
    KernelTimer timer(h, CP_KERNEL_DENSE_MTTKRP, st);
    CP_TIMED_LAUNCH(timer, (mttkrp_bf16x3_kernel<S>), grid, dim3(kThreads), 0, st, T, fac, p, part);
  }
  CP_LAUNCH_CHECK(h);
  CP_TRY(launch_splitk_reduce(h, part, ks, n_out, p.R, M, st));
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

DenseParams make_params(const Shape& s, int R, int mode) {
  DenseParams p{};
  p.N = s.N;
  p.mode = mode;
  p.R = R;
  for (int k = 0; k < s.N; ++k) {
    p.dims[k] = s.dims[k];
    p.foff[k] = s.off[k] * R;
  }
  p.I_left = 1;
  for (int k = 0; k < mode; ++k) p.I_left *= s.dims[k];
  p.I_n = s.dims[mode];
  p.I_right = 1;
  for (int k = mode + 1; k < s.N; ++k) p.I_right *= s.dims[k];
  p.C = p.I_left * p.I_right;
  p.ntiles = (p.C + kTile - 1) / kTile;
  return p;
}

}  // namespace

int stage_factors_f32(cp_handle* h, const double* u, int64_t L, float** out, hipStream_t st) {
  CP_TRY(ensure(h, h->stage, sizeof(float) * (size_t)L, st));
  float* y = static_cast<float*>(h->stage.ptr);
  if (L > 0) {
    hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, st, u, y, L);
    CP_LAUNCH_CHECK(h);
  }
  *out = y;
  return CP_OK;
}

int dense_mttkrp(cp_handle* h, const cp_tensor* T, const Shape& s, const double* u, int R,
                 int mode, int prec, double* M, hipStream_t st) {
  h->t_passes++;
  DenseParams p = make_params(s, R, mode);
  const int64_t L = s.sum_dims() * R;

  if (prec == CP_PREC_FP32 || prec == CP_PREC_BF16X3) {
    if (T->dtype != CP_F32)
      return fail(h, CP_EINVAL, "precision FP32/BF16X3 needs a float32 tensor");
    float* fac = nullptr;
    if (prec == CP_PREC_BF16X3) {
      // the matrix-core streaming kernels (which stage the float32 factors
      // in their table launch); shapes they do not cover (inner length not
      // a multiple of 8 or above 512) take the float32 vector kernels, which
      // are faster than the generic BF16x3 tiles there and at least as
      // accurate; the generic tiles are the last resort
      const float* Tv = static_cast<const float*>(T->values);
      int rc = dense_fast_bf16x3(h, Tv, u, s, R, mode, M, st);
      if (rc <= 0) return rc;   // launched (CP_OK) or failed
      CP_TRY(stage_factors_f32(h, u, L, &fac, st));
      rc = dense_fast_vec<float, float>(h, Tv, fac, s, R, mode, M, st);
      if (rc <= 0) return rc;
      return p.I_n > 64 ? launch_bf16x3<2>(h, Tv, fac, p, M, st)
                        : launch_bf16x3<1>(h, Tv, fac, p, M, st);
    }
    // float32 products: the matrix-core streaming kernels, else the vector ones
    {
      const int rc = dense_fast_mfma_f32(h, static_cast<const float*>(T->values), u, s, R, mode, M, st);
      if (rc <= 0) return rc;
    }
    CP_TRY(stage_factors_f32(h, u, L, &fac, st));
    {
      const int rc = dense_fast_vec<float, float>(h, static_cast<const float*>(T->values), fac, s, R,
                                                  mode, M, st);
      if (rc <= 0) return rc;
    }
    return dispatch_rank<float, float>(h, static_cast<const float*>(T->values), fac, p, M, st);
  }
  if (T->dtype == CP_F32) {
    // float64 products and sums of the widened float32 tensor: the matrix-core
    // streaming kernels (v_mfma_f64_16x16x4_f64), else the vector ones
    int rc = dense_fast_mfma_f64acc(h, static_cast<const float*>(T->values), u, s, R, mode, M, st);
    if (rc <= 0) return rc;
    rc = dense_fast_vec<float, double>(h, static_cast<const float*>(T->values), u, s, R, mode, M, st);
    if (rc <= 0) return rc;
    return dispatch_rank<float, double>(h, static_cast<const float*>(T->values), u, p, M, st);
  }
  {
    const int rc = dense_fast_vec<double, double>(h, static_cast<const double*>(T->values), u, s, R,
                                                  mode, M, st);
    if (rc <= 0) return rc;
  }
  return dispatch_rank<double, double>(h, static_cast<const double*>(T->values), u, p, M, st);
}

}  // namespace cpng
