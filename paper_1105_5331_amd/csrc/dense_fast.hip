// Streaming dense MTTKRP on the gfx950 matrix cores (BF16x3), for the two
// regular layouts that cover every mode of a C-order tensor whose innermost
// contracted mode has a length divisible by 8.
//
// Both kernels split the contraction of M^(n) = T_(n) Phibar^(n)  (Section 2.3)
// into an inner sum over one "inner" mode q and an outer sum over the rest:
//     M(i, r) = sum_o P(o, r) * Y_o(i, r),   Y_o(i, r) = sum_k T(o, i, k) A^(q)(k, r),
//     P(o, r) = prod_{modes m outside {n, q}} A^(m)(i_m(o), r).
// The inner factor A^(q) is the same for every o: it is split into bf16
// hi + lo once per workgroup and kept in LDS.  Y_o is a small GEMM on MFMA
// (v_mfma_f32_16x16x32_bf16, three products hi*hi + hi*lo + lo*hi, float32
// accumulation); the P(o, r) scaling is one FMA per accumulator.  The tensor
// is read exactly once, with non-temporal loads that each cover whole
// 128-byte lines, and split into bf16 hi + lo in registers.
//
//  * row kernels (n < N-1): inner mode q = N-1, contiguous in memory.  The A
//    operand is 8 consecutive k of a row per lane (rows l % 16), so only four
//    lanes share a row: each wave reads its k-step rows as whole lines into
//    registers, writes them to its own LDS area and reads the operands back
//    (wave-level ordering only).
//  * column kernel (n = N-1): inner mode q = N-2; the output index i is the
//    contiguous one.  The MFMA computes Y^T = A^(q)^T T_o with the factor as
//    the A operand (from LDS) and the tensor as the B operand: lane l reads
//    8 rows k of two adjacent columns i, straight into registers (16 lanes
//    read a whole line per k-row).
//
// Split-K over workgroups (blockIdx.x owns a contiguous range of outer
// indices o); each workgroup writes its float32 partial sums to its own
// slot; a second kernel adds the slots in slot order in float64.  No atomics.
#include "common.hpp"
#include "splitk.hpp"

#include <algorithm>
#include <type_traits>

namespace cpng {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef bf16x4 __attribute__((address_space(3)))* lds_bf16x4_p;
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kThr = 256;

// Tuning knobs (compile-time): workgroups per launch of the streaming
// kernels, and how many (outer index, k-step) operands each lane keeps in
// flight ahead of the MFMAs that consume them (1 or 2).
#ifndef CPNG_STREAM_BLOCKS
#define CPNG_STREAM_BLOCKS 1024
#endif
#ifndef CPNG_PREFETCH
#define CPNG_PREFETCH 1
#endif
#ifndef CPNG_ROWSTREAM_TW
#define CPNG_ROWSTREAM_TW 2
#endif

struct FastParams {
  int R;
  int nout;                          // number of outer modes
  int64_t ostride[CP_MAX_ORDER];     // element stride of each outer mode in T
  int64_t odims[CP_MAX_ORDER];
  int64_t ofoff[CP_MAX_ORDER];       // factor offsets (elements) of the outer modes
  int64_t qfoff;                     // factor offset of the inner mode
  int64_t I_n;                       // output rows
  int64_t K;                         // inner length (multiple of 8)
  int64_t istride;                   // stride of the output index in T (row kernel)
  int64_t kstride;                   // stride of the inner index in T (column kernel)
  int64_t O;                         // number of outer indices
  int64_t o_per_block;
  int kpad;                          // LDS row length (bf16) of the staged inner factor
  int nks;                           // K steps of 32
  int vec_ok;                        // wide loads along the unit-stride index are aligned
  int64_t Opad;                      // O rounded up to 4
  int ptrans;                        // P table rank-major (row-stream kernel) or o-major
};

__device__ inline void split8(const float (&v)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const __bf16 h = (__bf16)v[j];
    hi[j] = h;
    lo[j] = (__bf16)(v[j] - (float)h);   // v - h is exact in float32
  }
}

// ---- operand flavours of the streaming kernels ------------------------------
// For one 16x16 tile and one 32-wide k-step every lane holds the eight
// values k = 8g..8g+7 (g = lane / 16) of its tensor row (or column) and of its
// factor column; a flavour multiplies the two lane sets on the matrix cores
// and adds into the tile.  Any fixed grouping of the k's is a valid order of
// the sum, so the three flavours share the data movement:
//  * FlavBF16x3: each operand split into bf16 hi + lo, hi*hi + hi*lo + lo*hi
//    with one v_mfma_f32_16x16x32_bf16 each (float32 accumulation);
//  * FlavF32: float32 operands, eight v_mfma_f32_16x16x4_f32 (value j of every
//    lane in the j-th), float32 accumulation;
//  * FlavF64: the float32 tensor values widened exactly to float64, float64
//    factors, eight v_mfma_f64_16x16x4_f64 (float64 products and sums).
// The inner factor is staged in LDS as [r][kpad] in the flavour's form.
// Operand layouts are the same for all three (lane l: row or column l % 16,
// k group l / 16); the result tile's rows differ (drow).
typedef double doublex4 __attribute__((ext_vector_type(4)));

struct FlavBF16x3 {
  using S = float;     // outer scales, accumulators, per-workgroup partial sums
  // the two-sided kernel stages its tensor chunks already split into bf16
  // hi and lo planes (each value split once instead of once per operand)
  static constexpr bool kPreSplit = true;
  using V = floatx4;   // one MFMA tile: 4 values per lane
  using Src = float;   // factor values staged (the float32 copy)
  static constexpr int kMaxK = 512;
  static constexpr int kFacBytes = 2 * sizeof(__bf16);   // LDS bytes per staged value
  // padding (values) of a staged factor row: rows of an odd number of 16-byte
  // bank groups, so the 16 rows one operand read touches meet 16 groups
  static constexpr int kPad = 8;
  // row of the 16x16 tile held by result value q of lane group g (lane / 16)
  __device__ static int drow(int g, int q) { return 4 * g + q; }
  struct Op {
    bf16x8 h, l;
  };
  __device__ static Op from_t(const float (&v)[8]) {
    Op o;
    split8(v, o.h, o.l);
    return o;
  }
  __device__ static Op from_lds(const unsigned char* lds, int kpad, int off) {
    const __bf16* Sh = reinterpret_cast<const __bf16*>(lds);
    return Op{*reinterpret_cast<const bf16x8*>(Sh + off),
              *reinterpret_cast<const bf16x8*>(Sh + 32 * kpad + off)};
  }
  __device__ static void put(unsigned char* lds, int kpad, int r, int k, float v) {
    __bf16* Sh = reinterpret_cast<__bf16*>(lds);
    const __bf16 h = (__bf16)v;
    Sh[r * kpad + k] = h;
    Sh[32 * kpad + r * kpad + k] = (__bf16)(v - (float)h);
  }
  // the products of one tile, in order: hi*hi, hi*lo, lo*hi
  static constexpr int kSteps = 3;
  __device__ static V mma_step(const Op& a, const Op& b, int j, V c) {
    if (j == 0) return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, c, 0, 0, 0);
    if (j == 1) return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.l, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l, b.h, c, 0, 0, 0);
  }
};

struct FlavF32 {
  using S = float;
  static constexpr bool kPreSplit = false;
  using V = floatx4;
  using Src = float;
  static constexpr int kMaxK = 512;
  static constexpr int kFacBytes = sizeof(float);
  static constexpr int kPad = 4;
  __device__ static int drow(int g, int q) { return 4 * g + q; }
  struct Op {
    float x[8];
  };
  __device__ static Op from_t(const float (&v)[8]) {
    Op o;
#pragma unroll
    for (int j = 0; j < 8; ++j) o.x[j] = v[j];
    return o;
  }
  __device__ static Op from_lds(const unsigned char* lds, int, int off) {
    const float* S = reinterpret_cast<const float*>(lds) + off;
    const floatx4 a = *reinterpret_cast<const floatx4*>(S);
    const floatx4 b = *reinterpret_cast<const floatx4*>(S + 4);
    return Op{{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]}};
  }
  __device__ static void put(unsigned char* lds, int kpad, int r, int k, float v) {
    reinterpret_cast<float*>(lds)[r * kpad + k] = v;
  }
  static constexpr int kSteps = 8;
  __device__ static V mma_step(const Op& a, const Op& b, int j, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a.x[j], b.x[j], c, 0, 0, 0);
  }
};

struct FlavF64 {
  using S = double;
  static constexpr bool kPreSplit = false;
  using V = doublex4;
  using Src = double;   // the float64 factors themselves
  static constexpr int kMaxK = 256;
  static constexpr int kFacBytes = sizeof(double);
  static constexpr int kPad = 2;
  // the float64 16x16 result interleaves its rows: value q of group g is row g + 4q
  __device__ static int drow(int g, int q) { return g + 4 * q; }
  struct Op {
    double x[8];
  };
  __device__ static Op from_t(const float (&v)[8]) {
    Op o;
#pragma unroll
    for (int j = 0; j < 8; ++j) o.x[j] = (double)v[j];
    return o;
  }
  __device__ static Op from_lds(const unsigned char* lds, int, int off) {
    typedef double d2v __attribute__((ext_vector_type(2)));
    const double* S = reinterpret_cast<const double*>(lds) + off;
    Op o;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const d2v x = *reinterpret_cast<const d2v*>(S + 2 * j);
      o.x[2 * j] = x[0];
      o.x[2 * j + 1] = x[1];
    }
    return o;
  }
  __device__ static void put(unsigned char* lds, int kpad, int r, int k, double v) {
    reinterpret_cast<double*>(lds)[r * kpad + k] = v;
  }
  static constexpr int kSteps = 8;
  __device__ static V mma_step(const Op& a, const Op& b, int j, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a.x[j], b.x[j], c, 0, 0, 0);
  }
};

__device__ inline float fma_s(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double fma_s(double a, double b, double c) { return fma(a, b, c); }

// Stage the inner factor, columns r0..r0+31: S[r][k] = A^(q)(k, r0 + r) in the
// flavour's form, zero for r >= R and for k in [K, 32 * nks).
// First inner index (within a 32-wide k-step) of lane group g's operand:
// the MFMA operand of g is k = 8g..8g+7.
__device__ inline int kload_a(int g) { return 8 * g; }

template <class F>
__device__ inline void stage_inner(const typename F::Src* __restrict__ fac, const FastParams& p,
                                   int r0, unsigned char* lds) {
  const int kr = p.nks * 32;
  for (int e = threadIdx.x; e < 32 * kr; e += kThr) {
    const int k = e >> 5, r = e & 31;
    typename F::Src v = 0;
    if (k < p.K && r0 + r < p.R) v = fac[p.qfoff + (int64_t)k * p.R + r0 + r];
    F::put(lds, p.kpad, r, k, v);
  }
}

// Base offset of outer index o in T and the scale P(o, r) for one rank r.
__device__ inline int64_t outer_base(const FastParams& p, int64_t o) {
  int64_t base = 0;
  for (int m = p.nout - 1; m >= 0; --m) {
    const int64_t d = p.odims[m];
    const int64_t q = o / d;
    base += (o - q * d) * p.ostride[m];
    o = q;
  }
  return base;
}

// the product of the outer modes' factor values in S: for S = float each
// float64 factor value is rounded to float32 first (the same bits as reading
// the float32 copy), for S = double the values are used as they are
template <typename S>
__device__ inline S outer_scale(const double* __restrict__ fac, const FastParams& p, int64_t o,
                                int r) {
  if (r >= p.R) return S(0);
  S s = S(1);
  for (int m = p.nout - 1; m >= 0; --m) {
    const int64_t d = p.odims[m];
    const int64_t q = o / d;
    s *= (S)fac[p.ofoff[m] + (o - q * d) * p.R + r];
    o = q;
  }
  return s;
}

constexpr int kOChunk = 64;   // outer indices per LDS table chunk (VALU kernel)

// Outer-index tables of one launch: base offset of every outer index o and
// the scales P(o, r) = prod_{outer modes m} A^(m)(i_m(o), r) for all r < R.
// Computed once here instead of in every workgroup.
// P table: o-major Pg[o * R + r] for the row and column kernels, which read
// one o for many ranks; rank-major Pg[r * Opad + o] (zero for o >= O) for the
// row-stream kernel, whose MFMA D lanes hold four consecutive o of one rank
// (one 16-byte load).
// The same launch also writes the float32 copy of all L factor values
// (fac32, read by the float32-operand kernels for their inner mode; L = 0
// for the float64 flavour, which reads the factors themselves).
template <typename S>
__global__ void outer_tables_kernel(const double* __restrict__ fac, FastParams p,
                                    S* __restrict__ Pg, int64_t* __restrict__ bg,
                                    float* __restrict__ fac32, int64_t L) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < L) fac32[e] = (float)fac[e];
  const int64_t o = e / (p.R + 1);
  const int c = (int)(e - o * (p.R + 1));
  if (o >= p.Opad) return;
  if (c == p.R) {
    if (o < p.O) bg[o] = outer_base(p, o);
  } else if (p.ptrans) {
    Pg[c * p.Opad + o] = o < p.O ? outer_scale<S>(fac, p, o, c) : S(0);
  } else if (o < p.O) {
    Pg[o * p.R + c] = outer_scale<S>(fac, p, o, c);
  }
}

// P(o, r) from the o-major table (row and column kernels)
template <typename S>
__device__ inline S pscale(const S* __restrict__ Pg, const FastParams& p, int64_t o, int r) {
  return r < p.R ? Pg[o * p.R + r] : S(0);
}

// P(o, r) from the rank-major table (row-stream kernel)
template <typename S>
__device__ inline S pscale_t(const S* __restrict__ Pg, const FastParams& p, int64_t o, int r) {
  return r < p.R ? Pg[r * p.Opad + o] : S(0);
}

// P(o..o+3, r) from the rank-major table, o a multiple of 4 (Opad is, so the
// address is 4-element aligned)
template <typename S>
struct S4 {
  S x, y, z, w;
};
__device__ inline S4<float> pscale4(const float* __restrict__ Pg, const FastParams& p, int64_t o,
                                    int r) {
  if (r >= p.R) return S4<float>{0.f, 0.f, 0.f, 0.f};
  const float4 v = *reinterpret_cast<const float4*>(Pg + r * p.Opad + o);
  return S4<float>{v.x, v.y, v.z, v.w};
}
__device__ inline S4<double> pscale4(const double* __restrict__ Pg, const FastParams& p, int64_t o,
                                     int r) {
  if (r >= p.R) return S4<double>{0.0, 0.0, 0.0, 0.0};
  const double2 a = *reinterpret_cast<const double2*>(Pg + r * p.Opad + o);
  const double2 b = *reinterpret_cast<const double2*>(Pg + r * p.Opad + o + 2);
  return S4<double>{a.x, a.y, b.x, b.y};
}

// 16-byte load of T; NTR: non-temporal (rows are whole 128-byte lines)
template <bool NTR>
__device__ inline floatx4 load_t4(const float* ptr) {
  if constexpr (NTR) return __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(ptr));
  else return *reinterpret_cast<const floatx4*>(ptr);
}

// Row kernel: 4 waves x MT row tiles of 16 = 64*MT rows, 32 ranks.
template <class F, int MT, bool NTR>
__global__ __launch_bounds__(kThr) void mttkrp_rows_mfma(const float* __restrict__ T,
                                                         const typename F::Src* __restrict__ fac,
                                                         const typename F::S* __restrict__ Pg,
                                                         const int64_t* __restrict__ bg,
                                                         FastParams p,
                                                         typename F::S* __restrict__ part) {
  using S = typename F::S;
  using V = typename F::V;
  using Op = typename F::Op;
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int lr = lane & 15;
  const int kb = (lane >> 4) * 8;
  const int r0 = blockIdx.z * 32;
  const int64_t i0 = (int64_t)blockIdx.y * (64 * MT);
  constexpr int kRS = 36;              // staging row stride (floats)
  constexpr int NQ = 16 * MT * 8 / 64; // 16-byte loads per lane per k-step
  float* stg = reinterpret_cast<float*>(dyn_lds + (size_t)F::kFacBytes * 32 * p.kpad) +
               w * (16 * MT * kRS);
  stage_inner<F>(fac, p, r0, dyn_lds);
  __syncthreads();

  // whole-line loads: lane l reads 16 bytes at chunk l % 8 of the wave's rows
  // q*8 + l/8 (output rows i0 + 16 MT w + that)
  typedef float f4v __attribute__((ext_vector_type(4)));
  int64_t lrowoff[NQ];
  bool lrowok[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int64_t i = i0 + (int64_t)w * MT * 16 + q * 8 + (lane >> 3);
    lrowok[q] = i < p.I_n;
    lrowoff[q] = lrowok[q] ? i * p.istride : 0;
  }
  const int c4 = (lane & 7) * 4;
  auto gload = [&](int64_t base, int k0, f4v (&dst)[NQ]) {
    const int k = k0 + c4;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      dst[q] = (lrowok[q] && k < p.K)
                   ? load_t4<NTR>(T + base + lrowoff[q] + k) : f4v{0.f, 0.f, 0.f, 0.f};
  };
  V acc[MT][2];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = V{0, 0, 0, 0};

  const int64_t ob = (int64_t)blockIdx.x * p.o_per_block;
  const int64_t oe = min<int64_t>(p.O, ob + p.o_per_block);
  {
    const int64_t oc = ob;
    const int nc = (int)(oe - ob);
    const int64_t* base_tab = bg + oc;
    const int nit = nc * p.nks;
    // load ring: buf[0] is consumed this iteration, buf[1..PF] are in flight
    constexpr int PF = CPNG_PREFETCH;
    f4v buf[PF + 1][NQ];
    int jl = 0, kl = 0;   // (outer, k-step) of the next load
#pragma unroll
    for (int b = 0; b < PF; ++b) {
      if (b < nit) gload(base_tab[jl], kl * 32, buf[b]);
      if (++kl == p.nks) { kl = 0; ++jl; }
    }
    V Y[MT][2];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) Y[mt][nt] = V{0, 0, 0, 0};
    int j = 0, ks = 0;
    for (int it = 0; it < nit; ++it) {
      if (it + PF < nit) gload(base_tab[jl], kl * 32, buf[PF]);
      if (++kl == p.nks) { kl = 0; ++jl; }
      // stage the step's rows, then read back this lane's operands (8 k of a row)
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        *reinterpret_cast<f4v*>(stg + (q * 8 + (lane >> 3)) * kRS + c4) = buf[0][q];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      float v[MT][8];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const f4v a = *reinterpret_cast<const f4v*>(stg + (mt * 16 + lr) * kRS + kb);
        const f4v b = *reinterpret_cast<const f4v*>(stg + (mt * 16 + lr) * kRS + kb + 4);
        v[mt][0] = a.x; v[mt][1] = a.y; v[mt][2] = a.z; v[mt][3] = a.w;
        v[mt][4] = b.x; v[mt][5] = b.y; v[mt][6] = b.z; v[mt][7] = b.w;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      Op a[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) a[mt] = F::from_t(v[mt]);
      const int k = ks * 32 + kb;
      const Op b0 = F::from_lds(dyn_lds, p.kpad, lr * p.kpad + k);
      const Op b1 = F::from_lds(dyn_lds, p.kpad, (16 + lr) * p.kpad + k);
      // tile by tile, each tile's products in order (issuing step j of every
      // tile before step j + 1 of any measured no faster for FP32 and FP64
      // and slowed the BF16x3 row kernel from 172 to 220 us at 128^4)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
        for (int js = 0; js < F::kSteps; ++js) Y[mt][0] = F::mma_step(a[mt], b0, js, Y[mt][0]);
#pragma unroll
        for (int js = 0; js < F::kSteps; ++js) Y[mt][1] = F::mma_step(a[mt], b1, js, Y[mt][1]);
      }
      if (ks + 1 == p.nks) {
        const S P0 = pscale(Pg, p, oc + j, r0 + lr);
        const S P1 = pscale(Pg, p, oc + j, r0 + 16 + lr);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            acc[mt][0][q] = fma_s(P0, Y[mt][0][q], acc[mt][0][q]);
            acc[mt][1][q] = fma_s(P1, Y[mt][1][q], acc[mt][1][q]);
          }
          Y[mt][0] = V{0, 0, 0, 0};
          Y[mt][1] = V{0, 0, 0, 0};
        }
        ks = 0;
        ++j;
      } else {
        ++ks;
      }
#pragma unroll
      for (int b = 0; b < PF; ++b)
#pragma unroll
        for (int q = 0; q < NQ; ++q) buf[b][q] = buf[b + 1][q];
    }
  }
  S* out = part + (int64_t)blockIdx.x * p.I_n * p.R;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t i = i0 + (w * MT + mt) * 16 + F::drow(lane >> 4, q);
        const int r = r0 + nt * 16 + lr;
        if (i < p.I_n && r < p.R) out[i * p.R + r] = acc[mt][nt][q];
      }
}

// Column-kernel operand: rows k .. k+7 of the lane's NT consecutive columns
// col0 .. col0+NT-1 (column col0 + nt feeds MFMA tile nt), one NT-wide load
// per row when the group lies inside I_n and I_n is a multiple of NT (every
// row offset is a multiple of I_n, so the load is aligned).  The 2-wide load
// is non-temporal: each instruction reads whole 128-byte lines of a tensor
// that is read exactly once, so they need not stay in the caches (the last
// mode at 128^4 went from 199 to 177 us; the row kernels, whose lines are
// split over two instructions, got slower with the hint and do not use it).
template <int NT>
__device__ inline void load_cols(const float* __restrict__ T, const FastParams& p, int64_t base,
                                 int64_t col0, int k0, float (&v)[NT][8]) {
  // the lane group's 8 consecutive k-rows (K is a multiple of 8)
  const int k = k0 + kload_a((threadIdx.x & 63) >> 4);
  const float* src = T + base + (int64_t)k * p.kstride + col0;
  if (k < p.K && p.vec_ok && col0 < p.I_n) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float* s = src + (int64_t)q * p.kstride;
      if constexpr (NT == 4) {
        const float4 x = *reinterpret_cast<const float4*>(s);
        v[0][q] = x.x; v[1][q] = x.y; v[2][q] = x.z; v[3][q] = x.w;
      } else if constexpr (NT == 2) {
        typedef float f2v __attribute__((ext_vector_type(2)));
        const f2v x = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(s));
        v[0][q] = x.x; v[1][q] = x.y;
      } else {
        v[0][q] = s[0];
      }
    }
  } else {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const bool ok = k < p.K && col0 + nt < p.I_n;
#pragma unroll
      for (int q = 0; q < 8; ++q) v[nt][q] = ok ? src[(int64_t)q * p.kstride + nt] : 0.f;
    }
  }
}

// Column kernel: Y^T(r, i) = sum_k A^(q)(k, r) T(o, k, i); 4 waves x NT column
// tiles of 16 = 64*NT output rows i, 32 ranks (two 16-row MFMA tiles).
template <class F, int NT>
__global__ __launch_bounds__(kThr) void mttkrp_cols_mfma(const float* __restrict__ T,
                                                         const typename F::Src* __restrict__ fac,
                                                         const typename F::S* __restrict__ Pg,
                                                         const int64_t* __restrict__ bg,
                                                         FastParams p,
                                                         typename F::S* __restrict__ part) {
  using S = typename F::S;
  using V = typename F::V;
  using Op = typename F::Op;
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int lr = lane & 15;
  const int kb = (lane >> 4) * 8;
  const int r0 = blockIdx.z * 32;
  const int64_t i0 = (int64_t)blockIdx.y * (64 * NT);
  stage_inner<F>(fac, p, r0, dyn_lds);
  __syncthreads();

  // this lane's columns: col0 + nt for tile nt
  const int64_t col0 = i0 + (int64_t)w * 16 * NT + lr * NT;
  V acc[2][NT];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = V{0, 0, 0, 0};

  const int64_t ob = (int64_t)blockIdx.x * p.o_per_block;
  const int64_t oe = min<int64_t>(p.O, ob + p.o_per_block);
  {
    const int64_t oc = ob;
    const int nc = (int)(oe - ob);
    const int64_t* base_tab = bg + oc;
    const int nit = nc * p.nks;
    constexpr int PF = CPNG_PREFETCH;
    float buf[PF + 1][NT][8];
    int jl = 0, kl = 0;
#pragma unroll
    for (int b = 0; b < PF; ++b) {
      if (b < nit) load_cols<NT>(T, p, base_tab[jl], col0, kl * 32, buf[b]);
      if (++kl == p.nks) { kl = 0; ++jl; }
    }
    V Y[2][NT];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) Y[mt][nt] = V{0, 0, 0, 0};
    int j = 0, ks = 0;
    for (int it = 0; it < nit; ++it) {
      if (it + PF < nit) load_cols<NT>(T, p, base_tab[jl], col0, kl * 32, buf[PF]);
      if (++kl == p.nks) { kl = 0; ++jl; }
      const int k = ks * 32 + kb;
      const Op a0 = F::from_lds(dyn_lds, p.kpad, lr * p.kpad + k);
      const Op a1 = F::from_lds(dyn_lds, p.kpad, (16 + lr) * p.kpad + k);
      Op b[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) b[nt] = F::from_t(buf[0][nt]);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
        for (int js = 0; js < F::kSteps; ++js) Y[0][nt] = F::mma_step(a0, b[nt], js, Y[0][nt]);
#pragma unroll
        for (int js = 0; js < F::kSteps; ++js) Y[1][nt] = F::mma_step(a1, b[nt], js, Y[1][nt]);
      }
      if (ks + 1 == p.nks) {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const S P = pscale(Pg, p, oc + j, r0 + mt * 16 + F::drow(lane >> 4, q));
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mt][nt][q] = fma_s(P, Y[mt][nt][q], acc[mt][nt][q]);
          }
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) Y[mt][nt] = V{0, 0, 0, 0};
        }
        ks = 0;
        ++j;
      } else {
        ++ks;
      }
#pragma unroll
      for (int b = 0; b < PF; ++b)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int q = 0; q < 8; ++q) buf[b][nt][q] = buf[b + 1][nt][q];
    }
  }
  S* out = part + (int64_t)blockIdx.x * p.I_n * p.R;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + mt * 16 + F::drow(lane >> 4, q);
        const int64_t i = col0 + nt;
        if (i < p.I_n && r < p.R) out[i * p.R + r] = acc[mt][nt][q];
      }
}

// Row-stream kernel (n < N-2, long contiguous runs): output rows i taken
// grid-stride by the workgroups (one staging of the inner factor serves all
// of a workgroup's rows).  For fixed i the entries T(o, i, k) of consecutive outer
// indices o are contiguous in memory (runs of I_right elements), so here the
// MFMA M dimension is the outer index: Y(o, r) = sum_k T(o, i, k) A^(q)(k, r)
// for 16 consecutive o per tile, then acc(r) += sum_o P(o, r) Y(o, r).  A
// workgroup streams a contiguous range of o instead of 128 rows far apart.
// Each wave works on TW o-tiles (16 TW outer indices) at a time; the waves
// of a workgroup take consecutive groups.  The MFMA operand layout gives
// only four lanes to a row, so loading operands directly would split every
// 128-byte line over two instructions; instead each k-step's rows are read
// as whole lines (lane l: 16 bytes at chunk l % 8 of row l / 8, one step
// ahead; non-temporal when rows are whole lines), written to the wave's own
// LDS area (row stride 36 floats)
// and read back in the operand layout, ordered by wave-level fences only
// (modes 1-2 at 128^4, R = 32: 194 -> 178 us).
template <class F, bool NTR>
__global__ __launch_bounds__(kThr) void mttkrp_rowstream_mfma(const float* __restrict__ T,
                                                              const typename F::Src* __restrict__ fac,
                                                              const typename F::S* __restrict__ Pg,
                                                              const int64_t* __restrict__ bg,
                                                              FastParams p,
                                                              typename F::S* __restrict__ part) {
  using S = typename F::S;
  using V = typename F::V;
  using Op = typename F::Op;
  constexpr int TW = CPNG_ROWSTREAM_TW;
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  __shared__ S red[4][32];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int lr = lane & 15;
  const int kb = (lane >> 4) * 8;
  const int r0 = blockIdx.z * 32;
  const int64_t bx = blockIdx.x;
  constexpr int kRS = 36;                  // staging row stride (floats)
  constexpr int NQ = 16 * TW * 8 / 64;     // 16-byte loads per lane per k-step
  float* stg = reinterpret_cast<float*>(dyn_lds + (size_t)F::kFacBytes * 32 * p.kpad) +
               w * (16 * TW * kRS);
  stage_inner<F>(fac, p, r0, dyn_lds);
  __syncthreads();
  const int64_t ob = bx * p.o_per_block;
  const int64_t oe = min<int64_t>(p.O, ob + p.o_per_block);
  for (int64_t by = blockIdx.y; by < p.I_n; by += gridDim.y) {
  const int64_t ioff = by * p.istride;
  S acc0 = 0, acc1 = 0;   // rank columns r0 + lr and r0 + 16 + lr
  for (int64_t og = ob + w * 16 * TW; og < oe; og += 4 * 16 * TW) {
    // whole-line loads: lane l reads 16 bytes at chunk l % 8 of rows q*8 + l/8
    typedef float f4v __attribute__((ext_vector_type(4)));
    const float* lrow[NQ];
    bool lok[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int64_t o = og + q * 8 + (lane >> 3);
      lok[q] = o < oe;
      lrow[q] = T + (lok[q] ? bg[o] + ioff : 0);
    }
    const int c4 = (lane & 7) * 4;
    f4v ld[NQ];
    auto gload = [&](int ks) {
      const int k = ks * 32 + c4;
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        ld[q] = (lok[q] && k < p.K)
                    ? load_t4<NTR>(lrow[q] + k) : f4v{0.f, 0.f, 0.f, 0.f};
    };
    float v[TW][8];
    gload(0);
    V Y[TW][2];
#pragma unroll
    for (int t = 0; t < TW; ++t) Y[t][0] = Y[t][1] = V{0, 0, 0, 0};
    for (int ks = 0; ks < p.nks; ++ks) {
      // stage the step's rows, then read back this lane's operand (8 k of one row)
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        *reinterpret_cast<f4v*>(stg + (q * 8 + (lane >> 3)) * kRS + c4) = ld[q];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int t = 0; t < TW; ++t) {
        const f4v a = *reinterpret_cast<const f4v*>(stg + (t * 16 + lr) * kRS + kb);
        const f4v b = *reinterpret_cast<const f4v*>(stg + (t * 16 + lr) * kRS + kb + 4);
        v[t][0] = a.x; v[t][1] = a.y; v[t][2] = a.z; v[t][3] = a.w;
        v[t][4] = b.x; v[t][5] = b.y; v[t][6] = b.z; v[t][7] = b.w;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (ks + 1 < p.nks) gload(ks + 1);
      const int k = ks * 32 + kb;
      const Op b0 = F::from_lds(dyn_lds, p.kpad, lr * p.kpad + k);
      const Op b1 = F::from_lds(dyn_lds, p.kpad, (16 + lr) * p.kpad + k);
      Op a[TW];
#pragma unroll
      for (int t = 0; t < TW; ++t) a[t] = F::from_t(v[t]);
#pragma unroll
      for (int t = 0; t < TW; ++t) {
#pragma unroll
        for (int js = 0; js < F::kSteps; ++js) Y[t][0] = F::mma_step(a[t], b0, js, Y[t][0]);
#pragma unroll
        for (int js = 0; js < F::kSteps; ++js) Y[t][1] = F::mma_step(a[t], b1, js, Y[t][1]);
      }
    }
    // D rows are outer indices og + t*16 + drow(lane/16, q); the column is
    // the rank.  og is a multiple of 4 (o_per_block is a multiple of 16), so
    // where the four rows of a lane are consecutive they are one aligned
    // group of the rank-major P table.
#pragma unroll
    for (int t = 0; t < TW; ++t) {
      const int64_t o4 = og + t * 16 + F::drow(lane >> 4, 0);
      if (F::drow(0, 1) == 1 && o4 + 3 < oe) {
        const S4<S> pa = pscale4(Pg, p, o4, r0 + lr);
        const S4<S> pb = pscale4(Pg, p, o4, r0 + 16 + lr);
        acc0 = fma_s(pa.x, Y[t][0][0], acc0);
        acc0 = fma_s(pa.y, Y[t][0][1], acc0);
        acc0 = fma_s(pa.z, Y[t][0][2], acc0);
        acc0 = fma_s(pa.w, Y[t][0][3], acc0);
        acc1 = fma_s(pb.x, Y[t][1][0], acc1);
        acc1 = fma_s(pb.y, Y[t][1][1], acc1);
        acc1 = fma_s(pb.z, Y[t][1][2], acc1);
        acc1 = fma_s(pb.w, Y[t][1][3], acc1);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t o = og + t * 16 + F::drow(lane >> 4, q);
          if (o < oe) {
            acc0 = fma_s(pscale_t(Pg, p, o, r0 + lr), Y[t][0][q], acc0);
            acc1 = fma_s(pscale_t(Pg, p, o, r0 + 16 + lr), Y[t][1][q], acc1);
          }
        }
      }
    }
  }
  // sum the four lane groups (same rank column) in a fixed order, then the waves
  acc0 += __shfl_xor(acc0, 16);
  acc0 += __shfl_xor(acc0, 32);
  acc1 += __shfl_xor(acc1, 16);
  acc1 += __shfl_xor(acc1, 32);
  if (lane < 16) {
    red[w][lr] = acc0;
    red[w][16 + lr] = acc1;
  }
  __syncthreads();
  if (threadIdx.x < 32) {
    const int c = threadIdx.x;
    const S sum = (red[0][c] + red[2][c]) + (red[1][c] + red[3][c]);
    if (r0 + c < p.R) part[bx * p.I_n * p.R + by * p.R + r0 + c] = sum;
  }
  __syncthreads();   // red is rewritten for the next row
  }
}

// ---- two-sided kernel: both group partials of an evaluation from one pass ----
// The two-level evaluation needs, at the same point, X_L = T K_R and
// X_R = T^T K_L for T seen as a P x Q matrix (rows: the left group's modes
// 0..s-1, columns: the right group's modes s..N-1; K_L, K_R the Khatri-Rao
// products of each group's factors, Section 2.3).  Both are formed here from
// ONE read of T.  Write a = (oa, j) with j the left group's last mode
// (length J) and b = (ob, k) with k the last mode (length K).  Every J x K
// slab S = T(oa, :, ob, :) adds
//     X_L(oa, j, r) += PB(ob, r) sum_k S(j, k) A^(N-1)(k, r),
//     X_R(ob, k, r) += PA(oa, r) sum_j S(j, k) A^(s-1)(j, r),
// PA and PB the products of each group's other factors (tables built once
// per launch).  Workgroup (x, y) owns GA consecutive oa and GB consecutive
// ob and walks its slabs ob by ob, oa by oa, in chunks of 32 rows j: a chunk
// is read as whole 128-byte lines (loaded two chunks ahead, in registers), stored to
// one of two LDS buffers, and one barrier per chunk orders the buffers.  In
// a chunk wave w computes the left tile of rows 16 (w / 2).., ranks
// 16 (w % 2).. over all k, and the right rows k = (K / 4) w .. over the
// chunk's 32 j for both rank tiles: the same MFMA count for every wave.  The
// left operand is 8 consecutive k of one staged row, the right one 8 rows j
// of one column k.  Left sums stay in registers for the workgroup's GA oa
// (written to partial slot y at the end), right sums for the current ob
// (written to slot x once its GA slabs are done); the slots are added in
// slot order by the fixed-order split-K reduction.  No atomics.
struct TwoParams {
  int R;
  int64_t J, K;        // lengths of modes s-1 and N-1
  int64_t OA, OB;      // outer index counts of the left and right groups
  int64_t Q;           // row stride of the P x Q view (= OB K)
  int na, nb;          // outer modes of each group
  int64_t adims[CP_MAX_ORDER], afoff[CP_MAX_ORDER];   // modes 0..s-2
  int64_t bdims[CP_MAX_ORDER], bfoff[CP_MAX_ORDER];   // modes s..N-2
  int64_t jfoff, kfoff;   // factor offsets (elements) of modes s-1 and N-1
  int64_t GB;             // ob per workgroup
  int kpadK, kpadJ;       // LDS row lengths of the two staged factors
};

// product over one group's outer modes of its factor values at outer index
// o, rank r, in S (float32: each value rounded first, as the float32 copy)
template <typename S>
__device__ inline S group_scale(const double* __restrict__ fac, int n, const int64_t* dims,
                                const int64_t* foff, int R, int64_t o, int r) {
  S s = S(1);
  for (int m = n - 1; m >= 0; --m) {
    const int64_t d = dims[m];
    const int64_t q = o / d;
    s *= (S)fac[foff[m] + (o - q * d) * R + r];
    o = q;
  }
  return s;
}

// PA (OA x R), PB (OB x R), and the float32 copy of all L factor values
template <typename S>
__global__ void twosided_tables_kernel(const double* __restrict__ fac, TwoParams p,
                                       S* __restrict__ PA, S* __restrict__ PB,
                                       float* __restrict__ fac32, int64_t L) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < L) fac32[e] = (float)fac[e];
  const int64_t na = p.OA * p.R, nb = p.OB * p.R;
  if (e < na) {
    const int64_t o = e / p.R;
    PA[e] = group_scale<S>(fac, p.na, p.adims, p.afoff, p.R, o, (int)(e - o * p.R));
  } else if (e < na + nb) {
    const int64_t e2 = e - na;
    const int64_t o = e2 / p.R;
    PB[e2] = group_scale<S>(fac, p.nb, p.bdims, p.bfoff, p.R, o, (int)(e2 - o * p.R));
  }
}

// Waves per SIMD the two-sided kernel is compiled for: two (registers <= 256)
// for float32 operands with GA <= 4, where two workgroups fit a CU's LDS;
// one otherwise (the float64 flavour's staged factors fill most of the LDS).
template <class F, int GA>
constexpr int twosided_waves() {
#ifdef CPNG_TWOSIDED_WAVES
  return CPNG_TWOSIDED_WAVES;
#else
  return (sizeof(typename F::S) == 4 && GA <= 4) ? 2 : 1;
#endif
}

// oa per workgroup of the float32-operand flavours and of the float64
// flavour (compile-time knobs; outer counts the value does not divide run
// with 2).  The partial slots written per pass are (OA / GA + OB / GB) rows
// of P or Q: with GA = 4 at 128^4 that is 101 MB instead of 151 MB (GA = 2)
// for float32 slots, and the writes cost the streaming pass more than
// their share of the bytes.
#ifndef CPNG_TWOSIDED_GA
#define CPNG_TWOSIDED_GA 4
#endif
#ifndef CPNG_TWOSIDED_GA64
#define CPNG_TWOSIDED_GA64 4
#endif

// Staging geometry of one 32 x K chunk: float32 rows of K + 4 values, or
// (pre-split flavours) a bf16 hi plane and a lo plane with rows of K + 8
// values; row j starts at j RS + RO (j / 16), RO = 16 words, so the 16 rows
// of a left tile start in 16 different 16-byte bank groups and the four lane
// groups of a right operand read (rows 8g + q, 16 consecutive columns) fall
// in four disjoint quarters of the banks.
template <class F, int K>
struct TwoStage {
  static constexpr bool PS = F::kPreSplit;
  using E = typename std::conditional<PS, __bf16, float>::type;
  static constexpr int RS = PS ? K + 8 : K + 4;
  static constexpr int RO = PS ? 32 : 16;
  static constexpr int PL = 32 * RS + RO;        // one plane, elements
  static constexpr int CH = PS ? 2 * PL : PL;    // one staging buffer, elements
  static constexpr size_t kBufBytes = sizeof(E) * (size_t)CH;
  __device__ static int radd(int j) { return j * RS + RO * (j >> 4); }
};

template <class F, int KS, int NJ, int GA>
__global__ __launch_bounds__(kThr) __attribute__((amdgpu_waves_per_eu(twosided_waves<F, GA>())))
void mttkrp_twosided_mfma(const float* __restrict__ T,
                                                             const typename F::Src* __restrict__ fac,
                                                             const typename F::S* __restrict__ PA,
                                                             const typename F::S* __restrict__ PB,
                                                             TwoParams p,
                                                             typename F::S* __restrict__ partL,
                                                             typename F::S* __restrict__ partR) {
  using S = typename F::S;
  using V = typename F::V;
  using Op = typename F::Op;
  using Src = typename F::Src;
  typedef float f4v __attribute__((ext_vector_type(4)));
  constexpr int K = 32 * KS;    // slab columns
  constexpr int KT = KS / 2;    // right row tiles per wave (K / 64)
  constexpr int KW = K / 4;     // right rows per wave
  constexpr int NL = KS;        // 16-byte loads per thread per 32 x K chunk
  using St = TwoStage<F, K>;
  using E = typename St::E;
  constexpr bool PS = St::PS;
  constexpr int PL = St::PL, CH = St::CH;
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  unsigned char* Fk = dyn_lds;
  unsigned char* Fj = dyn_lds + (size_t)F::kFacBytes * 32 * p.kpadK;
  E* stg = reinterpret_cast<E*>(Fj + (size_t)F::kFacBytes * 32 * p.kpadJ);
  // outer scales of the workgroup: PA of its GA oa, then PB of its ob range
  S* psc = reinterpret_cast<S*>(stg + 2 * CH);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int lr = lane & 15;
  const int kb = (lane >> 4) * 8;
  const int rl = (w & 1) * 16 + lr;   // this lane's rank in the left tile
  // transpose-read address of the right operand (pre-split flavours): lane
  // 4e + h of lane group g points at row 8 g + e, columns 4 h .. (the
  // group's 8 rows lie in one 16-row half, so radd adds RO (g / 2))
  const int troff = (8 * (lane >> 4) + ((lane & 15) >> 2)) * TwoStage<F, 32 * KS>::RS +
                    TwoStage<F, 32 * KS>::RO * (lane >> 5) + 4 * (lane & 3);

  // both factors, ranks 0..31 (zero beyond R), in the flavour's form
  for (int e = tid; e < 32 * K; e += kThr) {
    const int k = e >> 5, r = e & 31;
    F::put(Fk, p.kpadK, r, k, r < p.R ? fac[p.kfoff + (int64_t)k * p.R + r] : Src(0));
  }
  for (int e = tid; e < 32 * 32 * NJ; e += kThr) {
    const int j = e >> 5, r = e & 31;
    F::put(Fj, p.kpadJ, r, j, r < p.R ? fac[p.jfoff + (int64_t)j * p.R + r] : Src(0));
  }

  const int64_t oa0 = (int64_t)blockIdx.x * GA;
  const int64_t ob0 = (int64_t)blockIdx.y * p.GB;
  const int nob = (int)min<int64_t>(p.GB, p.OB - ob0);
  // The outer scales go through LDS: a global load of one inside the chunk
  // loop would sit in the same in-order memory counter as the chunk loads,
  // and waiting for it would also wait for chunk loads issued before it.
  for (int e = tid; e < (GA + nob) * 32; e += kThr) {
    const int t = e >> 5, r = e & 31;
    S v = S(0);
    if (r < p.R) v = t < GA ? PA[(oa0 + t) * p.R + r] : PB[(ob0 + t - GA) * p.R + r];
    psc[e] = v;
  }
  const int nchunk = nob * GA * NJ;
  // chunk c = ((ob - ob0) GA + (oa - oa0)) NJ + j / 32
  auto chunk_base = [&](int c) -> const float* {
    const int jc = c % NJ;
    const int t = c / NJ;
    const int64_t oa = oa0 + t % GA, ob = ob0 + t / GA;
    return T + (oa * p.J + jc * 32) * p.Q + ob * K;
  };
  // thread's share of a chunk: load l covers row l RL + tid / (K / 4),
  // columns 4 (tid % (K / 4)) .. + 3 (32 Q < 2^31: 32-bit offsets)
  constexpr int RL = kThr / (K / 4);   // rows per load instruction
  const int trow = tid / (K / 4), tcol = (tid % (K / 4)) * 4;
  const int toff = trow * (int)p.Q + tcol;
  // two chunks in flight ahead of the one being multiplied: register sets
  // ld[0], ld[1] alternate (chunk c's data in set c % 2)
  f4v ld[2][NL];
  auto gload = [&](int set, const float* base) {
#pragma unroll
    for (int l = 0; l < NL; ++l)
      ld[set][l] = __builtin_nontemporal_load(
          reinterpret_cast<const f4v*>(base + (int64_t)l * RL * p.Q + toff));
  };
  auto sstore = [&](int set, E* buf) {
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const int off = St::radd(l * RL + trow) + tcol;
      if constexpr (PS) {
        // hi = bf16(x) two at a time; the hi values back in float32 from
        // the packed word (low half shifted up, high half masked), then
        // lo = bf16(x - hi) (x - hi is exact)
        typedef unsigned u2v __attribute__((ext_vector_type(2)));
        u2v h, lo;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const float x0 = ld[set][l][2 * i], x1 = ld[set][l][2 * i + 1];
          const bf16x2 hp = {(__bf16)x0, (__bf16)x1};
          unsigned hb = __builtin_bit_cast(unsigned, hp);
          // (opaque to the optimiser, which would otherwise redo the low
          // half's conversion on its own instead of shifting the word)
          asm("" : "+v"(hb));
          const bf16x2 lp = {(__bf16)(x0 - __uint_as_float(hb << 16)),
                             (__bf16)(x1 - __uint_as_float(hb & 0xffff0000u))};
          h[i] = hb;
          lo[i] = __builtin_bit_cast(unsigned, lp);
        }
        *reinterpret_cast<u2v*>(buf + off) = h;
        *reinterpret_cast<u2v*>(buf + PL + off) = lo;
      } else {
        *reinterpret_cast<f4v*>(buf + off) = ld[set][l];
      }
    }
  };

  V accL[GA][NJ];
#pragma unroll
  for (int a = 0; a < GA; ++a)
#pragma unroll
    for (int c = 0; c < NJ; ++c) accL[a][c] = V{0, 0, 0, 0};

  // Loads and stores are issued without branches (chunk indices past the
  // end are clamped to the last chunk, whose lines are then still in the
  // caches), so that the compiler's wait before staging a register set
  // counts only that set's loads and leaves the newer set in flight.
  static_assert((GA * NJ) % 2 == 0, "chunk parity is static within an ob");
  const int last = nchunk - 1;
  gload(0, chunk_base(0));
  gload(1, chunk_base(min(1, last)));
  sstore(0, stg);
  gload(0, chunk_base(min(2, last)));
  __syncthreads();   // factors and chunk 0 staged
  // the left product's factor operands are the same for every chunk: kept
  // in registers (they were a third of the LDS reads)
  Op bk[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) bk[ks] = F::from_lds(Fk, p.kpadK, rl * p.kpadK + 32 * ks + kb);

  int c = 0;
  for (int obi = 0; obi < nob; ++obi) {
    const int64_t ob = ob0 + obi;
    const S pb = psc[(GA + obi) * 32 + rl];
    V accR[KT][2];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) accR[kt][0] = accR[kt][1] = V{0, 0, 0, 0};
#pragma unroll
    for (int ai = 0; ai < GA; ++ai) {
      V YR[KT][2];
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) YR[kt][0] = YR[kt][1] = V{0, 0, 0, 0};
#pragma unroll
      for (int jci = 0; jci < NJ; ++jci, ++c) {
        const E* cur = stg + (c & 1) * CH;
        // left: chunk rows 16 (w / 2) + lr, all k
        V YL = V{0, 0, 0, 0};
        const E* lrow = cur + St::radd(16 * (w >> 1) + lr) + kb;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          Op a;
          if constexpr (PS) {
            a.h = *reinterpret_cast<const bf16x8*>(lrow + 32 * ks);
            a.l = *reinterpret_cast<const bf16x8*>(lrow + PL + 32 * ks);
          } else {
            const f4v x0 = *reinterpret_cast<const f4v*>(lrow + 32 * ks);
            const f4v x1 = *reinterpret_cast<const f4v*>(lrow + 32 * ks + 4);
            const float v[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
            a = F::from_t(v);
          }
#pragma unroll
          for (int js = 0; js < F::kSteps; ++js) YL = F::mma_step(a, bk[ks], js, YL);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) accL[ai][jci][q] = fma_s(pb, YL[q], accL[ai][jci][q]);
        // between the two products (so that the matrix cores still work on
        // the left tile meanwhile): the next chunk (loaded two chunks ago)
        // into the other buffer, whose readers all passed the previous
        // barrier (past the last chunk this stages a copy nobody reads); then
        // the loads of chunk c + 3 into the register set it freed (c is even
        // here exactly when ai NJ + jci is: GA NJ is even)
        {
          const int set = ((ai * NJ + jci) + 1) & 1;
          sstore(set, stg + ((c + 1) & 1) * CH);
          gload(set, chunk_base(min(c + 3, last)));
        }
        // right: rows k = KW w + 16 kt + lr, the chunk's 32 j
        const Op b0 = F::from_lds(Fj, p.kpadJ, lr * p.kpadJ + 32 * jci + kb);
        const Op b1 = F::from_lds(Fj, p.kpadJ, (16 + lr) * p.kpadJ + 32 * jci + kb);
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
          Op a;
          if constexpr (PS) {
            // the operand (8 rows j of one column k) with transpose reads:
            // in each 16-lane group the read hands lane t column t of the
            // 4 x 16 block whose row e the lanes 4e .. 4e + 3 point at (4
            // values each), so lane 4e + h points at row kb + e, columns
            // 4h .. 4h + 3 of the tile; a second read covers rows kb + 4 ..
            const E* col = cur + troff + KW * w + 16 * kt;
            const bf16x4 h0 = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4_p)(col));
            const bf16x4 h1 = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4_p)(col + 4 * St::RS));
            const bf16x4 l0 = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4_p)(col + PL));
            const bf16x4 l1 = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4_p)(col + PL + 4 * St::RS));
            a.h = __builtin_shufflevector(h0, h1, 0, 1, 2, 3, 4, 5, 6, 7);
            a.l = __builtin_shufflevector(l0, l1, 0, 1, 2, 3, 4, 5, 6, 7);
          } else {
            // rows kb .. kb + 7 lie in one 16-row half: radd(kb + q) = radd(kb) + q RS
            const E* col = cur + St::radd(kb) + KW * w + 16 * kt + lr;
            float v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = col[q * St::RS];
            a = F::from_t(v);
          }
#pragma unroll
          for (int js = 0; js < F::kSteps; ++js) YR[kt][0] = F::mma_step(a, b0, js, YR[kt][0]);
#pragma unroll
          for (int js = 0; js < F::kSteps; ++js) YR[kt][1] = F::mma_step(a, b1, js, YR[kt][1]);
        }
        __syncthreads();
      }
      const S pa0 = psc[ai * 32 + lr], pa1 = psc[ai * 32 + 16 + lr];
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          accR[kt][0][q] = fma_s(pa0, YR[kt][0][q], accR[kt][0][q]);
          accR[kt][1][q] = fma_s(pa1, YR[kt][1][q], accR[kt][1][q]);
        }
    }
    // partial slots in fragment order (16 x 16 tiles of 64 lanes x 4
    // values, see splitk_frag_kernel): one 16-byte store per lane and tile
    // instead of 4-byte stores into half lines
    S* outR = partR + (int64_t)blockIdx.x * p.Q * 32;
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
        *reinterpret_cast<V*>(outR + (((ob * K + KW * w + 16 * kt) / 16) * 2 + rt) * 256 + lane * 4) =
            accR[kt][rt];
  }
  S* outL = partL + (int64_t)blockIdx.y * p.OA * p.J * 32;
#pragma unroll
  for (int ai = 0; ai < GA; ++ai)
#pragma unroll
    for (int jci = 0; jci < NJ; ++jci)
      *reinterpret_cast<V*>(outL + ((((oa0 + ai) * p.J + 32 * jci + 16 * (w >> 1)) / 16) * 2 + (w & 1)) * 256 +
                            lane * 4) = accL[ai][jci];
}

// ---- vector (VALU) streaming kernel: float32 or float64 arithmetic --------------
// Same inner/outer split, on the vector ALUs: for each outer index o and
// each 64-wide chunk of the inner mode the workgroup loads the 64 x 64 tile
// T(o, i0..i0+63, k0..k0+63) with 16-byte coalesced loads along the unit-
// stride index, stores it [k][i] in LDS, builds the Khatri-Rao tile
// B(k, r) = P(o, r) A^(q)(k0 + k, r) next to it, and every lane (one row i)
// accumulates acc(r) += T(i, k) B(k, r) over its wave's quarter of the k's.
// The steps (o, k-chunk) are software-pipelined: the tensor tile and the
// factor values of step s + 1 are loaded into registers while step s is
// computed from LDS.  The four waves are summed in a fixed order at the end.
template <typename TT, typename CT, int RB, bool ROWS>
__global__ __launch_bounds__(kThr) void mttkrp_tiles_vec(const TT* __restrict__ T,
                                                         const CT* __restrict__ fac,
                                                         FastParams p, CT* __restrict__ part) {
  constexpr int TB = 64;                 // tile edge (rows i and inner k)
  constexpr int TS = TB + 1;             // padded LDS stride
  constexpr int VE = 16 / sizeof(TT);    // elements per 16-byte load
  constexpr int NL = TB * TB / VE / kThr;   // tensor loads per thread per step
  constexpr int NB = TB * RB / kThr;        // factor values per thread per step
  static_assert(NB >= 1, "RB too small for the B tile split");
  __shared__ CT Ts[TB * TS];       // [k][i]
  __shared__ CT Bs[TB * RB];       // [k][r]
  __shared__ int64_t base_tab[kOChunk];
  __shared__ CT P_tab[kOChunk * RB];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int g = tid >> 6;
  const int r0 = blockIdx.z * RB;
  const int64_t i0 = (int64_t)blockIdx.y * TB;
  const int nkc = (int)((p.K + TB - 1) / TB);

  CT acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = CT(0);

  TT v[NL][VE];   // next tensor tile
  CT b[NB];       // next factor values A^(q)(k, r)

  // loads of step (j, kc) of the current chunk into v and b
  auto load_step = [&](int j, int kc) {
    const int64_t base = base_tab[j];
    const int64_t k0 = (int64_t)kc * TB;
#pragma unroll
    for (int t = 0; t < NL; ++t) {
      const int e = tid + t * kThr;
      if (ROWS) {   // unit stride along k
        const int ii = e / (TB / VE), kk = (e % (TB / VE)) * VE;
        const int64_t i = i0 + ii, k = k0 + kk;
        if (p.vec_ok && i < p.I_n && k + VE <= p.K) {
          const TT* src = T + base + i * p.istride + k;
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
            v[t][q] = (i < p.I_n && k + q < p.K) ? T[base + i * p.istride + k + q] : TT(0);
        }
      } else {      // unit stride along i
        const int kk = e / (TB / VE), ii = (e % (TB / VE)) * VE;
        const int64_t i = i0 + ii, k = k0 + kk;
        if (p.vec_ok && k < p.K && i + VE <= p.I_n) {
          const TT* src = T + base + k * p.kstride + i;
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
            v[t][q] = (k < p.K && i + q < p.I_n) ? T[base + k * p.kstride + i + q] : TT(0);
        }
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
  // registers -> LDS for step j (B scaled by P(o_j, r))
  auto store_step = [&](int j) {
#pragma unroll
    for (int t = 0; t < NL; ++t) {
      const int e = tid + t * kThr;
      if (ROWS) {
        const int ii = e / (TB / VE), kk = (e % (TB / VE)) * VE;
#pragma unroll
        for (int q = 0; q < VE; ++q) Ts[(kk + q) * TS + ii] = (CT)v[t][q];
      } else {
        const int kk = e / (TB / VE), ii = (e % (TB / VE)) * VE;
#pragma unroll
        for (int q = 0; q < VE; ++q) Ts[kk * TS + ii + q] = (CT)v[t][q];
      }
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int e = tid + t * kThr;
      const int kk = e / RB, rr = e - (e / RB) * RB;
      Bs[kk * RB + rr] = P_tab[j * RB + rr] * b[t];
    }
  };

  const int64_t ob = (int64_t)blockIdx.x * p.o_per_block;
  const int64_t oe = min<int64_t>(p.O, ob + p.o_per_block);
  for (int64_t oc = ob; oc < oe; oc += kOChunk) {
    const int nc = (int)min<int64_t>(kOChunk, oe - oc);
    __syncthreads();   // the previous chunk's last step is done with the tables
    for (int e = tid; e < nc * (RB + 1); e += kThr) {
      const int j = e / (RB + 1), c = e - (e / (RB + 1)) * (RB + 1);
      if (c == RB) {
        base_tab[j] = outer_base(p, oc + j);
      } else {
        CT sc = CT(0);
        if (r0 + c < p.R) {
          sc = CT(1);
          int64_t o = oc + j;
          for (int m = p.nout - 1; m >= 0; --m) {
            const int64_t d = p.odims[m];
            const int64_t q = o / d;
            sc *= fac[p.ofoff[m] + (o - q * d) * p.R + r0 + c];
            o = q;
          }
        }
        P_tab[j * RB + c] = sc;
      }
    }
    __syncthreads();   // tables complete before any wave reads them
    const int nsteps = nc * nkc;
    load_step(0, 0);
    for (int s = 0; s < nsteps; ++s) {
      const int j = s / nkc, kc = s - (s / nkc) * nkc;
      __syncthreads();   // every wave is done computing the previous step
      store_step(j);
      __syncthreads();
      if (s + 1 < nsteps) load_step((s + 1) / nkc, (s + 1) % nkc);
      const int kv = (int)min<int64_t>(TB, p.K - (int64_t)kc * TB);   // valid k of this chunk
      for (int kk = g; kk < kv; kk += 4) {
        const CT x = Ts[kk * TS + lane];
#pragma unroll
        for (int r = 0; r < RB; ++r) acc[r] = fma(x, Bs[kk * RB + r], acc[r]);
      }
    }
  }
  // fixed-order sum of the four waves: (0 + 2) + (1 + 3), then 0 + 1
  __syncthreads();
  CT* red = Ts;   // 2 x [64][RB] fits in Ts + Bs? use Ts rows 0..(2*RB-1)
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
    const int64_t i = i0 + lane;
    if (i < p.I_n) {
      CT* out = part + (int64_t)blockIdx.x * p.I_n * p.R + i * p.R;
#pragma unroll
      for (int r = 0; r < RB; ++r)
        if (r0 + r < p.R) out[r0 + r] = acc[r] + red[r * TS + lane];
    }
  }
}

// Launches one streaming MTTKRP in flavour F.  Returns CP_OK after
// launching, or 1 if the shape is not one the streaming kernels cover (the
// caller then uses another kernel).
template <class F>
int launch_mfma(cp_handle* h, const float* T, const double* u, const Shape& s, int R, int mode,
                double* M, hipStream_t st) {
  using S = typename F::S;
  constexpr bool kF32Src = sizeof(typename F::Src) == 4;
  const int N = s.N;
  if (N < 2) return 1;
  const bool rows = mode < N - 1;
  const int q = rows ? N - 1 : N - 2;
  const int64_t K = s.dims[q];
  if (K % 8 != 0 || K > F::kMaxK) return 1;
  if (reinterpret_cast<uintptr_t>(T) % 16 != 0) return 1;
  // the float32 copy of the factors (float32-operand flavours), written by
  // the table launch below; the float64 flavour reads u itself
  const int64_t L = s.sum_dims() * R;
  float* fac32 = nullptr;
  if (kF32Src) {
    CP_TRY(ensure(h, h->stage, sizeof(float) * (size_t)L, st));
    fac32 = static_cast<float*>(h->stage.ptr);
  }
  const typename F::Src* fac = nullptr;
  if constexpr (kF32Src) fac = fac32;
  else fac = u;
  FastParams p{};
  p.R = R;
  int64_t stride[CP_MAX_ORDER];
  stride[N - 1] = 1;
  for (int k = N - 2; k >= 0; --k) stride[k] = stride[k + 1] * s.dims[k + 1];
  p.nout = 0;
  p.O = 1;
  for (int k = 0; k < N; ++k) {
    if (k == mode || k == q) continue;
    p.ostride[p.nout] = stride[k];
    p.odims[p.nout] = s.dims[k];
    p.ofoff[p.nout] = s.off[k] * R;
    p.O *= s.dims[k];
    p.nout++;
  }
  p.qfoff = s.off[q] * R;
  p.I_n = s.dims[mode];
  p.K = K;
  p.istride = stride[mode];
  p.kstride = stride[q];
  p.nks = (int)((K + 31) / 32);
  p.kpad = p.nks * 32 + F::kPad;
  // rows of mode n < N-2 are runs of I_right = J' * K >= 16 K contiguous
  // elements per (left index, i): stream them one output row per workgroup.
  const bool stream_rows = rows && mode < N - 2 && (stride[mode] / K) >= 16;
  const int tile = stream_rows ? 1 : (p.I_n > 64 ? 128 : 64);
  p.ptrans = stream_rows ? 1 : 0;
  // non-temporal row loads only when every row is whole 128-byte lines: with
  // rows of other lengths a line is shared by two rows and ordinary loads
  // keep it for the second (104^4: 145 vs 166 us, 128^4: 178 vs 195 us)
  const bool ntr = K % 32 == 0;
  // column kernel: one (tile / 64)-wide load per k-row when I_n allows it
  p.vec_ok = !rows && p.I_n % (tile / 64) == 0;
  const int64_t ychunks = (p.I_n + tile - 1) / tile;
  const int64_t rchunks = (R + 31) / 32;
  const int64_t target = CPNG_STREAM_BLOCKS;
  // row-stream workgroups loop over rows: at most about `target` of them
  const int64_t ygrid = stream_rows ? std::min<int64_t>(ychunks, (target + rchunks - 1) / rchunks)
                                    : ychunks;
  int64_t ks = std::max<int64_t>(1, std::min<int64_t>(p.O, (target + ychunks * rchunks - 1) / (ychunks * rchunks)));
  // the row-stream epilogue reads P for four consecutive o at a time from
  // o = multiples of 4: its ranges are multiples of 16; the other kernels
  // split O evenly (rounding there left 20 workgroups for a 152^3 tensor)
  p.o_per_block = (p.O + ks - 1) / ks;
  if (stream_rows) p.o_per_block = (p.o_per_block + 15) / 16 * 16;
  ks = (p.O + p.o_per_block - 1) / p.o_per_block;
  p.Opad = (p.O + 3) / 4 * 4;
  const int64_t n_out = p.I_n * R;
  CP_TRY(ensure(h, h->part, sizeof(S) * (size_t)(ks * n_out), st));
  S* part = static_cast<S*>(h->part.ptr);
  dim3 grid((unsigned)ks, (unsigned)ygrid, (unsigned)rchunks);
  // the row kernels stage each wave's k-step rows (16 per tile, 36-float stride)
  const int wave_rows = stream_rows ? 16 * CPNG_ROWSTREAM_TW : (rows ? tile / 4 : 0);
  const size_t lds = (size_t)F::kFacBytes * 32 * (size_t)p.kpad +
                     sizeof(float) * 4 * 36 * (size_t)wave_rows;
  // outer tables: P (O x R values of S) then base offsets (O int64)
  const size_t pbytes = (sizeof(S) * (size_t)(p.Opad * R) + 255) & ~size_t(255);
  CP_TRY(ensure(h, h->otab, pbytes + sizeof(int64_t) * (size_t)p.O, st));
  S* Pg = static_cast<S*>(h->otab.ptr);
  int64_t* bg = reinterpret_cast<int64_t*>(static_cast<char*>(h->otab.ptr) + pbytes);
  {
    const int64_t Lc = kF32Src ? L : 0;
    const int64_t nt = std::max<int64_t>(p.Opad * (R + 1), Lc);
    hipLaunchKernelGGL(outer_tables_kernel<S>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st,
                       u, p, Pg, bg, fac32, Lc);
    CP_LAUNCH_CHECK(h);
  }
  {
    KernelTimer timer(h, dense_kernel_id<S>(), st);
    if (stream_rows) {
      if (ntr) CP_TIMED_LAUNCH(timer, (mttkrp_rowstream_mfma<F, true>), grid, dim3(kThr), lds, st, T, fac, Pg, bg, p, part);
      else CP_TIMED_LAUNCH(timer, (mttkrp_rowstream_mfma<F, false>), grid, dim3(kThr), lds, st, T, fac, Pg, bg, p, part);
    } else if (rows) {
      if (tile == 128) {
        if (ntr) CP_TIMED_LAUNCH(timer, (mttkrp_rows_mfma<F, 2, true>), grid, dim3(kThr), lds, st, T, fac, Pg, bg, p, part);
        else CP_TIMED_LAUNCH(timer, (mttkrp_rows_mfma<F, 2, false>), grid, dim3(kThr), lds, st, T, fac, Pg, bg, p, part);
      } else {
        if (ntr) CP_TIMED_LAUNCH(timer, (mttkrp_rows_mfma<F, 1, true>), grid, dim3(kThr), lds, st, T, fac, Pg, bg, p, part);
        else CP_TIMED_LAUNCH(timer, (mttkrp_rows_mfma<F, 1, false>), grid, dim3(kThr), lds, st, T, fac, Pg, bg, p, part);
      }
    } else {
      if (tile == 128) CP_TIMED_LAUNCH(timer, (mttkrp_cols_mfma<F, 2>), grid, dim3(kThr), lds, st, T, fac, Pg, bg, p, part);
      else CP_TIMED_LAUNCH(timer, (mttkrp_cols_mfma<F, 1>), grid, dim3(kThr), lds, st, T, fac, Pg, bg, p, part);
    }
  }
  CP_LAUNCH_CHECK(h);
  CP_TRY(launch_splitk_reduce(h, part, ks, n_out, R, M, st));
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

// Launches the two-sided pass in flavour F: both group partials X_L and X_R
// (float64, P x R and Q x R) of the split before mode `split`, from one read
// of T.  Returns CP_OK after launching, or 1 where the shape is not covered
// (R > 32; modes s-1 and N-1 not of length 64 or 128; the left group's outer
// count not a multiple of GA; a misaligned tensor; too little LDS).
template <class F, int GA>
int launch_twosided(cp_handle* h, const float* T, const double* u, const Shape& s, int split,
                    int R, double* XL, double* XR, hipStream_t st) {
  using S = typename F::S;
  constexpr bool kF32Src = sizeof(typename F::Src) == 4;
  const int N = s.N;
  if (split < 1 || split >= N || R < 1 || R > 32) return 1;
  const int64_t J = s.dims[split - 1], K = s.dims[N - 1];
  if ((J != 64 && J != 128) || (K != 64 && K != 128)) return 1;
  if (reinterpret_cast<uintptr_t>(T) % 16 != 0) return 1;
  TwoParams p{};
  p.R = R;
  p.J = J;
  p.K = K;
  p.OA = 1;
  p.na = split - 1;
  for (int m = 0; m < split - 1; ++m) {
    p.adims[m] = s.dims[m];
    p.afoff[m] = s.off[m] * R;
    p.OA *= s.dims[m];
  }
  p.OB = 1;
  p.nb = N - 1 - split;
  for (int m = split; m < N - 1; ++m) {
    p.bdims[m - split] = s.dims[m];
    p.bfoff[m - split] = s.off[m] * R;
    p.OB *= s.dims[m];
  }
  if (p.OA % GA != 0) return 1;
  p.Q = p.OB * K;
  if (p.Q >= (int64_t(1) << 26)) return 1;   // in-chunk offsets stay 32-bit
  p.jfoff = s.off[split - 1] * R;
  p.kfoff = s.off[N - 1] * R;
  p.kpadK = (int)K + F::kPad;
  p.kpadJ = (int)J + F::kPad;
  // (the scales' part, (GA + GB) x 32 values, is added once GB is known)
  size_t lds = (size_t)F::kFacBytes * 32 * (size_t)(p.kpadK + p.kpadJ) +
               2 * (K == 128 ? TwoStage<F, 128>::kBufBytes : TwoStage<F, 64>::kBufBytes);
  if (h->max_lds == 0) {
    int v = 0;
    CP_HIP(h, hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
    h->max_lds = v > 0 ? v : 65536;
  }
  if (lds > (size_t)h->max_lds) return 1;
  // workgroups: GA oa by GB ob each; about as many as fit the chip at once
  const int64_t gx = p.OA / GA;
  const int64_t target = 256 * twosided_waves<F, GA>();
  int64_t gy = std::max<int64_t>(1, std::min<int64_t>(p.OB, (target + gx - 1) / gx));
  p.GB = (p.OB + gy - 1) / gy;
  gy = (p.OB + p.GB - 1) / p.GB;
  lds += sizeof(S) * 32 * (size_t)(GA + p.GB);
  if (lds > (size_t)h->max_lds) return 1;
  // partial slots, slot-major, in fragment order: 32 rank columns per row
  const int64_t nL = gy * p.OA * J * 32, nR = gx * p.Q * 32;
  const size_t pl = (sizeof(S) * (size_t)nL + 255) & ~size_t(255);
  CP_TRY(ensure(h, h->part, pl + sizeof(S) * (size_t)nR, st));
  S* partL = static_cast<S*>(h->part.ptr);
  S* partR = reinterpret_cast<S*>(static_cast<char*>(h->part.ptr) + pl);
  const size_t ta = (sizeof(S) * (size_t)(p.OA * R) + 255) & ~size_t(255);
  CP_TRY(ensure(h, h->otab, ta + sizeof(S) * (size_t)(p.OB * R), st));
  S* PA = static_cast<S*>(h->otab.ptr);
  S* PB = reinterpret_cast<S*>(static_cast<char*>(h->otab.ptr) + ta);
  const int64_t L = s.sum_dims() * R;
  float* fac32 = nullptr;
  if (kF32Src) {
    CP_TRY(ensure(h, h->stage, sizeof(float) * (size_t)L, st));
    fac32 = static_cast<float*>(h->stage.ptr);
  }
  const typename F::Src* fac = nullptr;
  if constexpr (kF32Src) fac = fac32;
  else fac = u;
  {
    const int64_t Lc = kF32Src ? L : 0;
    const int64_t nt = std::max<int64_t>((p.OA + p.OB) * R, Lc);
    hipLaunchKernelGGL(twosided_tables_kernel<S>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0,
                       st, u, p, PA, PB, fac32, Lc);
    CP_LAUNCH_CHECK(h);
  }
  const int kid = sizeof(S) == 8 ? CP_KERNEL_DENSE_TWOSIDED_F64 : CP_KERNEL_DENSE_TWOSIDED;
  const dim3 grid((unsigned)gx, (unsigned)gy);
  // returns 1 (not covered) if the runtime refuses the kernel this much LDS
  auto go = [&](auto kern) -> int {
    if (lds > 65536 &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
      (void)hipGetLastError();
      return 1;
    }
    KernelTimer timer(h, kid, st);
    CP_TIMED_LAUNCH(timer, kern, grid, dim3(kThr), lds, st, T, fac, PA, PB, p, partL, partR);
    return CP_OK;
  };
  int rc;
  if (K == 128 && J == 128) rc = go(mttkrp_twosided_mfma<F, 4, 4, GA>);
  else if (K == 128) rc = go(mttkrp_twosided_mfma<F, 4, 2, GA>);
  else if (J == 128) rc = go(mttkrp_twosided_mfma<F, 2, 4, GA>);
  else rc = go(mttkrp_twosided_mfma<F, 2, 2, GA>);
  if (rc != CP_OK) return rc;
  CP_LAUNCH_CHECK(h);
  h->t_passes++;
  CP_TRY(launch_splitk_frag(h, partL, gy, p.OA * J, R, sizeof(S) == 8, XL, st));
  CP_LAUNCH_CHECK(h);
  CP_TRY(launch_splitk_frag(h, partR, gx, p.Q, R, sizeof(S) == 8, XR, st));
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

}  // namespace

// The streaming matrix-core MTTKRP of one mode, per arithmetic: BF16x3
// split products, float32 products (both with float32 sums inside a
// workgroup), or float64 products and sums of the widened float32 tensor.
// Each returns CP_OK after launching, or 1 if the shape is not one the
// streaming kernels cover (inner length not a multiple of 8, or above 512;
// above 256 for float64; a misaligned tensor).
int dense_fast_bf16x3(cp_handle* h, const float* T, const double* u, const Shape& s, int R,
                      int mode, double* M, hipStream_t st) {
  return launch_mfma<FlavBF16x3>(h, T, u, s, R, mode, M, st);
}

int dense_fast_mfma_f32(cp_handle* h, const float* T, const double* u, const Shape& s, int R,
                        int mode, double* M, hipStream_t st) {
  return launch_mfma<FlavF32>(h, T, u, s, R, mode, M, st);
}

int dense_fast_mfma_f64acc(cp_handle* h, const float* T, const double* u, const Shape& s, int R,
                           int mode, double* M, hipStream_t st) {
  return launch_mfma<FlavF64>(h, T, u, s, R, mode, M, st);
}

// Both group partials of the two-level evaluation (split before mode
// `split`) from one pass over T, per arithmetic (as the single-mode calls
// above).  CP_OK after launching, 1 where the shape is not covered.
int dense_twosided(cp_handle* h, const float* T, const double* u, const Shape& s, int split, int R,
                   int prec, double* XL, double* XR, hipStream_t st) {
  // (launch_twosided returns 1 before launching anything where GA does not
  // divide the left outer count; those shapes run with GA = 2)
  constexpr int ga = CPNG_TWOSIDED_GA, ga64 = CPNG_TWOSIDED_GA64;
  int rc = 1;
  if (prec == CP_PREC_BF16X3) {
    rc = launch_twosided<FlavBF16x3, ga>(h, T, u, s, split, R, XL, XR, st);
    if (rc == 1 && ga != 2) rc = launch_twosided<FlavBF16x3, 2>(h, T, u, s, split, R, XL, XR, st);
  } else if (prec == CP_PREC_FP32) {
    rc = launch_twosided<FlavF32, ga>(h, T, u, s, split, R, XL, XR, st);
    if (rc == 1 && ga != 2) rc = launch_twosided<FlavF32, 2>(h, T, u, s, split, R, XL, XR, st);
  } else {
    rc = launch_twosided<FlavF64, ga64>(h, T, u, s, split, R, XL, XR, st);
    if (rc == 1 && ga64 != 2) rc = launch_twosided<FlavF64, 2>(h, T, u, s, split, R, XL, XR, st);
  }
  return rc;
}

}  // namespace cpng

namespace cpng {

// Fills the inner/outer description of mode `mode`; the inner mode is N-1
// for the row layout and N-2 for the column layout.
static void fill_params(const Shape& s, int R, int mode, FastParams* pp) {
  FastParams& p = *pp;
  const int N = s.N;
  const bool rows = mode < N - 1;
  const int q = rows ? N - 1 : N - 2;
  p = FastParams{};
  p.R = R;
  int64_t stride[CP_MAX_ORDER];
  stride[N - 1] = 1;
  for (int k = N - 2; k >= 0; --k) stride[k] = stride[k + 1] * s.dims[k + 1];
  p.nout = 0;
  p.O = 1;
  for (int k = 0; k < N; ++k) {
    if (k == mode || k == q) continue;
    p.ostride[p.nout] = stride[k];
    p.odims[p.nout] = s.dims[k];
    p.ofoff[p.nout] = s.off[k] * R;
    p.O *= s.dims[k];
    p.nout++;
  }
  p.qfoff = s.off[q] * R;
  p.I_n = s.dims[mode];
  p.K = s.dims[q];
  p.istride = stride[mode];
  p.kstride = stride[q];
  p.nks = (int)((p.K + 31) / 32);
  p.kpad = p.nks * 32 + 8;
}

template <typename TT, typename CT, int RB>
static int launch_tiles(cp_handle* h, const TT* T, const CT* fac, FastParams p, bool rows,
                        double* M, hipStream_t st) {
  const int64_t ychunks = (p.I_n + 63) / 64;
  const int64_t rchunks = (p.R + RB - 1) / RB;
  const int64_t target = 1024;
  int64_t ks = std::max<int64_t>(1, std::min<int64_t>(p.O, (target + ychunks * rchunks - 1) / (ychunks * rchunks)));
  p.o_per_block = (p.O + ks - 1) / ks;
  ks = (p.O + p.o_per_block - 1) / p.o_per_block;
  const int64_t n_out = p.I_n * p.R;
  CP_TRY(ensure(h, h->part, sizeof(CT) * (size_t)(ks * n_out), st));
  CT* part = static_cast<CT*>(h->part.ptr);
  dim3 grid((unsigned)ks, (unsigned)ychunks, (unsigned)rchunks);
  {
    KernelTimer timer(h, dense_kernel_id<CT>(), st);
    if (rows) CP_TIMED_LAUNCH(timer, (mttkrp_tiles_vec<TT, CT, RB, true>), grid, dim3(kThr), 0, st, T, fac, p, part);
    else CP_TIMED_LAUNCH(timer, (mttkrp_tiles_vec<TT, CT, RB, false>), grid, dim3(kThr), 0, st, T, fac, p, part);
  }
  CP_LAUNCH_CHECK(h);
  CP_TRY(launch_splitk_reduce(h, part, ks, n_out, p.R, M, st));
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

// Vector-ALU streaming MTTKRP for FP32 (TT = CT = float) and FP64
// accumulation (CT = double, TT = float or double).  Returns 1 if the layout
// is not covered (order < 2 or a misaligned base pointer).
template <typename TT, typename CT>
int dense_fast_vec(cp_handle* h, const TT* T, const CT* fac, const Shape& s, int R, int mode,
                   double* M, hipStream_t st) {
  if (s.N < 2) return 1;
  if (reinterpret_cast<uintptr_t>(T) % 16 != 0) return 1;
  FastParams p;
  fill_params(s, R, mode, &p);
  const bool rows = mode < s.N - 1;
  // 16-byte loads stay aligned when the unit-stride extent is a multiple of
  // 16 bytes (every row or k-row then starts on a 16-byte boundary);
  // otherwise the tile is loaded element by element.
  p.vec_ok = rows ? (p.K * sizeof(TT)) % 16 == 0 : (p.I_n * sizeof(TT)) % 16 == 0;
  if (R <= 8) return launch_tiles<TT, CT, 8>(h, T, fac, p, rows, M, st);
  if (R <= 16) return launch_tiles<TT, CT, 16>(h, T, fac, p, rows, M, st);
  return launch_tiles<TT, CT, 32>(h, T, fac, p, rows, M, st);
}

template int dense_fast_vec<float, float>(cp_handle*, const float*, const float*, const Shape&, int,
                                          int, double*, hipStream_t);
template int dense_fast_vec<float, double>(cp_handle*, const float*, const double*, const Shape&, int,
                                           int, double*, hipStream_t);
template int dense_fast_vec<double, double>(cp_handle*, const double*, const double*, const Shape&,
                                            int, int, double*, hipStream_t);

}  // namespace cpng
