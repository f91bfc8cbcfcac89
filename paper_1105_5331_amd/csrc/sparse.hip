// Sparse (coordinate format) MTTKRP on gfx950 (Section 2.3, the product
// T_(n) Phibar^(n) restricted to the nonzeros):
//     M(i, r) = sum_{z : i_n(z) = i} v_z prod_{k != n} A^(k)(i_k(z), r).
//
// Preparation builds, for every mode n, a copy of the nonzeros stably sorted
// by i_n (other modes' coordinates and the values, structure of arrays) and
// the segment pointers seg[i] = first nonzero of row i.  The MTTKRP then
// gives each group of W lanes (lane = rank r) a contiguous, equal-sized range
// of sorted nonzeros.  A group sums each row it meets in registers: rows that
// lie strictly inside its range are complete and written directly; the first
// and the last row it meets may continue in a neighbouring group and are
// written as two carry slots.  A fix-up kernel adds the carries of each row
// in slot order.  No atomics: the result is bitwise reproducible.
#include "common.hpp"

#include <hipcub/hipcub.hpp>

#include <algorithm>

namespace cpng {

namespace {

constexpr int kChunk = 512;   // nonzeros per lane group

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
  int N, mode, R;
  int64_t nnz, I_n, ngroups;
  const int32_t* coords;          // (N-1) x nnz, other modes in increasing order
  const int64_t* seg;             // I_n + 1
  int64_t foff[CP_MAX_ORDER - 1]; // factor element offsets of the other modes
};

// W lanes per group (W >= R, power of two), 256 / W groups per workgroup.
template <typename TT, typename CT, int W>
__global__ __launch_bounds__(256) void sparse_mttkrp_kernel(const TT* __restrict__ vals,
                                                            const CT* __restrict__ fac,
                                                            SparseParams p,
                                                            double* __restrict__ M,
                                                            int64_t* __restrict__ carry_row,
                                                            double* __restrict__ carry_val) {
  const int lane = threadIdx.x % W;
  const int64_t gidx = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / W;
  if (gidx >= p.ngroups) return;
  const int64_t z0 = gidx * kChunk;
  const int64_t z1 = min<int64_t>(p.nnz, z0 + kChunk);
  const bool active = lane < p.R;
  // row of z0: largest i with seg[i] <= z0
  int64_t lo = 0, hi = p.I_n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (p.seg[mid] <= z0) lo = mid;
    else hi = mid - 1;
  }
  int64_t row = lo;
  int64_t next = p.seg[row + 1];
  const int lr = active ? lane : 0;   // inactive lanes read a valid address
  CT acc = CT(0);
  bool first = true;
  for (int64_t z = z0; z < z1; ++z) {
    if (z >= next) {
      // row finished inside this group
      if (first) {
        if (active) carry_val[(2 * gidx) * p.R + lane] = (double)acc;
        if (lane == 0) carry_row[2 * gidx] = row;
        first = false;
      } else if (active) {
        M[row * p.R + lane] = (double)acc;
      }
      acc = CT(0);
      do {
        ++row;
        next = p.seg[row + 1];
      } while (z >= next);
    }
    CT prod = (CT)vals[z];
    for (int k = 0; k < p.N - 1; ++k) {
      const int32_t c = p.coords[(int64_t)k * p.nnz + z];
      prod *= fac[p.foff[k] + (int64_t)c * p.R + lr];
    }
    acc += prod;
  }
  if (first) {
    if (active) {
      carry_val[(2 * gidx) * p.R + lane] = (double)acc;
      carry_val[(2 * gidx + 1) * p.R + lane] = 0.0;
    }
    if (lane == 0) {
      carry_row[2 * gidx] = row;
      carry_row[2 * gidx + 1] = row;
    }
  } else {
    if (active) carry_val[(2 * gidx + 1) * p.R + lane] = (double)acc;
    if (lane == 0) carry_row[2 * gidx + 1] = row;
  }
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

template <typename TT, typename CT, int W>
int launch_sparse(cp_handle* h, const TT* vals, const CT* fac, SparseParams p, double* M,
                  hipStream_t st) {
  const int64_t nslots = 2 * p.ngroups;
  CP_TRY(ensure(h, h->carry, (sizeof(int64_t) + sizeof(double) * p.R) * (size_t)std::max<int64_t>(1, nslots), st));
  int64_t* crow = static_cast<int64_t*>(h->carry.ptr);
  double* cval = reinterpret_cast<double*>(crow + nslots);
  const int64_t threads = p.ngroups * W;
  {
    KernelTimer timer(h, CP_KERNEL_SPARSE_MTTKRP, st);
    hipLaunchKernelGGL((sparse_mttkrp_kernel<TT, CT, W>), dim3(nblk(threads, 256)), dim3(256), 0,
                       st, vals, fac, p, M, crow, cval);
  }
  CP_LAUNCH_CHECK(h);
  hipLaunchKernelGGL(carry_fixup_kernel, dim3(nblk(nslots * p.R, 256)), dim3(256), 0, st, crow,
                     cval, nslots, p.R, M);
  CP_LAUNCH_CHECK(h);
  return CP_OK;
}

template <typename TT, typename CT>
int dispatch_w(cp_handle* h, const TT* vals, const CT* fac, const SparseParams& p, double* M,
               hipStream_t st) {
  if (p.R <= 4) return launch_sparse<TT, CT, 4>(h, vals, fac, p, M, st);
  if (p.R <= 8) return launch_sparse<TT, CT, 8>(h, vals, fac, p, M, st);
  if (p.R <= 16) return launch_sparse<TT, CT, 16>(h, vals, fac, p, M, st);
  if (p.R <= 32) return launch_sparse<TT, CT, 32>(h, vals, fac, p, M, st);
  if (p.R <= 64) return launch_sparse<TT, CT, 64>(h, vals, fac, p, M, st);
  return fail(h, CP_EINVAL, "sparse MTTKRP supports R <= 64 (got %d)", p.R);
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
  hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, coords, keys_out, perm_in, perm_out,
                                     (int)nnz, 0, 32, st);
  if (hipMalloc(&temp, temp_bytes + 16) != hipSuccess) {
    cleanup();
    return fail(h, CP_ENOMEM, "sparse prepare: sort workspace allocation failed");
  }
  for (int n = 0; n < N && rc == CP_OK; ++n) {
    SparseMode& md = sp->mode[n];
    if (hipMalloc(&md.coords, sizeof(int32_t) * std::max<int64_t>(1, (N - 1) * nnz)) != hipSuccess ||
        hipMalloc(&md.values, sizeof(V) * nnz) != hipSuccess ||
        hipMalloc(&md.seg, sizeof(int64_t) * (s.dims[n] + 1)) != hipSuccess) {
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
  int rc = CP_OK;
  if (nnz > 0) {
    int* dflag = nullptr;
    CP_HIP(h, hipMalloc(&dflag, 2 * sizeof(int)));
    CP_HIP(h, hipMemsetAsync(dflag, 0, 2 * sizeof(int), st));
    hipLaunchKernelGGL(bounds_kernel, dim3(nblk(nnz, 256)), dim3(256), 0, st, T->coords, nnz, s.N,
                       s, dflag);
    // duplicate check on the full linear index when it fits in 64 bits
    double lim = 1.0;
    for (int k = 0; k < s.N; ++k) lim *= (double)s.dims[k];
    uint64_t *key = nullptr, *key2 = nullptr;
    void* temp = nullptr;
    if (lim < 1.8e19) {
      size_t tb = 0;
      if (hipMalloc(&key, sizeof(uint64_t) * nnz) == hipSuccess &&
          hipMalloc(&key2, sizeof(uint64_t) * nnz) == hipSuccess) {
        hipcub::DeviceRadixSort::SortKeys(nullptr, tb, key, key2, (int)nnz, 0, 64, st);
        if (hipMalloc(&temp, tb + 16) == hipSuccess) {
          hipStreamSynchronize(st);
          int bad = 0;
          hipMemcpy(&bad, dflag, sizeof(int), hipMemcpyDeviceToHost);
          if (!bad) {   // keys are only meaningful with in-range coordinates
            hipLaunchKernelGGL(linear_key_kernel, dim3(nblk(nnz, 256)), dim3(256), 0, st, T->coords,
                               nnz, s, key);
            hipcub::DeviceRadixSort::SortKeys(temp, tb, key, key2, (int)nnz, 0, 64, st);
            hipLaunchKernelGGL(adjacent_equal_kernel, dim3(nblk(nnz, 256)), dim3(256), 0, st, key2,
                               nnz, dflag + 1);
          }
        } else {
          rc = fail(h, CP_ENOMEM, "sparse prepare: duplicate-check workspace allocation failed");
        }
      } else {
        rc = fail(h, CP_ENOMEM, "sparse prepare: duplicate-check allocation failed");
      }
    }
    hipStreamSynchronize(st);
    int flags[2] = {0, 0};
    hipMemcpy(flags, dflag, 2 * sizeof(int), hipMemcpyDeviceToHost);
    if (key) hipFree(key);
    if (key2) hipFree(key2);
    if (temp) hipFree(temp);
    hipFree(dflag);
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
      hipMemsetAsync(md.seg, 0, sizeof(int64_t) * (s.dims[n] + 1), st);
    }
    hipStreamSynchronize(st);
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
  (void)hipDeviceSynchronize();
  for (int n = 0; n < sp->N; ++n) {
    if (sp->mode[n].coords) (void)hipFree(sp->mode[n].coords);
    if (sp->mode[n].values) (void)hipFree(sp->mode[n].values);
    if (sp->mode[n].seg) (void)hipFree(sp->mode[n].seg);
  }
  delete sp;
  T->prepared = nullptr;
  (void)h;
  return CP_OK;
}

int sparse_mttkrp(cp_handle* h, const cp_tensor* T, const Shape& s, const double* u, int R,
                  int mode, int prec, double* M, hipStream_t st) {
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
  p.I_n = I;
  p.ngroups = (sp->nnz + kChunk - 1) / kChunk;
  p.coords = sp->mode[mode].coords;
  p.seg = sp->mode[mode].seg;
  int kk = 0;
  for (int k = 0; k < s.N; ++k)
    if (k != mode) p.foff[kk++] = s.off[k] * R;
  const void* vals = sp->mode[mode].values;
  if (prec == CP_PREC_FP32) {
    if (sp->dtype != CP_F32) return fail(h, CP_EINVAL, "precision FP32 needs float32 values");
    float* fac = nullptr;
    CP_TRY(stage_factors_f32(h, u, s.sum_dims() * R, &fac, st));
    return dispatch_w<float, float>(h, static_cast<const float*>(vals), fac, p, M, st);
  }
  if (sp->dtype == CP_F32)
    return dispatch_w<float, double>(h, static_cast<const float*>(vals), u, p, M, st);
  return dispatch_w<double, double>(h, static_cast<const double*>(vals), u, p, M, st);
}

}  // namespace cpng
