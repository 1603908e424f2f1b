// Attribute gather through the frozen new -> old vertex map, and its
// backward (scatter-add), for per-vertex float attributes that follow the
// re-indexed vertices (Section 3 mentions vertices carrying attributes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/meshrx.h"

namespace {

constexpr int32_t kErrIndex = 3;

int64_t grid_for(int64_t work, int block, int64_t cap = 16384) {
  return std::max<int64_t>(1, std::min<int64_t>((work + block - 1) / block, cap));
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}

// A row of C scalars of type T is moved as C / VEC vectors of VEC scalars.
template <typename T, int VEC>
struct alignas(sizeof(T) * VEC) Vec {
  T v[VEC];
};

// out[j, :] = attrs[new2old[j], :]
template <typename T, int VEC>
__global__ void k_gather_rows(const Vec<T, VEC>* __restrict__ attrs, int64_t num_old, int32_t vpr,
                              const int32_t* __restrict__ new2old, int64_t num_new,
                              Vec<T, VEC>* __restrict__ out, int32_t* status) {
  const int64_t total = num_new * vpr;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t j = t / vpr;
    const int32_t q = int32_t(t - j * vpr);
    const int32_t r = new2old[j];
    if (r >= 0 && r < num_old) {
      out[t] = attrs[int64_t(r) * vpr + q];
    } else {
      Vec<T, VEC> z;
#pragma unroll
      for (int i = 0; i < VEC; ++i) z.v[i] = T(0);
      out[t] = z;
      if (status) atomicMax(status, kErrIndex);
    }
  }
}

__global__ void k_zero_words(uint32_t* __restrict__ p, int64_t nwords) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t n4 = nwords / 4;
  uint4* p4 = reinterpret_cast<uint4*>(p);  // p is 16-byte aligned (checked on the host)
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n4; i += stride)
    p4[i] = make_uint4(0, 0, 0, 0);
  for (int64_t i = n4 * 4 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nwords; i += stride)
    p[i] = 0;
}

// grad[new2old[j], :] = 0 + g[j, :] when new2old is injective (every row
// receives at most one contribution; 0 + g also turns -0 into +0, as
// accumulating into zeros does).
template <typename T, int VEC>
__global__ void k_scatter_rows_store(const Vec<T, VEC>* __restrict__ g, int64_t num_new, int32_t vpr,
                                     const int32_t* __restrict__ new2old, int64_t num_old,
                                     Vec<T, VEC>* __restrict__ grad, int32_t* status) {
  const int64_t total = num_new * vpr;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t j = t / vpr;
    const int32_t q = int32_t(t - j * vpr);
    const int32_t r = new2old[j];
    if (r >= 0 && r < num_old) {
      Vec<T, VEC> x = g[t];
#pragma unroll
      for (int i = 0; i < VEC; ++i) x.v[i] = T(0) + x.v[i];
      grad[int64_t(r) * vpr + q] = x;
    } else if (status) {
      atomicMax(status, kErrIndex);
    }
  }
}

// grad[new2old[j], c] += g[j, c] with atomics (any map).
template <typename T>
__global__ void k_scatter_add(const T* __restrict__ g, int64_t num_new, int32_t channels,
                              const int32_t* __restrict__ new2old, int64_t num_old, T* grad,
                              int32_t* status) {
  const int64_t total = num_new * channels;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t j = t / channels;
    const int32_t c = int32_t(t - j * channels);
    const int32_t r = new2old[j];
    if (r >= 0 && r < num_old) {
      atomicAdd(grad + int64_t(r) * channels + c, g[t]);
    } else if (status) {
      atomicMax(status, kErrIndex);
    }
  }
}

template <typename T, int VEC>
void launch_gather(const void* attrs, int64_t num_old, int32_t channels, const int32_t* new2old,
                   int64_t num_new, void* out, int32_t* status, hipStream_t s) {
  const int32_t vpr = channels / VEC;
  hipLaunchKernelGGL((k_gather_rows<T, VEC>), dim3(grid_for(num_new * vpr, 256)), dim3(256), 0, s,
                     static_cast<const Vec<T, VEC>*>(attrs), num_old, vpr, new2old, num_new,
                     static_cast<Vec<T, VEC>*>(out), status);
}

template <typename T, int VEC>
void launch_scatter_store(const void* g, int64_t num_new, int32_t channels, const int32_t* new2old,
                          int64_t num_old, void* grad, int32_t* status, hipStream_t s) {
  const int32_t vpr = channels / VEC;
  hipLaunchKernelGGL((k_scatter_rows_store<T, VEC>), dim3(grid_for(num_new * vpr, 256)), dim3(256), 0, s,
                     static_cast<const Vec<T, VEC>*>(g), num_new, vpr, new2old, num_old,
                     static_cast<Vec<T, VEC>*>(grad), status);
}

template <typename T>
mrx_status gather_typed(const void* attrs, int64_t num_old, int32_t channels, const int32_t* new2old,
                        int64_t num_new, void* out, int32_t* status, hipStream_t s) {
  constexpr int V = 16 / sizeof(T);
  if (channels % V == 0 && aligned(attrs, 16) && aligned(out, 16))
    launch_gather<T, V>(attrs, num_old, channels, new2old, num_new, out, status, s);
  else
    launch_gather<T, 1>(attrs, num_old, channels, new2old, num_new, out, status, s);
  return hipGetLastError() == hipSuccess ? MRX_OK : MRX_ERR_HIP;
}

template <typename T>
mrx_status backward_typed(const void* g, int64_t num_new, int32_t channels, const int32_t* new2old,
                          int64_t num_old, void* grad, bool injective, int32_t* status, hipStream_t s) {
  const int64_t words = num_old * channels * int64_t(sizeof(T) / 4);
  if (words > 0)
    hipLaunchKernelGGL(k_zero_words, dim3(grid_for(words / 4 + 1, 256)), dim3(256), 0, s,
                       static_cast<uint32_t*>(grad), words);
  if (num_new > 0) {
    constexpr int V = 16 / sizeof(T);
    if (!injective) {
      hipLaunchKernelGGL((k_scatter_add<T>), dim3(grid_for(num_new * channels, 256)), dim3(256), 0, s,
                         static_cast<const T*>(g), num_new, channels, new2old, num_old,
                         static_cast<T*>(grad), status);
    } else if (channels % V == 0 && aligned(g, 16)) {
      launch_scatter_store<T, V>(g, num_new, channels, new2old, num_old, grad, status, s);
    } else {
      launch_scatter_store<T, 1>(g, num_new, channels, new2old, num_old, grad, status, s);
    }
  }
  return hipGetLastError() == hipSuccess ? MRX_OK : MRX_ERR_HIP;
}

}  // namespace

extern "C" {

mrx_status mrx_gather_attrs(const void* attrs, int64_t num_old, int32_t channels, int32_t dtype,
                            const int32_t* new2old, int64_t num_new, void* out, int32_t* dev_status,
                            void* stream) {
  if (channels < 1 || (dtype != 0 && dtype != 1) || num_old < 0 || num_new < 0)
    return MRX_ERR_INVALID_ARGUMENT;
  if (num_old > INT32_MAX || num_new > INT32_MAX) return MRX_ERR_TOO_LARGE;
  const size_t es = dtype == 0 ? 4 : 8;
  if (num_new > 0 && (!out || !new2old || (num_old > 0 && !attrs))) return MRX_ERR_INVALID_ARGUMENT;
  if (!aligned(attrs, 16) || !aligned(out, es) || !aligned(new2old, 4) || !aligned(dev_status, 4))
    return MRX_ERR_INVALID_ARGUMENT;
  if (overlaps(out, size_t(num_new) * channels * es, attrs, size_t(num_old) * channels * es) ||
      overlaps(out, size_t(num_new) * channels * es, new2old, size_t(num_new) * 4))
    return MRX_ERR_INVALID_ARGUMENT;
  if (num_new == 0) return MRX_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return dtype == 0 ? gather_typed<float>(attrs, num_old, channels, new2old, num_new, out, dev_status, s)
                    : gather_typed<double>(attrs, num_old, channels, new2old, num_new, out, dev_status, s);
}

mrx_status mrx_gather_attrs_backward(const void* grad_out, int64_t num_new, int32_t channels, int32_t dtype,
                                     const int32_t* new2old, int64_t num_old, void* grad_attrs,
                                     int32_t assume_injective, int32_t* dev_status, void* stream) {
  if (channels < 1 || (dtype != 0 && dtype != 1) || num_old < 0 || num_new < 0)
    return MRX_ERR_INVALID_ARGUMENT;
  if (num_old > INT32_MAX || num_new > INT32_MAX) return MRX_ERR_TOO_LARGE;
  const size_t es = dtype == 0 ? 4 : 8;
  if (num_old > 0 && !grad_attrs) return MRX_ERR_INVALID_ARGUMENT;
  if (num_new > 0 && (!grad_out || !new2old)) return MRX_ERR_INVALID_ARGUMENT;
  if (!aligned(grad_attrs, 16) || !aligned(grad_out, es) || !aligned(new2old, 4) ||
      !aligned(dev_status, 4))
    return MRX_ERR_INVALID_ARGUMENT;
  if (overlaps(grad_attrs, size_t(num_old) * channels * es, grad_out, size_t(num_new) * channels * es) ||
      overlaps(grad_attrs, size_t(num_old) * channels * es, new2old, size_t(num_new) * 4))
    return MRX_ERR_INVALID_ARGUMENT;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool inj = assume_injective != 0;
  return dtype == 0
             ? backward_typed<float>(grad_out, num_new, channels, new2old, num_old, grad_attrs, inj, dev_status, s)
             : backward_typed<double>(grad_out, num_new, channels, new2old, num_old, grad_attrs, inj, dev_status, s);
}

}  // extern "C"
