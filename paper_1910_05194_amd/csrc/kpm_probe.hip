// HBM bandwidth probes: the ceiling that streaming kernels reach on this
// device for the access patterns of the hot path, and the reference kernel
// of known traffic used to calibrate hardware byte counters.
//
// Patterns (float4 elements, grid-stride loops):
//   0 copy   dst = src                      (1 read, 1 write per element)
//   1 read   acc += src                     (1 read)
//   2 rmw    w = 2 v - w  (in place)        (2 reads, 1 write: the Chebyshev step's pattern)
//   3 copy   dst = src, four elements per thread and iteration, all four
//            loads issued before the stores (more bytes in flight per wave)

#include "kpm_internal.h"

namespace kpm {

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ void probe_copy(const f32x4* __restrict__ src, f32x4* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if constexpr (NT) {
      f32x4 x = __builtin_nontemporal_load(src + i);
      __builtin_nontemporal_store(x, dst + i);
    } else {
      dst[i] = src[i];
    }
  }
}

template <bool NT>
__global__ void probe_read(const f32x4* __restrict__ src, float* __restrict__ out, int64_t n) {
  float acc = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    f32x4 x;
    if constexpr (NT) x = __builtin_nontemporal_load(src + i);
    else x = src[i];
    acc += x.x + x.y + x.z + x.w;
  }
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

template <bool NT>
__global__ void probe_copy4(const f32x4* __restrict__ src, f32x4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    f32x4 x[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = NT ? __builtin_nontemporal_load(src + i + k * stride) : src[i + k * stride];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if constexpr (NT) __builtin_nontemporal_store(x[k], dst + i + k * stride);
      else dst[i + k * stride] = x[k];
    }
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

template <bool NT>
__global__ void probe_rmw(const f32x4* __restrict__ v, f32x4* __restrict__ w, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    f32x4 a, b;
    if constexpr (NT) {
      a = __builtin_nontemporal_load(v + i);
      b = __builtin_nontemporal_load(w + i);
    } else {
      a = v[i];
      b = w[i];
    }
    f32x4 o = 2.f * a - b;
    if constexpr (NT) __builtin_nontemporal_store(o, w + i);
    else w[i] = o;
  }
}

}  // namespace kpm

extern "C" int kpm_bandwidth_probe(int32_t pattern, int64_t bytes_per_array, int32_t iters, int32_t grid,
                                   int32_t block, int32_t nontemporal, void* hip_stream, double* ms_per_iter,
                                   double* bytes_moved_per_iter) {
  using namespace kpm;
  clear_error();
  KPM_CHECK_ARG(pattern >= 0 && pattern <= 3, "pattern must be 0 (copy), 1 (read), 2 (rmw) or 3 (copy, 4 per thread)");
  KPM_CHECK_ARG(bytes_per_array >= 16 && iters >= 1, "need bytes_per_array >= 16 and iters >= 1");
  KPM_CHECK_ARG(grid >= 1 && block >= 64 && block <= 1024 && block % 64 == 0, "bad launch shape");
  KPM_CHECK_ARG(ms_per_iter && bytes_moved_per_iter, "NULL output");
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t n = bytes_per_array / 16;
  f32x4 *a = nullptr, *b = nullptr;
  float* red = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int st = KPM_OK;
  auto cleanup = [&]() {
    if (a) (void)::kpm::dev_free(a);
    if (b) (void)::kpm::dev_free(b);
    if (red) (void)::kpm::dev_free(red);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  hipError_t e = ::kpm::dev_malloc(&a, n * 16);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&b, n * 16);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&red, (size_t)grid * block * sizeof(float));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipMemsetAsync(a, 0, n * 16, s);
  if (e == hipSuccess) e = hipMemsetAsync(b, 0, n * 16, s);
  auto launch = [&]() {
    const bool nt = nontemporal != 0;
    if (pattern == 0) {
      if (nt) hipLaunchKernelGGL(probe_copy<true>, dim3(grid), dim3(block), 0, s, a, b, n);
      else hipLaunchKernelGGL(probe_copy<false>, dim3(grid), dim3(block), 0, s, a, b, n);
    } else if (pattern == 3) {
      if (nt) hipLaunchKernelGGL(probe_copy4<true>, dim3(grid), dim3(block), 0, s, a, b, n);
      else hipLaunchKernelGGL(probe_copy4<false>, dim3(grid), dim3(block), 0, s, a, b, n);
    } else if (pattern == 1) {
      if (nt) hipLaunchKernelGGL(probe_read<true>, dim3(grid), dim3(block), 0, s, a, red, n);
      else hipLaunchKernelGGL(probe_read<false>, dim3(grid), dim3(block), 0, s, a, red, n);
    } else {
      if (nt) hipLaunchKernelGGL(probe_rmw<true>, dim3(grid), dim3(block), 0, s, a, b, n);
      else hipLaunchKernelGGL(probe_rmw<false>, dim3(grid), dim3(block), 0, s, a, b, n);
    }
  };
  if (e == hipSuccess) {
    launch();  // warm-up
    e = hipEventRecord(e0, s);
  }
  for (int i = 0; e == hipSuccess && i < iters; ++i) launch();
  if (e == hipSuccess) e = ::kpm::launch_status();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e != hipSuccess) {
    set_error("kpm_bandwidth_probe: %s", hipGetErrorString(e));
    st = (e == hipErrorOutOfMemory) ? KPM_E_NOMEM : KPM_E_DEVICE;
  } else {
    *ms_per_iter = ms / iters;
    *bytes_moved_per_iter = (double)n * 16 * ((pattern == 0 || pattern == 3) ? 2 : (pattern == 1 ? 1 : 3));
  }
  cleanup();
  return st;
}
