// Measurement utilities of libsca: a plain streaming copy and a streaming read of a
// buffer of known size (16-byte accesses, grid-stride).  They give the achievable HBM
// bandwidth beside the round kernels and calibrate hardware byte counters.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sca_internal.h"

using namespace sca;

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_stream_copy(f4* __restrict__ dst, const f4* __restrict__ src,
                                                     long long n16) {
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n16; i += (long long)gridDim.x * 256)
    dst[i] = __builtin_nontemporal_load(src + i);
}

__global__ void __launch_bounds__(256) k_stream_read(const f4* __restrict__ src, long long n16,
                                                     float* __restrict__ sink) {
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n16; i += (long long)gridDim.x * 256)
    acc += __builtin_nontemporal_load(src + i);
  const float v = acc[0] + acc[1] + acc[2] + acc[3];
  if (v == 1.2345678e-30f) sink[blockIdx.x] = v;  // keeps the loads; practically never stores
}

}  // namespace

extern "C" sca_status sca_stream_copy(void* dst, const void* src, int64_t bytes, int32_t grid,
                                      void* stream) {
  if (!dst || !src || bytes < 0 || bytes % 16 || ((uintptr_t)dst) % 16 || ((uintptr_t)src) % 16)
    return set_error(SCA_EINVAL, "16-byte aligned buffers and a size multiple of 16 expected");
  if (grid <= 0) grid = 4 * device_cu_count();
  hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, (hipStream_t)stream, (f4*)dst,
                     (const f4*)src, (long long)(bytes / 16));
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SCA_OK : set_error(SCA_EHIP, "stream copy: %s", hipGetErrorString(e));
}

extern "C" sca_status sca_stream_read(const void* src, int64_t bytes, void* sink_dev, int32_t grid,
                                      void* stream) {
  if (!src || !sink_dev || bytes < 0 || bytes % 16 || ((uintptr_t)src) % 16)
    return set_error(SCA_EINVAL, "a 16-byte aligned buffer and a size multiple of 16 expected");
  if (grid <= 0) grid = 4 * device_cu_count();
  hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const f4*)src,
                     (long long)(bytes / 16), (float*)sink_dev);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SCA_OK : set_error(SCA_EHIP, "stream read: %s", hipGetErrorString(e));
}
