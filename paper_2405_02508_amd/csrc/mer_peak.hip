// mer_peak.hip -- reference kernels for the rooflines the benchmark reports
// the micro-edge kernels against: a plain streaming copy (the HBM bandwidth
// a simple kernel reaches on this chip) and float atomic adds into a buffer
// of a given footprint (the rate of device-scope float atomics, which bound
// the gradient scatter).  Built into its own library, libmer_peak.so; the
// micro-edge library does not use it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mer_peak.h"

namespace {

// Grid-stride copy, 16 bytes per lane per iteration.
__global__ void __launch_bounds__(256) k_copy16(const float4* __restrict__ src, float4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Float atomic adds: lane i of the grid adds 1.0f to element
// (i + r * stride) mod footprint for r = 0 .. per_lane - 1, so a wave's 64
// adds hit 64 consecutive floats (two 128-byte lines) and the grid sweeps the
// footprint; no address is touched twice within one round.
__global__ void __launch_bounds__(256) k_atomic_add(float* __restrict__ buf, int64_t footprint, int per_lane) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t a = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) % footprint;
  const int64_t step = stride % footprint;
  for (int r = 0; r < per_lane; ++r) {
    atomicAdd(buf + a, 1.0f);
    a += step;
    if (a >= footprint) a -= footprint;
  }
}

}  // namespace

extern "C" {

int mer_peak_copy(const float* src, float* dst, int64_t n_floats, void* stream) {
  if (!src || !dst || n_floats < 4 || (n_floats & 3) || (((uintptr_t)src | (uintptr_t)dst) & 15)) return -1;
  const int64_t n = n_floats / 4;
  const int64_t blocks = (n + 255) / 256 < 256 * 64 ? (n + 255) / 256 : 256 * 64;
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (const float4*)src,
                     (float4*)dst, n);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int mer_peak_atomic_add(float* buf, int64_t footprint, int64_t lanes, int per_lane, void* stream) {
  if (!buf || footprint < 1 || lanes < 256 || (lanes & 255) || per_lane < 1 || lanes / 256 > 0x7fffffff) return -1;
  hipLaunchKernelGGL(k_atomic_add, dim3((unsigned)(lanes / 256)), dim3(256), 0, (hipStream_t)stream, buf, footprint,
                     per_lane);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
