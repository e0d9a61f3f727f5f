// mer_transform.hip -- vertex transform module and its backward (supplement,
// "Implementation detail": vertices to the camera frame, then projected onto
// the image plane; the backward pass is the derivative of that map).
//
//   k_vprep          per-view prefix of screen-vertex counts (one block)
//   k_transform      one thread per (view, vertex): camera frame, projection
//   k_transform_bwd  one thread per (view, vertex): J^T g into the world
//                    vertex with float atomics (views of one mesh share rows)
#include "mer_internal.h"

namespace mer {

__global__ void __launch_bounds__(1024) k_vprep(const mer_view* __restrict__ views, int n_views,
                                                long long* __restrict__ vbase) {
  __shared__ long long s_v[1024];
  const int tid = threadIdx.x;
  const int per = (n_views + 1023) / 1024;
  const int lo = tid * per, hi = min(n_views, lo + per);
  long long a = 0;
  for (int i = lo; i < hi; ++i) a += views[i].n_v;
  s_v[tid] = a;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const long long x = tid >= off ? s_v[tid - off] : 0;
    __syncthreads();
    s_v[tid] += x;
    __syncthreads();
  }
  long long e = s_v[tid] - a;
  for (int i = lo; i < hi; ++i) {
    vbase[i] = e;
    e += views[i].n_v;
  }
  if (tid == 1023) vbase[n_views] = s_v[1023];
}

// Camera-frame position of world vertex pw: R (pw - C), each row summed in a
// fixed order (the library is built without fused multiply-add).
__device__ __forceinline__ void cam_frame(const mer_camera& c, const float* pw, float pc[3]) {
  const float d0 = pw[0] - c.C[0], d1 = pw[1] - c.C[1], d2 = pw[2] - c.C[2];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    float a = c.R[3 * r] * d0;
    a = a + c.R[3 * r + 1] * d1;
    a = a + c.R[3 * r + 2] * d2;
    pc[r] = a;
  }
}

__global__ void __launch_bounds__(256) k_transform(const mer_view* __restrict__ views, int n_views,
                                                   const mer_camera* __restrict__ cams,
                                                   const long long* __restrict__ vbase, long long total_v,
                                                   const float* __restrict__ v_world, float* __restrict__ v_screen) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int vi = wave_bucket(vbase, n_views, g < total_v ? g : total_v - 1);
  if (g >= total_v) return;
  const mer_view vw = views[vi];
  const mer_camera c = cams[vi];
  const long long j = g - vbase[vi];
  float pc[3];
  cam_frame(c, v_world + (c.w_off + j) * 3, pc);
  float* o = v_screen + (vw.v_off + j) * 3;
  o[0] = c.f * pc[0] / pc[2] + c.cx;
  o[1] = c.f * pc[1] / pc[2] + c.cy;
  o[2] = pc[2];
}

__global__ void __launch_bounds__(256) k_transform_bwd(const mer_view* __restrict__ views, int n_views,
                                                       const mer_camera* __restrict__ cams,
                                                       const long long* __restrict__ vbase, long long total_v,
                                                       const float* __restrict__ v_world,
                                                       const float* __restrict__ g_screen,
                                                       float* __restrict__ g_world) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int vi = wave_bucket(vbase, n_views, g < total_v ? g : total_v - 1);
  if (g >= total_v) return;
  const mer_view vw = views[vi];
  const mer_camera c = cams[vi];
  const long long j = g - vbase[vi];
  float pc[3];
  cam_frame(c, v_world + (c.w_off + j) * 3, pc);
  const float* gs = g_screen + (vw.v_off + j) * 3;
  // x_px = f x / z + cx, y_px = f y / z + cy, z_out = z  (x, y, z: camera frame)
  const float iz = 1.0f / pc[2];
  const float fz = c.f * iz;
  const float gx = gs[0] * fz, gy = gs[1] * fz;
  const float gz = gs[2] - (gx * pc[0] + gy * pc[1]) * iz;
  // camera frame = R (world - C): the world gradient is R^T (gx, gy, gz)
  float* o = g_world + (c.w_off + j) * 3;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float a = c.R[k] * gx;
    a = a + c.R[3 + k] * gy;
    a = a + c.R[6 + k] * gz;
    if (a != 0.f) atomicAdd(o + k, a);
  }
}

int launch_transform(const mer_plan* P, const mer_view* views, const mer_camera* cams, const float* v_world,
                     float* v_screen, void* ws, hipStream_t st) {
  long long* vbase = (long long*)((char*)ws + P->off_vbase);
  hipLaunchKernelGGL(k_vprep, dim3(1), dim3(1024), 0, st, views, P->n_views, vbase);
  if (P->total_v > 0)
    hipLaunchKernelGGL(k_transform, dim3((unsigned)((P->total_v + 255) / 256)), dim3(256), 0, st, views, P->n_views,
                       cams, vbase, P->total_v, v_world, v_screen);
  return hipGetLastError() == hipSuccess ? MER_OK : MER_ELAUNCH;
}

int launch_transform_bwd(const mer_plan* P, const mer_view* views, const mer_camera* cams, const float* v_world,
                         const float* g_screen, float* g_world, void* ws, hipStream_t st) {
  long long* vbase = (long long*)((char*)ws + P->off_vbase);
  hipLaunchKernelGGL(k_vprep, dim3(1), dim3(1024), 0, st, views, P->n_views, vbase);
  if (P->total_v > 0)
    hipLaunchKernelGGL(k_transform_bwd, dim3((unsigned)((P->total_v + 255) / 256)), dim3(256), 0, st, views,
                       P->n_views, cams, vbase, P->total_v, v_world, g_screen, g_world);
  return hipGetLastError() == hipSuccess ? MER_OK : MER_ELAUNCH;
}

}  // namespace mer
