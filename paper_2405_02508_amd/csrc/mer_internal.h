// mer_internal.h -- launchers shared between the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "mer_device.h"

namespace mer {
constexpr int kBinBlock = 256;  // threads per workgroup of the binning passes (one triangle each)

// attr/out (nullable): interpolate in the resolve, as launch_interpolate would
int launch_rasterize(const mer_plan* P, const mer_view* views, const float* v, const int32_t* tri, int32_t* tri_id,
                     float* depth, float* bary, const float* attr, int C_a, int append_z, float* out, void* ws,
                     hipStream_t st);
int launch_interpolate(const mer_plan* P, const mer_view* views, const float* attr, int C_a, const float* v,
                       const int32_t* tri, const int32_t* tri_id, const float* bary, int append_z, float* out,
                       hipStream_t st);
int launch_transform(const mer_plan* P, const mer_view* views, const mer_camera* cams, const float* v_world,
                     float* v_screen, void* ws, hipStream_t st);
int launch_transform_bwd(const mer_plan* P, const mer_view* views, const mer_camera* cams, const float* v_world,
                         const float* g_screen, float* g_world, void* ws, hipStream_t st);
int launch_backface(const mer_plan* P, const mer_view* views, const float* v, const int32_t* tri,
                    const int32_t* tri_id, float* out, hipStream_t st);
// g: dL/d(img) rows of ld_g floats, or NULL with target != NULL for the fused
// L2 loss (dL/d(img) = 2 w (img - target), loss += w sum (img - target)^2).
// Scratch: tab, 2 (n_views + 1) int64 (the 16x16 tile prefix per view, written
// here); loss_part, 4 total_btiles floats (per-wave loss partials, written
// here; only read when loss != NULL).
int launch_backward(const mer_plan* P, const mer_view* views, const float* v, const int32_t* tri,
                    const int32_t* tri_id, const float* attr, int C_a, int append_z, const float* img,
                    const float* g, const float* target, float w_l2, float* loss, int C_e, int ld_g, int flags,
                    float* g_attr, float* g_v, long long* tab, float* loss_part, hipStream_t st);
// forward-mode image tangent (flags: MER_NO_INTERSECT, MER_SKIP_EDGE, MER_SKIP_INTERP)
int launch_jvp(const mer_plan* P, const mer_view* views, const float* v, const int32_t* tri, const int32_t* tri_id,
               const float* attr, const float* dattr, int C_a, int append_z, const float* img, int C_e,
               const float* dv, int flags, float* dimg, void* ws, hipStream_t st);
// bilinear clamp-to-edge texture sampling and its adjoint
int launch_texture(const mer_plan* P, const mer_view* views, const int32_t* tri_id, const float* uv, int ld_uv,
                   const float* tex, int th, int tw, int C, float* out, hipStream_t st);
int launch_texture_bwd(const mer_plan* P, const mer_view* views, const int32_t* tri_id, const float* uv, int ld_uv,
                       const float* tex, int th, int tw, int C, const float* g_out, float* g_tex, float* g_uv,
                       void* ws, hipStream_t st);
// per-view prefix tables (triangles, tiles of 2^tw_log2 x 2^th_log2) and status reset
__global__ void __launch_bounds__(1024) k_prep(const mer_view* __restrict__ views, int n_views, int tw_log2, int th_log2,
                       long long* __restrict__ tri_base, long long* __restrict__ tile_base,
                       long long* __restrict__ status);
}  // namespace mer
