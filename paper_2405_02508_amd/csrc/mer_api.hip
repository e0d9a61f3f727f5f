// mer_api.hip -- the C ABI (include/mer.h): plan, argument checks, launches,
// status.  No call allocates device memory or synchronises (mer_status aside).
#include <limits.h>
#include <cmath>
#include <mutex>
#include <string.h>

#include "mer_internal.h"

namespace {

constexpr int kVersion = 1;

int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

bool tile_supported(int w, int h) {
  return (w == 8 && h == 8) || (w == 16 && h == 16) || (w == 32 && h == 8) || (w == 16 && h == 8);
}

}  // namespace

extern "C" {

int mer_version(void) { return kVersion; }

const char* mer_strerror(int code) {
  switch (code) {
    case MER_OK: return "ok";
    case MER_EINVAL: return "invalid argument";
    case MER_EWORKSPACE: return "workspace missing or inconsistent with the plan";
    case MER_ELAUNCH: return "kernel launch failed";
    case MER_ETUNING: return "unsupported tile shape";
    case MER_EINTERNAL: return "binning integrity check failed (library defect)";
    case MER_ESCRATCH: return "the plan needs more than the fixed scratch of the no-workspace call";
    default: return "unknown error";
  }
}

int mer_plan_init(const mer_view* views, int n_views, const mer_tuning* tun, mer_plan* P) {
  if (!views || !P || n_views < 1) return MER_EINVAL;
  const int tw = tun ? tun->tile_w : 8, th = tun ? tun->tile_h : 8;
  if (!tile_supported(tw, th)) return MER_ETUNING;
  memset(P, 0, sizeof(*P));
  int64_t tris = 0, tiles = 0, btiles = 0, px_end = 0, verts = 0;
  for (int i = 0; i < n_views; ++i) {
    const mer_view& w = views[i];
    if (w.H < 1 || w.W < 1 || w.H > 32767 || w.W > 32767) return MER_EINVAL;
    if (w.n_v < 0 || w.n_t < 0 || w.v_off < 0 || w.t_off < 0 || w.a_off < 0 || w.px_off < 0) return MER_EINVAL;
    if (w.px_off < px_end) return MER_EINVAL;  // views packed in order, no overlap
    px_end = w.px_off + (int64_t)w.H * w.W;
    tris += w.n_t;
    verts += w.n_v;
    tiles += (int64_t)((w.W + tw - 1) / tw) * ((w.H + th - 1) / th);
    btiles += (int64_t)((w.W + 15) / 16) * ((w.H + 15) / 16);
  }
  if (tris > INT_MAX || tiles >= INT_MAX || btiles >= INT_MAX) return MER_EINVAL;
  P->n_views = n_views;
  P->px_begin = views[0].px_off;
  P->tile_w = tw;
  P->tile_h = th;
  P->total_tris = tris;
  P->total_tiles = tiles;
  P->total_btiles = btiles;
  P->total_px = px_end;
  P->total_v = verts;
  int64_t cap = (tun && tun->bin_cap > 0) ? tun->bin_cap : 16 * tris + 16 * tiles + 4096;
  if (cap > INT_MAX - 1) cap = INT_MAX - 1;  // a saturated bin offset (INT_MAX) always overflows
  P->bin_cap = cap;
  P->small_px = (tun && tun->small_px != 0) ? (tun->small_px < 0 ? 0 : tun->small_px) : 16;
  P->big_tiles = (tun && tun->big_tiles != 0) ? (tun->big_tiles < 0 ? INT_MAX : tun->big_tiles) : 16;
  P->n_part = (tiles + 1023) / 1024;
  int64_t off = 0;
  P->off_viewtab = off;
  off = align256(off + 2 * (int64_t)(n_views + 1) * 8);
  P->off_rec = off;
  off = align256(off + tris * 64);
  P->off_bbox = off;
  off = align256(off + tris * 8);
  P->off_count = off;
  off = align256(off + tiles * 4);
  P->off_offs = off;
  off = align256(off + (tiles + 1) * 4);
  P->off_part = off;
  off = align256(off + P->n_part * 8);
  P->off_bins = off;
  off = align256(off + cap * 4);
  P->off_status = off;
  off = align256(off + 8 * 8);
  P->off_key = off;
  off = align256(off + (px_end - P->px_begin) * 8);
  P->off_bviewtab = off;
  off = align256(off + 2 * (int64_t)(n_views + 1) * 8);
  P->off_vbase = off;
  off = align256(off + (int64_t)(n_views + 1) * 8);
  P->off_bloss = off;
  off = align256(off + btiles * 4 * 4);  // one float per wave
  const int64_t bin_groups = (tris + mer::kBinBlock - 1) / mer::kBinBlock;
  P->off_big = off;
  off = align256(off + bin_groups * mer::kBinBlock * 4);
  P->n_bingroups = bin_groups;
  P->off_bign = off;
  off = align256(off + (bin_groups * 2 + 1) * 4);  // list lengths, then their offsets
  P->off_bigpart = off;
  off = align256(off + (bin_groups + 1023) / 1024 * 8);
  P->off_bigflat = off;
  off = align256(off + tris * 4);
  P->ws_bytes = off;
  return MER_OK;
}

static bool plan_ok(const mer_plan* P) {
  return P && P->n_views >= 1 && P->ws_bytes > 0 && tile_supported(P->tile_w, P->tile_h);
}

// The backward calls' scratch inside the plan's workspace.
static long long* bwd_tab(const mer_plan* P, void* ws) { return (long long*)((char*)ws + P->off_bviewtab); }
static float* bwd_loss(const mer_plan* P, void* ws) { return (float*)((char*)ws + P->off_bloss); }

int mer_rasterize(const mer_plan* P, const mer_view* views_dev, const float* v, const int32_t* tri, int32_t* tri_id,
                  float* depth, float* bary, void* ws, void* stream) {
  if (!plan_ok(P) || !views_dev || !tri_id || (P->total_tris > 0 && (!v || !tri))) return MER_EINVAL;
  if (!ws) return MER_EWORKSPACE;
  return mer::launch_rasterize(P, views_dev, v, tri, tri_id, depth, bary, nullptr, 0, 0, nullptr, ws,
                               (hipStream_t)stream);
}

int mer_rasterize_interpolate(const mer_plan* P, const mer_view* views_dev, const float* v, const int32_t* tri,
                              int32_t* tri_id, float* depth, float* bary, const float* attr, int C_a, int append_z,
                              float* out, void* ws, void* stream) {
  if (!plan_ok(P) || !views_dev || !tri_id || !attr || !out || !tri || C_a < 1 || C_a + (append_z ? 1 : 0) > 64)
    return MER_EINVAL;
  if (P->total_tris > 0 && !v) return MER_EINVAL;
  if (append_z && !v) return MER_EINVAL;
  if (!ws) return MER_EWORKSPACE;
  return mer::launch_rasterize(P, views_dev, v, tri, tri_id, depth, bary, attr, C_a, append_z ? 1 : 0, out, ws,
                               (hipStream_t)stream);
}

int mer_interpolate(const mer_plan* P, const mer_view* views_dev, const float* attr, int C_a, const float* v,
                    const int32_t* tri, const int32_t* tri_id, const float* bary, int append_z, float* out,
                    void* stream) {
  if (!plan_ok(P) || !views_dev || !attr || !tri || !tri_id || !out || C_a < 1 || C_a + (append_z ? 1 : 0) > 64)
    return MER_EINVAL;
  if ((append_z || !bary) && !v) return MER_EINVAL;
  return mer::launch_interpolate(P, views_dev, attr, C_a, v, tri, tri_id, bary, append_z ? 1 : 0, out,
                                 (hipStream_t)stream);
}

int mer_transform(const mer_plan* P, const mer_view* views_dev, const mer_camera* cams_dev, const float* v_world,
                  float* v_screen, void* ws, void* stream) {
  if (!plan_ok(P) || !views_dev || !cams_dev || !v_world || !v_screen) return MER_EINVAL;
  if (!ws) return MER_EWORKSPACE;
  return mer::launch_transform(P, views_dev, cams_dev, v_world, v_screen, ws, (hipStream_t)stream);
}

int mer_transform_bwd(const mer_plan* P, const mer_view* views_dev, const mer_camera* cams_dev,
                      const float* v_world, const float* g_screen, float* g_world, void* ws, void* stream) {
  if (!plan_ok(P) || !views_dev || !cams_dev || !v_world || !g_screen || !g_world) return MER_EINVAL;
  if (!ws) return MER_EWORKSPACE;
  return mer::launch_transform_bwd(P, views_dev, cams_dev, v_world, g_screen, g_world, ws, (hipStream_t)stream);
}

int mer_backface(const mer_plan* P, const mer_view* views_dev, const float* v, const int32_t* tri,
                 const int32_t* tri_id, float* out, void* stream) {
  if (!plan_ok(P) || !views_dev || !v || !tri || !tri_id || !out) return MER_EINVAL;
  return mer::launch_backface(P, views_dev, v, tri, tri_id, out, (hipStream_t)stream);
}

int mer_edge_grad(const mer_plan* P, const mer_view* views_dev, const float* v, const int32_t* tri,
                  const int32_t* tri_id, const float* img, const float* g_img, int C_e, int flags, float* g_v,
                  void* ws, void* stream) {
  if (!plan_ok(P) || !views_dev || !v || !tri || !tri_id || !img || !g_img || !g_v || C_e < 1 || C_e > 64)
    return MER_EINVAL;
  if (!ws) return MER_EWORKSPACE;
  return mer::launch_backward(P, views_dev, v, tri, tri_id, nullptr, 0, 0, img, g_img, nullptr, 0.f, nullptr, C_e, C_e,
                              (flags & MER_NO_INTERSECT) | MER_SKIP_INTERP, nullptr, g_v, bwd_tab(P, ws), bwd_loss(P, ws),
                              (hipStream_t)stream);
}

int mer_interpolate_bwd(const mer_plan* P, const mer_view* views_dev, const float* attr, int C_a, const float* v,
                        const int32_t* tri, const int32_t* tri_id, int append_z, const float* g_out, int ld_out,
                        float* g_attr, float* g_v, void* ws, void* stream) {
  const int C = C_a + (append_z ? 1 : 0);
  if (!plan_ok(P) || !views_dev || !attr || !v || !tri || !tri_id || !g_out || C_a < 1 || C_a > 64 || ld_out < C)
    return MER_EINVAL;
  if (!ws) return MER_EWORKSPACE;
  if (!g_attr && !g_v) return MER_OK;
  return mer::launch_backward(P, views_dev, v, tri, tri_id, attr, C_a, append_z ? 1 : 0, nullptr, g_out, nullptr,
                              0.f, nullptr, ld_out,
                              ld_out, MER_SKIP_EDGE, g_attr, g_v, bwd_tab(P, ws), bwd_loss(P, ws), (hipStream_t)stream);
}

int mer_backward_fused(const mer_plan* P, const mer_view* views_dev, const float* v, const int32_t* tri,
                       const int32_t* tri_id, const float* attr, int C_a, int append_z, const float* img,
                       const float* g_img, int C_e, int flags, float* g_attr, float* g_v, void* ws, void* stream) {
  const int C = C_a + (append_z ? 1 : 0);
  if (!plan_ok(P) || !views_dev || !v || !tri || !tri_id || !g_img || C_e < 1 || C_e > 64) return MER_EINVAL;
  if (!(flags & MER_SKIP_EDGE) && (!img || !g_v)) return MER_EINVAL;
  if (!(flags & MER_SKIP_INTERP) && (!attr || C_a < 1 || C_a > 64 || C > C_e)) return MER_EINVAL;
  if (!ws) return MER_EWORKSPACE;
  return mer::launch_backward(P, views_dev, v, tri, tri_id, attr, C_a, append_z ? 1 : 0, img, g_img, nullptr, 0.f,
                              nullptr, C_e, C_e, flags & (MER_NO_INTERSECT | MER_SKIP_EDGE | MER_SKIP_INTERP), g_attr,
                              g_v, bwd_tab(P, ws), bwd_loss(P, ws), (hipStream_t)stream);
}

int mer_backward_l2(const mer_plan* P, const mer_view* views_dev, const float* v, const int32_t* tri,
                    const int32_t* tri_id, const float* attr, int C_a, int append_z, const float* img,
                    const float* target, float weight, int C_e, int flags, float* g_attr, float* g_v, float* loss,
                    void* ws, void* stream) {
  const int C = C_a + (append_z ? 1 : 0);
  if (!plan_ok(P) || !views_dev || !v || !tri || !tri_id || !img || !target || C_e < 1 || C_e > 64)
    return MER_EINVAL;
  if (!std::isfinite(weight)) return MER_EINVAL;
  if (!(flags & MER_SKIP_EDGE) && !g_v) return MER_EINVAL;
  if (!(flags & MER_SKIP_INTERP) && (!attr || C_a < 1 || C_a > 64 || C > C_e)) return MER_EINVAL;
  if (!ws) return MER_EWORKSPACE;
  return mer::launch_backward(P, views_dev, v, tri, tri_id, attr, C_a, append_z ? 1 : 0, img, nullptr, target, weight,
                              loss, C_e, C_e, flags & (MER_NO_INTERSECT | MER_SKIP_EDGE | MER_SKIP_INTERP), g_attr,
                              g_v, bwd_tab(P, ws), bwd_loss(P, ws), (hipStream_t)stream);
}

int mer_jvp(const mer_plan* P, const mer_view* views_dev, const float* v, const int32_t* tri,
            const int32_t* tri_id, const float* attr, const float* dattr, int C_a, int append_z, const float* img,
            int C_e, const float* dv, int flags, float* dimg, void* ws, void* stream) {
  const int C = C_a + (append_z ? 1 : 0);
  if (!plan_ok(P) || !views_dev || !v || !tri || !tri_id || !dimg || C_e < 1 || C_e > 64) return MER_EINVAL;
  if (!(flags & MER_SKIP_EDGE) && dv && !img) return MER_EINVAL;
  if (!(flags & MER_SKIP_INTERP) && (!attr || C_a < 1 || C_a > 64 || C > C_e)) return MER_EINVAL;
  if (!ws) return MER_EWORKSPACE;
  return mer::launch_jvp(P, views_dev, v, tri, tri_id, attr, dattr, C_a, append_z ? 1 : 0, img, C_e, dv,
                         flags & (MER_NO_INTERSECT | MER_SKIP_EDGE | MER_SKIP_INTERP), dimg, ws,
                         (hipStream_t)stream);
}

int mer_texture(const mer_plan* P, const mer_view* views_dev, const int32_t* tri_id, const float* uv, int ld_uv,
                const float* tex, int tex_h, int tex_w, int C_t, float* out, void* stream) {
  if (!plan_ok(P) || !views_dev || !uv || !tex || !out || ld_uv < 2 || tex_h < 1 || tex_w < 1 || C_t < 1 ||
      C_t > 64)
    return MER_EINVAL;
  return mer::launch_texture(P, views_dev, tri_id, uv, ld_uv, tex, tex_h, tex_w, C_t, out, (hipStream_t)stream);
}

int mer_texture_bwd(const mer_plan* P, const mer_view* views_dev, const int32_t* tri_id, const float* uv, int ld_uv,
                    const float* tex, int tex_h, int tex_w, int C_t, const float* g_out, float* g_tex, float* g_uv,
                    void* ws, void* stream) {
  if (!plan_ok(P) || !views_dev || !uv || !tex || !g_out || ld_uv < 2 || tex_h < 1 || tex_w < 1 || C_t < 1 ||
      C_t > 64 || (long long)tex_h * tex_w > 2147483647ll)
    return MER_EINVAL;
  if (!ws) return MER_EWORKSPACE;
  if (!g_tex && !g_uv) return MER_OK;
  return mer::launch_texture_bwd(P, views_dev, tri_id, uv, ld_uv, tex, tex_h, tex_w, C_t, g_out, g_tex, g_uv, ws,
                                 (hipStream_t)stream);
}

}  // extern "C"

// ------------------------------------------------ no-workspace backward
// Fixed device scratch of mer_backward_l2_noalloc: every GPU the library runs
// on holds one copy until the process ends.  In host code `scratch` only
// names the symbol; its device address (per device) comes from
// hipGetSymbolAddress, taken once per device with that device current.
namespace {
constexpr size_t kScratchBytes = (size_t)MER_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// Device address of the current device's scratch, or nullptr on failure.
void* scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}
}  // namespace

extern "C" {

int mer_backward_l2_noalloc(const mer_plan* P, const mer_view* views_dev, const float* v, const int32_t* tri,
                            const int32_t* tri_id, const float* attr, int C_a, int append_z, const float* img,
                            const float* target, float weight, int C_e, int flags, float* g_attr, float* g_v,
                            float* loss, void* stream) {
  const int C = C_a + (append_z ? 1 : 0);
  if (!plan_ok(P) || !views_dev || !v || !tri || !tri_id || !img || !target || C_e < 1 || C_e > 64)
    return MER_EINVAL;
  if (!std::isfinite(weight)) return MER_EINVAL;
  if (!(flags & MER_SKIP_EDGE) && !g_v) return MER_EINVAL;
  if (!(flags & MER_SKIP_INTERP) && (!attr || C_a < 1 || C_a > 64 || C > C_e)) return MER_EINVAL;
  // the scratch holds the per-view tile prefix, then the per-wave loss partials
  const int64_t tab_bytes = align256(2 * (int64_t)(P->n_views + 1) * 8);
  const int64_t need = tab_bytes + (loss ? 4 * P->total_btiles * (int64_t)sizeof(float) : 0);
  if (need > (int64_t)kScratchBytes) return MER_ESCRATCH;
  char* base = (char*)scratch_address();
  if (!base) return MER_ELAUNCH;
  return mer::launch_backward(P, views_dev, v, tri, tri_id, attr, C_a, append_z ? 1 : 0, img, nullptr, target, weight,
                              loss, C_e, C_e, flags & (MER_NO_INTERSECT | MER_SKIP_EDGE | MER_SKIP_INTERP), g_attr,
                              g_v, (long long*)base, (float*)(base + tab_bytes), (hipStream_t)stream);
}

int mer_status(const mer_plan* P, const void* ws, void* stream, int64_t out[6]) {
  if (!plan_ok(P) || !out) return MER_EINVAL;
  if (!ws) return MER_EWORKSPACE;
  long long st[8];
  if (hipMemcpyAsync(st, (const char*)ws + P->off_status, sizeof(st), hipMemcpyDeviceToHost, (hipStream_t)stream) !=
      hipSuccess)
    return MER_ELAUNCH;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return MER_ELAUNCH;
  out[0] = st[0];
  out[1] = st[1];
  out[2] = st[2];
  out[3] = P->bin_cap;
  out[4] = st[5];
  out[5] = st[6];
  return (st[5] != 0 || st[6] != 0) ? MER_EINTERNAL : MER_OK;
}

}  // extern "C"
