// mer_texture.hip -- deferred texturing: a texture sampled at per-pixel uv
// coordinates (which the interpolator produces from per-vertex uv), and its
// adjoint to the texture and to uv (supplement, "Implementation detail":
// uv interpolated per pixel, then a neural texture sampled in a deferred
// shading step; Sec. 3 lists the texture sampler among the parts the smooth
// term differentiates through).
//
// Bilinear filtering, clamp-to-edge addressing.  Texel (x, y) of a th x tw
// texture is centred at ((x + 1/2) / tw, (y + 1/2) / th); s = u tw - 1/2 and
// t = v th - 1/2 are clamped to [-1, tw] and [-1, th], x0 = floor(s),
// fx = s - x0 (likewise y0, fy), and texels (x0 + i, y0 + j) are read with
// each index clamped into the texture.
#include "mer_internal.h"

namespace mer {

struct TexCell {
  int x[2], y[2];  // clamped texel indices
  float fx, fy;
  bool ok;         // sampled (covered pixel, finite uv)
};

// want == false gives an unsampled cell (indices 0).  The texel coordinate
// is formed in binary64: u * tw for tw ~ 1000 would otherwise lose the
// fraction's low bits (binary32 spacing 2^-14 at 1000).
__device__ __forceinline__ TexCell tex_cell(bool want, float u, float v, int th, int tw) {
  TexCell c;
  c.ok = want && isfinite(u) && isfinite(v);
  double s = c.ok ? (double)u * (double)tw - 0.5 : 0.0;
  double t = c.ok ? (double)v * (double)th - 0.5 : 0.0;
  s = fmin(fmax(s, -1.0), (double)tw);
  t = fmin(fmax(t, -1.0), (double)th);
  const double x0 = floor(s), y0 = floor(t);
  c.fx = (float)(s - x0);
  c.fy = (float)(t - y0);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    c.x[i] = c.ok ? min(max((int)x0 + i, 0), tw - 1) : 0;
    c.y[i] = c.ok ? min(max((int)y0 + i, 0), th - 1) : 0;
  }
  return c;
}

// Pixel p's view (searched once per wave, then per lane only across a view
// end) and whether p lies inside it (not in a gap between views).
__device__ __forceinline__ bool pixel_in_view(const mer_view* views, int n_views, long long p, int wvi) {
  int vi = wvi;
  if (vi + 1 < n_views && p >= views[vi + 1].px_off) vi = find_view_px(views, n_views, p);
  const mer_view& vw = views[vi];
  const long long local = p - vw.px_off;
  return local >= 0 && local < (long long)vw.H * vw.W;
}

// ---------------------------------------------------------------- forward
// One thread per pixel: out[p, :] = bilinear sample, or 0.  V4: C is a
// multiple of 4 and tex, out are 16-byte aligned, so texel rows and output
// rows move as float4.
template <bool V4>
__global__ void __launch_bounds__(256) k_texture(const mer_view* __restrict__ views, int n_views,
                                                 const int32_t* __restrict__ tri_id, const float* __restrict__ uv,
                                                 int ld_uv, const float* __restrict__ tex, int th, int tw, int C,
                                                 float* __restrict__ out, long long px_begin, long long total_px) {
  const long long p = px_begin + (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int wvi = wave_view(views, n_views, p - (threadIdx.x & 63));
  // the wave's view through scalar loads; lanes past its end (a wave across
  // two views) look theirs up
  const long long off0 = views[wvi].px_off, n0 = (long long)views[wvi].H * views[wvi].W;
  bool in = p < total_px && p - off0 < n0;
  if (__builtin_amdgcn_ballot_w64(p < total_px && p - off0 >= n0))
    in = p < total_px && pixel_in_view(views, n_views, p, wvi);
  if (!in) return;
  float* o = out + p * C;
  // the uv row (every pixel has one) and the index in flight together
  const float u = uv[p * ld_uv], v = uv[p * ld_uv + 1];
  const int tid = tri_id ? tri_id[p] : 0;
  const bool want = tid >= 0;
  const TexCell cell = tex_cell(want, u, v, th, tw);
  if (!cell.ok) {
    if constexpr (V4) {
      for (int c = 0; c < C; c += 4) *reinterpret_cast<float4*>(o + c) = make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
      for (int c = 0; c < C; ++c) o[c] = 0.f;
    }
    return;
  }
  const float w00 = (1.0f - cell.fx) * (1.0f - cell.fy), w10 = cell.fx * (1.0f - cell.fy);
  const float w01 = (1.0f - cell.fx) * cell.fy, w11 = cell.fx * cell.fy;
  const float* t00 = tex + ((long long)cell.y[0] * tw + cell.x[0]) * C;
  const float* t10 = tex + ((long long)cell.y[0] * tw + cell.x[1]) * C;
  const float* t01 = tex + ((long long)cell.y[1] * tw + cell.x[0]) * C;
  const float* t11 = tex + ((long long)cell.y[1] * tw + cell.x[1]) * C;
  if constexpr (V4) {
    auto mix = [&](float4 a, float4 b, float4 d, float4 e) {
      float4 r;
      r.x = (w00 * a.x + w10 * b.x) + (w01 * d.x + w11 * e.x);
      r.y = (w00 * a.y + w10 * b.y) + (w01 * d.y + w11 * e.y);
      r.z = (w00 * a.z + w10 * b.z) + (w01 * d.z + w11 * e.z);
      r.w = (w00 * a.w + w10 * b.w) + (w01 * d.w + w11 * e.w);
      return r;
    };
    auto ld = [](const float* q) { return *reinterpret_cast<const float4*>(q); };
    int c = 0;
    for (; c + 8 <= C; c += 8) {  // eight channels: all eight texel loads before the arithmetic
      const float4 a0 = ld(t00 + c), b0 = ld(t10 + c), d0 = ld(t01 + c), e0 = ld(t11 + c);
      const float4 a1 = ld(t00 + c + 4), b1 = ld(t10 + c + 4), d1 = ld(t01 + c + 4), e1 = ld(t11 + c + 4);
      *reinterpret_cast<float4*>(o + c) = mix(a0, b0, d0, e0);
      *reinterpret_cast<float4*>(o + c + 4) = mix(a1, b1, d1, e1);
    }
    if (c < C) *reinterpret_cast<float4*>(o + c) = mix(ld(t00 + c), ld(t10 + c), ld(t01 + c), ld(t11 + c));
  } else {
    for (int c = 0; c < C; ++c) o[c] = (w00 * t00[c] + w10 * t10[c]) + (w01 * t01[c] + w11 * t11[c]);
  }
}

// --------------------------------------------------------------- backward
// One workgroup per 16x16 pixel tile of one view.  g_uv is written per
// pixel.  The texture gradient is summed in LDS over the box of texels the
// tile touches when that box holds at most kTexWin values (then one global
// atomic per touched texel channel), else added straight to memory.
//
// The LDS sums are 64-bit fixed point: LDS float atomics cost about one
// cycle per active lane on this chip, integer ones a few cycles per
// instruction.  With M the tile's largest |dL/d(out)| (every contribution
// w g has |w g| <= M, and a texel takes at most 4 x 256 of them) and
// M < 2^e, contributions are scaled by 2^(51 - e) and rounded to integers:
// the sums stay below 2^61, each contribution is rounded by at most
// 2^(e - 52) <= 2^-51 M, and the sum is exact and independent of order.  A
// tile with a non-finite dL/d(out) adds straight to memory instead.
constexpr int kTexWin = 3072;

// round(x s) to the nearest integer (ties to even) for |x s| < 2^51, as the
// bits of a 64-bit integer: x s + 1.5 2^52 lies in [2^52, 2^53), where the
// binary64 spacing is 1, so the one rounding of the fused multiply-add is
// the rounding to an integer, and the integer is the difference of the sum's
// bits and the constant's
__device__ __forceinline__ unsigned long long fixed_round(float x, double s) {
  const double magic = 6755399441055744.0;  // 1.5 * 2^52
  return (unsigned long long)(__double_as_longlong(fma((double)x, s, magic)) - __double_as_longlong(magic));
}

template <bool V4>
__global__ void __launch_bounds__(256) k_texture_bwd(const mer_view* __restrict__ views, int n_views,
                                                     const long long* __restrict__ btile_base,
                                                     const int32_t* __restrict__ tri_id,
                                                     const float* __restrict__ uv, int ld_uv,
                                                     const float* __restrict__ tex, int th, int tw, int C,
                                                     const float* __restrict__ g_out, float* __restrict__ g_tex,
                                                     float* __restrict__ g_uv) {
  __shared__ unsigned long long s_acc[kTexWin];
  __shared__ int s_box[6];  // x min, y min, -x max, -y max, bits of max |g|, any non-finite g
  const long long tile = xcd_tile(blockIdx.x, gridDim.x);
  const int vi = __builtin_amdgcn_readfirstlane(find_bucket(btile_base, n_views, tile));
  const mer_view vw = views[vi];
  const long long local_tile = tile - btile_base[vi];
  const int tiles_x = (vw.W + 15) >> 4;
  int px, py;
  grid_xy(local_tile, tiles_x, px, py);
  px = px * 16 + (threadIdx.x & 15);
  py = py * 16 + (threadIdx.x >> 4);
  const bool inside = px < vw.W && py < vw.H;
  const long long p = vw.px_off + (long long)py * vw.W + px;
  if (threadIdx.x < 4) s_box[threadIdx.x] = 0x7fffffff;
  if (threadIdx.x == 4 || threadIdx.x == 5) s_box[threadIdx.x] = 0;

  const bool want = inside && (!tri_id || tri_id[p] >= 0);
  const TexCell cell = tex_cell(want, want ? uv[p * ld_uv] : 0.f, want ? uv[p * ld_uv + 1] : 0.f, th, tw);
  const float* g = g_out + (cell.ok ? p : 0) * C;
  const float w00 = (1.0f - cell.fx) * (1.0f - cell.fy), w10 = cell.fx * (1.0f - cell.fy);
  const float w01 = (1.0f - cell.fx) * cell.fy, w11 = cell.fx * cell.fy;
  const long long r00 = ((long long)cell.y[0] * tw + cell.x[0]) * C, r10 = ((long long)cell.y[0] * tw + cell.x[1]) * C;
  const long long r01 = ((long long)cell.y[1] * tw + cell.x[0]) * C, r11 = ((long long)cell.y[1] * tw + cell.x[1]) * C;

  float gmax = 0.f;
  bool gbad = false;
  if (g_uv && inside) {
    float du = 0.f, dv = 0.f;
    if (cell.ok) {
      if constexpr (V4) {
        for (int c = 0; c < C; c += 4) {
          const float4 gg = *reinterpret_cast<const float4*>(g + c);
          const float4 a = *reinterpret_cast<const float4*>(tex + r00 + c);
          const float4 b = *reinterpret_cast<const float4*>(tex + r10 + c);
          const float4 d = *reinterpret_cast<const float4*>(tex + r01 + c);
          const float4 f = *reinterpret_cast<const float4*>(tex + r11 + c);
          const float gs[4] = {gg.x, gg.y, gg.z, gg.w};
          const float t00[4] = {a.x, a.y, a.z, a.w}, t10[4] = {b.x, b.y, b.z, b.w};
          const float t01[4] = {d.x, d.y, d.z, d.w}, t11[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            du += gs[k] * ((1.0f - cell.fy) * (t10[k] - t00[k]) + cell.fy * (t11[k] - t01[k]));
            dv += gs[k] * ((1.0f - cell.fx) * (t01[k] - t00[k]) + cell.fx * (t11[k] - t10[k]));
          }
        }
      } else {
        for (int c = 0; c < C; ++c) {
          const float t00 = tex[r00 + c], t10 = tex[r10 + c], t01 = tex[r01 + c], t11 = tex[r11 + c];
          du += g[c] * ((1.0f - cell.fy) * (t10 - t00) + cell.fy * (t11 - t01));
          dv += g[c] * ((1.0f - cell.fx) * (t01 - t00) + cell.fx * (t11 - t10));
        }
      }
    }
    g_uv[2 * p] = du * (float)tw;
    g_uv[2 * p + 1] = dv * (float)th;
  }
  if (!g_tex) return;  // uniform: every thread leaves before the barriers
  if (cell.ok)
    for (int c = 0; c < C; ++c) {
      const float a = fabsf(g[c]);
      gbad |= !(a <= 3.40282347e38f);  // inf or NaN
      gmax = fmaxf(gmax, a);
    }

  // per-wave reductions (every lane takes part), then one atomic per wave
  const int big = 0x7fffffff;
  int r0 = cell.ok ? cell.x[0] : big, r1 = cell.ok ? cell.y[0] : big;
  int r2 = cell.ok ? -cell.x[1] : big, r3 = cell.ok ? -cell.y[1] : big;
  int r4 = __float_as_int(gmax), r5 = gbad ? 1 : 0;  // gmax >= 0: its bits order like its value
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    r0 = min(r0, __shfl_xor(r0, o, 64));
    r1 = min(r1, __shfl_xor(r1, o, 64));
    r2 = min(r2, __shfl_xor(r2, o, 64));
    r3 = min(r3, __shfl_xor(r3, o, 64));
    r4 = max(r4, __shfl_xor(r4, o, 64));
    r5 = r5 | __shfl_xor(r5, o, 64);
  }
  __syncthreads();  // s_box initialised
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&s_box[0], r0);
    atomicMin(&s_box[1], r1);
    atomicMin(&s_box[2], r2);
    atomicMin(&s_box[3], r3);
    atomicMax(&s_box[4], r4);
    if (r5) atomicOr(&s_box[5], 1);
  }
  __syncthreads();
  const int bx0 = s_box[0], by0 = s_box[1];
  const bool any = bx0 != 0x7fffffff;
  const long long bw = any ? (long long)(-s_box[2]) - bx0 + 1 : 0, bh = any ? (long long)(-s_box[3]) - by0 + 1 : 0;
  const long long nwin = bw * bh * C;
  const float M = __int_as_float(s_box[4]);
  if (!any || M == 0.f) return;  // nothing to add (uniform)
  if (nwin > kTexWin || s_box[5]) {
    // Straight to memory (uniform: the whole workgroup is here).  Each wave
    // stages its pixels' four (texel row, weight) pairs in the window's LDS,
    // then adds them channel-fastest: lanes l and l + 1 take channels c and
    // c + 1 of one pair, so an instruction falls on the few cache lines of
    // 64 / C texel rows (one L2 atomic request per line) instead of on one
    // line per lane.
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    long long* s_row = reinterpret_cast<long long*>(s_acc) + wv * 320;  // 256 texel rows (-1: none), 64 g rows
    float* s_w = reinterpret_cast<float*>(s_acc + 4 * 320) + wv * 256;  // 256 weights
    const long long rr[4] = {r00, r10, r01, r11};
    const float ww[4] = {w00, w10, w01, w11};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      s_row[4 * ln + k] = cell.ok ? rr[k] : -1;
      s_w[4 * ln + k] = ww[k];
    }
    s_row[256 + ln] = cell.ok ? p * C : 0;
    __syncthreads();
    const int dq = 64 / C, dr = 64 % C;  // (pair, channel) steps per 64 values
    int pr = ln / C, c = ln % C;
    for (int i = ln; i < 256 * C; i += 64) {
      const long long r = s_row[pr];
      if (r >= 0) {
        const float gc = g_out[s_row[256 + (pr >> 2)] + c];
        if (gc != 0.f) atomicAdd(g_tex + r + c, s_w[pr] * gc);
      }
      pr += dq;
      c += dr;
      if (c >= C) {
        c -= C;
        ++pr;
      }
    }
    return;
  }
  int e;
  frexpf(M, &e);  // M < 2^e
  const int sh = 51 - e;
  const double scale = ldexp(1.0, sh);
  for (int i = threadIdx.x; i < (int)nwin; i += blockDim.x) s_acc[i] = 0ull;
  __syncthreads();
  // channel-major window (value c of texel i at c * ncell + i): the lanes of
  // a wave touch neighbouring texels, which then sit 8 bytes apart in LDS
  // rather than C * 8 bytes (with C = 8, four banks for the whole wave)
  const int ncell = (int)(bw * bh);
  if (cell.ok) {
    const int l00 = (int)((cell.y[0] - by0) * bw + (cell.x[0] - bx0));
    const int l10 = (int)((cell.y[0] - by0) * bw + (cell.x[1] - bx0));
    const int l01 = (int)((cell.y[1] - by0) * bw + (cell.x[0] - bx0));
    const int l11 = (int)((cell.y[1] - by0) * bw + (cell.x[1] - bx0));
    // |w g 2^sh| < 2^51: exact in binary64, rounded to the nearest integer
    auto add = [&](int c, float gc) {
      unsigned long long* a = s_acc + c * ncell;
      atomicAdd(a + l00, fixed_round(w00 * gc, scale));
      atomicAdd(a + l10, fixed_round(w10 * gc, scale));
      atomicAdd(a + l01, fixed_round(w01 * gc, scale));
      atomicAdd(a + l11, fixed_round(w11 * gc, scale));
    };
    if constexpr (V4) {
      // the row four channels a load, every load issued before the adds
      for (int c0 = 0; c0 < C; c0 += 8) {
        const float4 ga = *reinterpret_cast<const float4*>(g + c0);
        const float4 gb = c0 + 4 < C ? *reinterpret_cast<const float4*>(g + c0 + 4) : make_float4(0.f, 0.f, 0.f, 0.f);
        add(c0, ga.x);
        add(c0 + 1, ga.y);
        add(c0 + 2, ga.z);
        add(c0 + 3, ga.w);
        if (c0 + 4 < C) {
          add(c0 + 4, gb.x);
          add(c0 + 5, gb.y);
          add(c0 + 6, gb.z);
          add(c0 + 7, gb.w);
        }
      }
    } else {
      for (int c = 0; c < C; ++c) add(c, g[c]);
    }
  }
  __syncthreads();
  // the flush walks texel-major, so a wave's global atomics stay contiguous
  for (int i = threadIdx.x; i < (int)nwin; i += blockDim.x) {
    const int c = i % C, cell_i = i / C;
    const long long q = (long long)s_acc[c * ncell + cell_i];
    if (q == 0) continue;
    const long long ty = by0 + cell_i / bw, tx = bx0 + cell_i % bw;
    atomicAdd(g_tex + (ty * tw + tx) * C + c, (float)ldexp((double)q, -sh));
  }
}

int launch_texture(const mer_plan* P, const mer_view* views, const int32_t* tri_id, const float* uv, int ld_uv,
                   const float* tex, int th, int tw, int C, float* out, hipStream_t st) {
  const long long n = P->total_px - P->px_begin;
  const bool v4 = C % 4 == 0 && ((uintptr_t)tex % 16) == 0 && ((uintptr_t)out % 16) == 0;
  if (n > 0) {
    if (v4)
      hipLaunchKernelGGL(k_texture<true>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, views, P->n_views,
                         tri_id, uv, ld_uv, tex, th, tw, C, out, P->px_begin, P->total_px);
    else
      hipLaunchKernelGGL(k_texture<false>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, views, P->n_views,
                         tri_id, uv, ld_uv, tex, th, tw, C, out, P->px_begin, P->total_px);
  }
  return hipGetLastError() == hipSuccess ? MER_OK : MER_ELAUNCH;
}

int launch_texture_bwd(const mer_plan* P, const mer_view* views, const int32_t* tri_id, const float* uv, int ld_uv,
                       const float* tex, int th, int tw, int C, const float* g_out, float* g_tex, float* g_uv,
                       void* ws, hipStream_t st) {
  long long* tab = (long long*)((char*)ws + P->off_bviewtab);
  hipLaunchKernelGGL(k_prep, dim3(1), dim3(1024), 0, st, views, P->n_views, 4, 4, tab, tab + (P->n_views + 1),
                     (long long*)nullptr);
  const bool v4 = C % 4 == 0 && ((uintptr_t)tex % 16) == 0 && ((uintptr_t)g_out % 16) == 0;
  if (P->total_btiles > 0) {
    if (v4)
      hipLaunchKernelGGL(k_texture_bwd<true>, dim3((unsigned)P->total_btiles), dim3(256), 0, st, views, P->n_views,
                         tab + (P->n_views + 1), tri_id, uv, ld_uv, tex, th, tw, C, g_out, g_tex, g_uv);
    else
      hipLaunchKernelGGL(k_texture_bwd<false>, dim3((unsigned)P->total_btiles), dim3(256), 0, st, views, P->n_views,
                         tab + (P->n_views + 1), tri_id, uv, ld_uv, tex, th, tw, C, g_out, g_tex, g_uv);
  }
  return hipGetLastError() == hipSuccess ? MER_OK : MER_ELAUNCH;
}

}  // namespace mer
