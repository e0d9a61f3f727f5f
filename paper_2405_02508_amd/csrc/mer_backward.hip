// mer_backward.hip -- attribute interpolation (forward) and the fused
// backward pass: the micro-edge term of EdgeGrad (Sec. 4.2-4.4) plus the
// interpolation adjoint with the smooth term Omega (Sec. 3), one sweep over
// the pixels.
#include "mer_internal.h"

namespace mer {

// ---------------------------------------------------------- interpolate
// One thread per pixel computes its C values into LDS; the block then writes
// its 256 x C floats as one contiguous span (coalesced), unless the block
// straddles a gap between views, where each pixel writes its own values.
__global__ void __launch_bounds__(256) k_interp(const mer_view* __restrict__ views, int n_views,
                                                const float* __restrict__ attr, int C_a,
                                                const float* __restrict__ v, const int32_t* __restrict__ tri,
                                                const int32_t* __restrict__ tri_id, const float* __restrict__ bary,
                                                int append_z, float* __restrict__ out, long long px_begin,
                                                long long total_px) {
  extern __shared__ float s_out[];
  __shared__ int s_gap;
  const int C = C_a + append_z;
  const long long p0 = px_begin + (long long)blockIdx.x * blockDim.x;
  const long long p = p0 + threadIdx.x;
  if (threadIdx.x == 0) s_gap = 0;
  __syncthreads();
  bool valid = false;
  float b0 = 0.f, b1 = 0.f, b2 = 0.f;
  int idx[3] = {0, 0, 0};
  mer_view vw;
  const int wvi = wave_view(views, n_views, p - (threadIdx.x & 63));
  if (p < total_px) {
    int vi = wvi;
    if (vi + 1 < n_views && p >= views[vi + 1].px_off) vi = find_view_px(views, n_views, p);
    vw = views[vi];
    const long long local = p - vw.px_off;
    valid = local >= 0 && local < (long long)vw.H * vw.W;
    if (valid) {
      int t = tri_id[p];
      if (t >= 0 && t < vw.n_t) {
        const int32_t* row = tri_row(tri, vw, (int)t);
        idx[0] = row[0];
        idx[1] = row[1];
        idx[2] = row[2];
        bool ok = idx[0] >= 0 && idx[0] < vw.n_v && idx[1] >= 0 && idx[1] < vw.n_v && idx[2] >= 0 &&
                  idx[2] < vw.n_v;
        if (ok) {
          if (bary) {
            const float2 bb = *reinterpret_cast<const float2*>(bary + 2 * p);
            b0 = bb.x;
            b1 = bb.y;
            b2 = (1.0f - b0) - b1;
          } else {
            // exactly as the rasterizer's resolve computes them
            const Snap sn = snap_triangle(v, vw, row);
            ok = sn.ok;
            if (ok) {
              float a, b, n;
              resolve_products(sn, (int)(local % vw.W), (int)(local / vw.W), a, b, n);
              const float r = __builtin_amdgcn_rcpf(n);
              b0 = a * r;
              b1 = b * r;
              b2 = (1.0f - b0) - b1;
            }
          }
        }
        if (!ok) b0 = b1 = b2 = 0.f;
        if (!ok) idx[0] = -1;
      } else {
        idx[0] = -1;
      }
    } else {
      atomicOr(&s_gap, 1);
    }
  }
  float* so = s_out + threadIdx.x * C;
  if (valid && idx[0] >= 0) {
    const float* a0 = attr + (vw.a_off + idx[0]) * C_a;
    const float* a1 = attr + (vw.a_off + idx[1]) * C_a;
    const float* a2 = attr + (vw.a_off + idx[2]) * C_a;
    for (int c = 0; c < C_a; ++c) so[c] = (b0 * a0[c] + b1 * a1[c]) + b2 * a2[c];
    if (append_z) {
      const float z0 = v[(vw.v_off + idx[0]) * 3 + 2], z1 = v[(vw.v_off + idx[1]) * 3 + 2],
                  z2 = v[(vw.v_off + idx[2]) * 3 + 2];
      so[C_a] = (b0 * z0 + b1 * z1) + b2 * z2;
    }
  } else {
    for (int c = 0; c < C; ++c) so[c] = 0.f;
  }
  __syncthreads();
  if (s_gap) {
    if (valid)
      for (int c = 0; c < C; ++c) out[p * C + c] = so[c];
    return;
  }
  const long long n_here = min((long long)blockDim.x, total_px - p0);
  float* dst = out + p0 * C;
  for (long long i = threadIdx.x; i < n_here * C; i += blockDim.x) dst[i] = s_out[i];
}

// ------------------------------------------------------------- back faces
// One thread per pixel: 1 where the visible triangle's snapped signed area
// is positive (its back side faces the viewer), else 0.
__global__ void __launch_bounds__(256) k_backface(const mer_view* __restrict__ views, int n_views,
                                                  const float* __restrict__ v, const int32_t* __restrict__ tri,
                                                  const int32_t* __restrict__ tri_id, float* __restrict__ out,
                                                  long long px_begin, long long total_px) {
  const long long p = px_begin + (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int wvi = wave_view(views, n_views, p - (threadIdx.x & 63));
  if (p >= total_px) return;
  int vi = wvi;
  if (vi + 1 < n_views && p >= views[vi + 1].px_off) vi = find_view_px(views, n_views, p);
  const mer_view vw = views[vi];
  const long long local = p - vw.px_off;
  if (local < 0 || local >= (long long)vw.H * vw.W) return;  // gap between views
  const int t = tri_id[p];
  float r = 0.f;
  if (t >= 0 && t < vw.n_t) {
    const Snap sn = snap_triangle<false>(v, vw, tri_row(tri, vw, t));
    r = sn.ok && sn.D > 0 ? 1.f : 0.f;
  }
  out[p] = r;
}

int launch_backface(const mer_plan* P, const mer_view* views, const float* v, const int32_t* tri,
                    const int32_t* tri_id, float* out, hipStream_t st) {
  const long long n = P->total_px - P->px_begin;
  hipLaunchKernelGGL(k_backface, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, views, P->n_views, v, tri,
                     tri_id, out, P->px_begin, P->total_px);
  return hipGetLastError() == hipSuccess ? MER_OK : MER_ELAUNCH;
}

// ------------------------------------------------------------- backward
template <bool EXACT_Q>
__device__ __forceinline__ Snap snap_id(const float* v, const int32_t* tri, const mer_view& vw, int t) {
  return snap_triangle<EXACT_Q>(v, vw, tri_row(tri, vw, (int)t));
}

// Segmented inclusive sum over lanes [hir, lir] of one 16-lane row of a
// wave, with DPP row shifts (row_shr:1, 2, 4, 8).
template <int CTRL>
__device__ __forceinline__ float dpp_row_shr(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xf, 0xf, true));
}
// m[i] is 1 where the lane 2^i places to the left is in the same run, else 0
// (so the fused multiply-add below adds either the neighbour or exactly 0).
struct RunMask {
  float m1, m2, m4, m8;
};
__device__ __forceinline__ RunMask run_mask(int lir, int hir) {
  return {lir - 1 >= hir ? 1.f : 0.f, lir - 2 >= hir ? 1.f : 0.f, lir - 4 >= hir ? 1.f : 0.f,
          lir - 8 >= hir ? 1.f : 0.f};
}
__device__ __forceinline__ float seg_sum(float x, const RunMask& m) {
  x = __builtin_fmaf(dpp_row_shr<0x111>(x), m.m1, x);
  x = __builtin_fmaf(dpp_row_shr<0x112>(x), m.m2, x);
  x = __builtin_fmaf(dpp_row_shr<0x114>(x), m.m4, x);
  x = __builtin_fmaf(dpp_row_shr<0x118>(x), m.m8, x);
  return x;
}

// Backward sweep over 16x16 pixel tiles of one view per workgroup (256
// threads; wave w holds rows 4w..4w+3, 16 lanes per row).
//  1. each lane computes its pixel's fragment gradient from the micro-edges
//     it belongs to (Sec. 4.2-4.4) and its interpolation adjoint (Omega);
//  2. lanes sum runs of equal triangle along each 16-pixel row (a triangle
//     meets a row in one run: it is convex) with a segmented wave reduction;
//  3. the last lane of each run adds the run's sums into an LDS table keyed
//     by vertex (a vertex is shared by the runs of several triangles);
//  4. the workgroup flushes the table with one global float atomic per
//     (vertex, component).  Vertices that do not fit the table, and
//     attribute channels beyond kCTab, go straight to global atomics.
constexpr int kSlots = 256;  // vertex slots per workgroup
constexpr int kCTab = 8;     // attribute channels reduced in LDS
constexpr int kNV = 3 + kCTab;

// Find or claim the slot of vertex `key`; a new slot has its values zeroed
// and is appended to the occupied list.  -1 when the probe limit is hit.
__device__ __forceinline__ int slot_of(int* s_key, float* s_val, int* s_list, int* s_nocc, int key) {
  unsigned h = ((unsigned)key * 2654435761u) >> 24;  // 8 bits
#pragma unroll 1
  for (int probe = 0; probe < 32; ++probe) {
    const int s = (int)((h + probe) & (kSlots - 1));
    const int old = atomicCAS(&s_key[s], -1, key);
    if (old == -1) {
#pragma unroll
      for (int j = 0; j < kNV; ++j) s_val[s * kNV + j] = 0.f;
      s_list[atomicAdd(s_nocc, 1)] = s;
      return s;
    }
    if (old == key) return s;
  }
  return -1;
}

// L2: dL/d(img) = 2 w (img - target) is formed here instead of read from g.
// LOSS: w * sum (img - target)^2 over each wave's 64 pixels goes to
// loss_part[4 tile + wave] (computed last, when few registers are live).
template <bool L2, bool LOSS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) k_backward(const mer_view* __restrict__ views, int n_views,
                                                  const long long* __restrict__ btile_base,
                                                  const float* __restrict__ v, const int32_t* __restrict__ tri,
                                                  const int32_t* __restrict__ tri_id, const float* __restrict__ attr,
                                                  int C_a, int append_z, const float* __restrict__ img,
                                                  const float* __restrict__ g, int C_e, int ld_g, int flags,
                                                  float* __restrict__ g_attr, float* __restrict__ g_v,
                                                  const float* __restrict__ target, float w_l2,
                                                  float* __restrict__ loss_part) {
  __shared__ int s_key[kSlots];
  __shared__ float s_val[kSlots * kNV];
  __shared__ int s_list[kSlots];
  __shared__ int s_nocc;
  for (int i = threadIdx.x; i < kSlots; i += blockDim.x) s_key[i] = -1;
  if (threadIdx.x == 0) s_nocc = 0;

  const long long tile = xcd_tile(blockIdx.x, gridDim.x);
  const int vi = __builtin_amdgcn_readfirstlane(find_bucket(btile_base, n_views, tile));
  const mer_view vw = views[vi];
  const long long local_tile = tile - btile_base[vi];
  const int tiles_x = (vw.W + 15) >> 4;
  const int lane = threadIdx.x & 63;
  const int px = (int)(local_tile % tiles_x) * 16 + (lane & 15);
  const int py = (int)(local_tile / tiles_x) * 16 + (threadIdx.x >> 4);
  const bool inside = px < vw.W && py < vw.H;
  const long long p = vw.px_off + (long long)py * vw.W + px;
  int t = -1;
  if (inside) {
    t = tri_id[p];
    if (t >= vw.n_t || t < 0) t = -1;
  }
  Snap S;
  S.ok = false;
  if (t >= 0) S = snap_id<false>(v, tri, vw, t);
  if (t >= 0 && !S.ok) t = -1;

  // ---- micro-edge term: fragment gradient (rx, ry, rq) of this pixel
  float rx = 0.f, ry = 0.f, rq = 0.f;
  // a background pixel is never the top side of a pair, so it receives nothing.
  // First the cheap part: which of the four neighbours differ (bit dir of
  // `pend`); then the wave iterates only as often as its busiest lane has
  // differing neighbours, each lane taking its next pending pair.
  unsigned pend = 0;
  int tn4[4] = {-1, -1, -1, -1};
  if (t >= 0 && !(flags & MER_SKIP_EDGE)) {
#pragma unroll
    for (int dir = 0; dir < 4; ++dir) {
      const int nx = px + (dir == 0 ? -1 : dir == 1 ? 1 : 0);
      const int ny = py + (dir == 2 ? -1 : dir == 3 ? 1 : 0);
      if (nx < 0 || ny < 0 || nx >= vw.W || ny >= vw.H) continue;
      int tn = tri_id[vw.px_off + (long long)ny * vw.W + nx];
      if (tn >= vw.n_t || tn < 0) tn = -1;
      tn4[dir] = tn;
      if (tn != t) pend |= 1u << dir;
    }
  }
#pragma unroll 1
  while (__ballot(pend != 0)) {
    if (pend == 0) continue;
    const int dir = __builtin_ctz(pend);
    pend &= pend - 1;
    const int tn = dir == 0 ? tn4[0] : dir == 1 ? tn4[1] : dir == 2 ? tn4[2] : tn4[3];
    const int nx = px + (dir == 0 ? -1 : dir == 1 ? 1 : 0);
    const int ny = py + (dir == 2 ? -1 : dir == 3 ? 1 : 0);
    const long long pn = vw.px_off + (long long)ny * vw.W + nx;
    const bool selfA = dir == 1 || dir == 3;  // self has the smaller coordinate
    const int axis = dir < 2 ? 0 : 1;
    const long long pA = selfA ? p : pn, pB = selfA ? pn : p;
    float acc = 0.f;
    const float* ia = img + pA * C_e;
    const float* ib = img + pB * C_e;
    if constexpr (L2) {
      const float* ta = target + pA * C_e;
      const float* tb = target + pB * C_e;
      for (int c = 0; c < C_e; ++c) {
        const float gs = (2.0f * w_l2) * (ia[c] - ta[c]) + (2.0f * w_l2) * (ib[c] - tb[c]);
        acc += gs * (ia[c] - ib[c]);
      }
    } else {
      const float* ga = g + pA * ld_g;
      const float* gb = g + pB * ld_g;
      for (int c = 0; c < C_e; ++c) acc += (ga[c] + gb[c]) * (ia[c] - ib[c]);
    }
    const float dLdp = 0.5f * acc;
    if (tn < 0) {
      // overhang over background: this (covered) side is on top
      if (axis == 0) rx += dLdp;
      else ry += dLdp;
      continue;
    }
    const Snap Sn = snap_id<false>(v, tri, vw, tn);
    Snap SA, SB;  // by value: a conditional reference would force the structs to scratch
    if (selfA) {
      SA = S;
      SB = Sn;
    } else {
      SA = Sn;
      SB = S;
    }
    const int ax_ = selfA ? px : nx, ay_ = selfA ? py : ny;
    const int bx_ = selfA ? nx : px, by_ = selfA ? ny : py;
    const bool cA = contains(SB, ax_, ay_);  // B's triangle holds A's centre
    const bool cB = contains(SA, bx_, by_);  // A's triangle holds B's centre
    if (!cA && !cB) continue;                // adjacent: nothing
    if (cA != cB) {
      if (cA == selfA) {                     // the contained side is on top
        if (axis == 0) rx += dLdp;
        else ry += dLdp;
      }
      continue;
    }
    if (flags & MER_NO_INTERSECT) continue;
    const float sA = plane_slope(SA, axis), sB = plane_slope(SB, axis);
    const float dlt = sB - sA;
    if (!(dlt > 0.f) || !isfinite(dlt)) continue;
    const float u = dLdp / dlt;
    const float ra = selfA ? -sA * u : sB * u;
    if (axis == 0) rx += ra;
    else ry += ra;
    rq += selfA ? u : -u;
  }

  // ---- runs of equal triangle along each 16-pixel row of the wave
  const int t_prev = __shfl_up(t, 1, 64);
  const bool head_flag = (lane & 15) == 0 || t != t_prev;
  const unsigned long long F = __ballot(head_flag);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int head = 63 - __clzll((long long)(F & upto));
  const bool tail = lane == 63 || ((F >> (lane + 1)) & 1ull);
  const bool emit = tail && t >= 0;
  const RunMask rm = run_mask(lane & 15, head & 15);  // runs never cross a 16-lane row

  PixBary pb;
  pb.beta[0] = pb.beta[1] = pb.beta[2] = 0.f;
  pb.b[0] = pb.b[1] = pb.b[2] = 0.f;
  pb.Wq = 1.f;
  if (t >= 0) pb = pixel_bary(S, px, py);
  float gx[3], gy[3], gz[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float qk = t >= 0 ? S.q[k] : 0.f;
    gx[k] = pb.beta[k] * rx;
    gy[k] = pb.beta[k] * ry;
    gz[k] = pb.beta[k] * rq * (-(qk * qk));
  }
  __syncthreads();  // keys cleared
  int slot[3] = {-1, -1, -1};
  if (emit) {
#pragma unroll
    for (int k = 0; k < 3; ++k) slot[k] = slot_of(s_key, s_val, s_list, &s_nocc, S.idx[k]);
  }
  __syncthreads();  // every slot this tile uses is claimed and zeroed

  // ---- interpolation adjoint and Omega
  if (!(flags & MER_SKIP_INTERP)) {
    // this pixel's dL/d(image) row
    const long long pg = t >= 0 ? p : 0;
    const float* gp = L2 ? img + pg * C_e : g + pg * ld_g;
    const float* tp = L2 ? target + pg * C_e : nullptr;
    auto gown = [&](int c) -> float {
      if constexpr (L2) return (2.0f * w_l2) * (gp[c] - tp[c]);
      else return gp[c];
    };
    long long arow[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) arow[k] = t >= 0 ? (vw.a_off + S.idx[k]) * C_a : 0;
    float G[3] = {0.f, 0.f, 0.f};
    for (int c = 0; c < C_a; ++c) {  // uniform trip count: every lane joins the reductions
      const float gc = t >= 0 ? gown(c) : 0.f;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (t >= 0) G[k] += gc * attr[arow[k] + c];
        if (g_attr) {
          const float s = seg_sum(pb.b[k] * gc, rm);
          if (emit && s != 0.f) {
            if (c < kCTab && slot[k] >= 0) atomicAdd(&s_val[slot[k] * kNV + 3 + c], s);
            else atomicAdd(g_attr + arow[k] + c, s);
          }
        }
      }
    }
    if (t >= 0) {
      if (append_z) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          G[k] += gown(C_a) * S.z[k];
          gz[k] += pb.b[k] * gown(C_a);
        }
      }
      const float Gb = (pb.b[0] * G[0] + pb.b[1] * G[1]) + pb.b[2] * G[2];
      const float iW = __builtin_amdgcn_rcpf(pb.Wq);
      float dbeta[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float dw = (G[k] - Gb) * iW;
        dbeta[k] = dw * S.q[k];
        gz[k] += (dw * pb.beta[k]) * (-(S.q[k] * S.q[k]));
      }
      // d beta_i / d v_j = -beta_j * grad_P beta_i;  grad_P beta_i = 256 (-(Yb-Ya), Xb-Xa) / D
      const float invD = 256.0f * __builtin_amdgcn_rcpf((float)S.D);
      float sx = 0.f, sy = 0.f;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int a = (i + 1) % 3, b = (i + 2) % 3;
        sx += dbeta[i] * ((float)(-(S.Y[b] - S.Y[a])) * invD);
        sy += dbeta[i] * ((float)(S.X[b] - S.X[a]) * invD);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        gx[k] += -pb.beta[k] * sx;
        gy[k] += -pb.beta[k] * sy;
      }
    }
  }
  if (g_v) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float sums[3] = {seg_sum(gx[k], rm), seg_sum(gy[k], rm), seg_sum(gz[k], rm)};
      if (emit) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          if (sums[j] == 0.f) continue;
          if (slot[k] >= 0) atomicAdd(&s_val[slot[k] * kNV + j], sums[j]);
          else atomicAdd(g_v + (vw.v_off + S.idx[k]) * 3 + j, sums[j]);
        }
      }
    }
  }
  __syncthreads();

  // ---- flush: one global atomic per (vertex, component) of this tile
  const int nv = 3 + min(C_a, kCTab);
  const int nocc = s_nocc;
  for (int i = threadIdx.x >> 4; i < nocc; i += (int)(blockDim.x >> 4)) {
    const int s = s_list[i];
    const int key = s_key[s];
    for (int j = threadIdx.x & 15; j < nv; j += 16) {
      const float x = s_val[s * kNV + j];
      if (x == 0.f) continue;
      if (j < 3) {
        if (g_v) atomicAdd(g_v + (vw.v_off + key) * 3 + j, x);
      } else if (g_attr) {
        atomicAdd(g_attr + (vw.a_off + key) * C_a + (j - 3), x);
      }
    }
  }
  if constexpr (LOSS) {
    {
      float e2 = 0.f;
      if (inside)
        for (int c = 0; c < C_e; ++c) {
          const float d = img[p * C_e + c] - target[p * C_e + c];
          e2 += d * d;
        }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) e2 += __shfl_xor(e2, o, 64);
      if (lane == 0) loss_part[4 * tile + (threadIdx.x >> 6)] = w_l2 * e2;
    }
  }
}

int launch_interpolate(const mer_plan* P, const mer_view* views, const float* attr, int C_a, const float* v,
                       const int32_t* tri, const int32_t* tri_id, const float* bary, int append_z, float* out,
                       hipStream_t st) {
  const long long n = P->total_px - P->px_begin;
  const int C = C_a + append_z;
  const int bs = C <= 32 ? 256 : 128;  // keeps the LDS staging buffer at or below 32 KB
  const size_t lds = (size_t)bs * C * sizeof(float);
  hipLaunchKernelGGL(k_interp, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), lds, st, views, P->n_views, attr, C_a, v,
                     tri, tri_id, bary, append_z, out, P->px_begin, P->total_px);
  return hipGetLastError() == hipSuccess ? MER_OK : MER_ELAUNCH;
}

// Sum of the per-tile loss partials, one workgroup, then one atomic.
__global__ void __launch_bounds__(1024) k_loss_sum(const float* __restrict__ part, long long n,
                                                   float* __restrict__ loss) {
  __shared__ float s_w[16];
  float a = 0.f;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) a += part[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += s_w[i];
    atomicAdd(loss, t);
  }
}

int launch_backward(const mer_plan* P, const mer_view* views, const float* v, const int32_t* tri,
                    const int32_t* tri_id, const float* attr, int C_a, int append_z, const float* img,
                    const float* g, const float* target, float w_l2, float* loss, int C_e, int ld_g, int flags,
                    float* g_attr, float* g_v, void* ws, hipStream_t st) {
  long long* tab = (long long*)((char*)ws + P->off_bviewtab);
  float* bloss = loss ? (float*)((char*)ws + P->off_bloss) : nullptr;
  // 16x16 tile prefix per view; the rasterizer's status words are left alone
  hipLaunchKernelGGL(k_prep, dim3(1), dim3(1024), 0, st, views, P->n_views, 4, 4, tab, tab + (P->n_views + 1),
                     (long long*)nullptr);
#define MER_BACKWARD(L2, LOSS)                                                                                 \
  hipLaunchKernelGGL((k_backward<L2, LOSS>), dim3((unsigned)P->total_btiles), dim3(256), 0, st, views, P->n_views, \
                     tab + (P->n_views + 1), v, tri, tri_id, attr, C_a, append_z, img, g, C_e, ld_g, flags, g_attr,  \
                     g_v, target, w_l2, bloss)
  if (!target) MER_BACKWARD(false, false);
  else if (!bloss) MER_BACKWARD(true, false);
  else MER_BACKWARD(true, true);
#undef MER_BACKWARD
  if (bloss) hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(1024), 0, st, bloss, 4 * P->total_btiles, loss);
  return hipGetLastError() == hipSuccess ? MER_OK : MER_ELAUNCH;
}

}  // namespace mer
