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
              int lx, ly;
              grid_xy(local, vw.W, lx, ly);
              resolve_products(sn, lx, ly, a, b, n);
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
    // four channels a load where the rows allow it
    const int va = row_vec(C_a, attr) == 3 ? 3 : row_vec(C_a, attr) == 4 && ((vw.a_off * C_a) & 3) == 0 ? 4 : 0;
    for (int c0 = 0; c0 < C_a; c0 += 4) {
      const int na = min(4, C_a - c0);
      const float4 x0 = row4(a0 + c0, va, na), x1 = row4(a1 + c0, va, na), x2 = row4(a2 + c0, va, na);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j < na) so[c0 + j] = (b0 * f4(x0, j) + b1 * f4(x1, j)) + b2 * f4(x2, j);
    }
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
// wave: doubling steps x += m_S * x[lane - S] (S = 1, 2, 4, 8), each a
// v_fmac_f32 whose first operand is read through a
// DPP row shift (a lane at the start of its 16-lane row reads 0).  m_S is 1
// where the lane S places to the left is in the same run, else 0, so a step
// adds the neighbour's partial sum or exactly 0.  A run of length L is summed
// after ceil(log2 L) steps, so a wave takes only the steps its longest run of
// covered pixels needs (steps, the same in every lane); the code that sums is
// compiled once per step count and a wave branches once to its copy.  Each
// step's s_nop covers the two wait states a DPP read of a register needs
// after a VALU write to it.
struct RunMask {
  float m1, m2, m4, m8;
  int steps;
};
__device__ __forceinline__ RunMask run_mask(int lir, int hir, bool covered) {
  RunMask m = {lir - 1 >= hir ? 1.f : 0.f, lir - 2 >= hir ? 1.f : 0.f, lir - 4 >= hir ? 1.f : 0.f,
               lir - 8 >= hir ? 1.f : 0.f, 0};
  const int pos = lir - hir;
  m.steps = __ballot(covered && pos >= 8) ? 4 : __ballot(covered && pos >= 4) ? 3 : __ballot(covered && pos >= 2) ? 2
            : __ballot(covered && pos >= 1) ? 1 : 0;
  return m;
}
// Nearest integer of x (halves rounded up) in one instruction: floor(x + 0.5),
// exact for |x| < 2^22 (x + 0.5 is then representable).
__device__ __forceinline__ int round_half_up(float x) {
  int q;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(q) : "v"(x));
  return q;
}

template <int STEPS>
__device__ __forceinline__ float seg_sum(float x, const RunMask& m) {
  if constexpr (STEPS >= 1)
    asm("s_nop 1\n\tv_fmac_f32_dpp %0, %0, %1 row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1" : "+v"(x) : "v"(m.m1));
  if constexpr (STEPS >= 2)
    asm("s_nop 1\n\tv_fmac_f32_dpp %0, %0, %1 row_shr:2 row_mask:0xf bank_mask:0xf bound_ctrl:1" : "+v"(x) : "v"(m.m2));
  if constexpr (STEPS >= 3)
    asm("s_nop 1\n\tv_fmac_f32_dpp %0, %0, %1 row_shr:4 row_mask:0xf bank_mask:0xf bound_ctrl:1" : "+v"(x) : "v"(m.m4));
  if constexpr (STEPS >= 4)
    asm("s_nop 1\n\tv_fmac_f32_dpp %0, %0, %1 row_shr:8 row_mask:0xf bank_mask:0xf bound_ctrl:1" : "+v"(x) : "v"(m.m8));
  return x;
}
template <int N>
struct Steps {
  static constexpr int value = N;
};

// Backward sweep over 16x16 pixel tiles of one view per workgroup (256
// threads; wave w holds rows 4w..4w+3, 16 lanes per row).
//  1. each lane snaps its pixel's triangle once and computes its exact edge
//     values, from which it decides which of its four neighbours' centres
//     the triangle holds; it publishes that 4-bit mask and its triangle id
//     in LDS.  The first wave does the same for the tile's ring (the 64
//     pixels just outside it next to its border pixels), each ring pixel's
//     bit being whether its triangle holds its tile neighbour's centre;
//  2. each lane takes the micro-edges it belongs to (Sec. 4.2-4.4): a pair's
//     classification needs "B's triangle holds A's centre" and "A's triangle
//     holds B's centre", one bit of each side's mask, so no neighbour
//     triangle is snapped again (intersections, which need both planes'
//     slopes, snap the neighbour's triangle).  Image and dL/d(image) rows are
//     read with vector loads;
//  3. its interpolation adjoint (Omega);
//  4. lanes sum runs of equal triangle along each 16-pixel row (a triangle
//     meets a row in one run: it is convex) with a segmented wave reduction;
//     the last lane of each run adds the run's sums into an LDS table keyed
//     by vertex (a vertex is shared by the runs of several triangles);
//  5. the workgroup flushes the table with one global float atomic per
//     (vertex, component).  Vertices that do not fit the table, and
//     attribute channels beyond kCTab, go straight to global atomics.
constexpr int kSlots = 256;  // vertex slots per workgroup
constexpr int kCTab = 8;     // attribute channels reduced in LDS (two groups of four)
constexpr int kNV = 3 + kCTab;
constexpr int kQ = 256 + 64;  // tile pixels and ring pixels

// Find or claim the slot of vertex `key`; a new slot is appended to the
// occupied list.  -1 when the probe limit is hit.
__device__ __forceinline__ int slot_of(int* s_key, int* s_list, int* s_nocc, int key) {
  unsigned h = ((unsigned)key * 2654435761u) >> 24;  // 8 bits
#pragma unroll 1
  for (int probe = 0; probe < 32; ++probe) {
    const int s = (int)((h + probe) & (kSlots - 1));
    const int old = atomicCAS(&s_key[s], -1, key);
    if (old == -1) {
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
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) k_backward(const mer_view* __restrict__ views, int n_views,
                                                  const long long* __restrict__ btile_base,
                                                  const float* __restrict__ v, const int32_t* __restrict__ tri,
                                                  const int32_t* __restrict__ tri_id, const float* __restrict__ attr,
                                                  int C_a, int append_z, const float* __restrict__ img,
                                                  const float* __restrict__ g, int C_e, int ld_g, int flags,
                                                  float* __restrict__ g_attr, float* __restrict__ g_v,
                                                  const float* __restrict__ target, float w_l2,
                                                  float* __restrict__ loss_part) {
  __shared__ int s_key[kSlots];
  __shared__ __align__(16) int s_acc[kSlots * kNV];  // fixed-point sums (the table, below)
  __shared__ int s_list[kSlots];
  __shared__ int s_nocc;
  __shared__ __align__(16) unsigned s_mx[kSlots * 3];  // per slot and group: bits of the largest |run sum| added
  // the tile's 256 pixels, then its ring: the 64 pixels just outside it that
  // are neighbours of its border pixels (16 per side: left, right, up, down)
  __shared__ int s_t[kQ];
  __shared__ unsigned char s_cm[kQ];
  // the table starts empty and zero: a run end may raise a slot's maximum as
  // soon as another lane has claimed the slot
  for (int i = threadIdx.x; i < kSlots; i += blockDim.x) s_key[i] = -1;
  for (int i = threadIdx.x; i < kSlots * kNV / 4; i += blockDim.x) reinterpret_cast<int4*>(s_acc)[i] = make_int4(0, 0, 0, 0);
  for (int i = threadIdx.x; i < kSlots * 3 / 4; i += blockDim.x) reinterpret_cast<uint4*>(s_mx)[i] = make_uint4(0u, 0u, 0u, 0u);
  if (threadIdx.x == 0) s_nocc = 0;

  const long long tile = xcd_tile(blockIdx.x, gridDim.x);
  const int vi = __builtin_amdgcn_readfirstlane(find_bucket(btile_base, n_views, tile));
  const mer_view vw = views[vi];
  const long long local_tile = tile - btile_base[vi];
  const int tiles_x = (vw.W + 15) >> 4;
  int x0, y0;
  grid_xy(local_tile, tiles_x, x0, y0);
  x0 *= 16;
  y0 *= 16;
  const int lane = threadIdx.x & 63;
  const int lt = threadIdx.x;  // pixel (lt & 15, lt >> 4) of the tile
  const int lx = lt & 15, ly = lt >> 4;
  const int px = x0 + lx, py = y0 + ly;
  const bool inside = px < vw.W && py < vw.H;
  const long long p = vw.px_off + (long long)py * vw.W + px;
  const bool want_edge = !(flags & MER_SKIP_EDGE);
  const bool want_interp = !(flags & MER_SKIP_INTERP);
  // image, target and dL/d(image) rows: vector widths (uniform)
  const int vimg = row_vec(C_e, img), vtar = L2 ? row_vec(C_e, target) : 0;
  const int vg = L2 ? 0 : (ld_g == C_e ? row_vec(C_e, g) : (((ld_g & 3) == 0 && ((uintptr_t)g & 15) == 0) ? 4 : 0));
  const bool v2img = (C_e & 1) == 0 && ((uintptr_t)img & 7) == 0;
  const bool v2tar = L2 && (C_e & 1) == 0 && ((uintptr_t)target & 7) == 0;
  const bool v2g = !L2 && (ld_g & 1) == 0 && ((uintptr_t)g & 7) == 0;

  // ---- the ring, by the first wave: each lane one ring pixel.  Its id, and
  // whether its triangle holds the centre of its neighbour in the tile (as
  // the bit that neighbour looks up: the direction back from the ring pixel)
  if (want_edge && threadIdx.x < 64) {
    const int r = threadIdx.x, side = r >> 4, i = r & 15;
    const int ix = side == 0 ? x0 : side == 1 ? x0 + 15 : x0 + i;  // the tile pixel next to it
    const int iy = side == 2 ? y0 : side == 3 ? y0 + 15 : y0 + i;
    const int qx = side == 0 ? x0 - 1 : side == 1 ? x0 + 16 : ix;
    const int qy = side == 2 ? y0 - 1 : side == 3 ? y0 + 16 : iy;
    const bool rin = qx >= 0 && qy >= 0 && qx < vw.W && qy < vw.H;
    int rt = -1;
    if (rin) {
      rt = tri_id[vw.px_off + (long long)qy * vw.W + qx];
      if (rt >= vw.n_t || rt < 0) rt = -1;
    }
    unsigned rc = 0;
    if (rt >= 0 && contains(snap_triangle<false>(v, vw, tri_row(tri, vw, rt)), ix, iy)) rc = 1u << (side ^ 1);
    s_t[256 + r] = rt;
    s_cm[256 + r] = (unsigned char)rc;
  }

  int t = -1;
  if (inside) {
    t = tri_id[p];
    if (t >= vw.n_t || t < 0) t = -1;
  }
  // the id as the neighbours see it (a triangle that does not snap is still
  // a triangle to them, one that holds no centre); -1 below if it does not
  const int t_id = t;
  Snap S;
  S.ok = false;
  if (t >= 0) S = snap_triangle<false>(v, vw, tri_row(tri, vw, t));
  if (t >= 0 && !S.ok) t = -1;
  unsigned cm = 0;  // bit d: this triangle holds neighbour d's centre
  if (want_edge && t >= 0) cm = cover_mask(S, px, py);
  s_t[lt] = t_id;
  s_cm[lt] = (unsigned char)cm;
  __syncthreads();

  // ---- micro-edge term: fragment gradient (rx, ry, rq) of this pixel.
  // A background pixel is never the top side of a pair, so it receives
  // nothing.  Neighbour d: 0 left, 1 right, 2 up, 3 down; q(d) its place in
  // the tile or the ring.
  auto nq = [&](int dir) -> int {
    if (dir == 0) return lx > 0 ? lt - 1 : 256 + ly;
    if (dir == 1) return lx < 15 ? lt + 1 : 256 + 16 + ly;
    if (dir == 2) return ly > 0 ? lt - 16 : 256 + 32 + lx;
    return ly < 15 ? lt + 16 : 256 + 48 + lx;
  };
  // The pair is classified from the two masks before any image row is read:
  // with mine = this triangle holds the neighbour's centre and theirs = the
  // neighbour's triangle holds this centre, this side is on top when the
  // neighbour is background (overhang), or theirs and not mine (the side
  // whose centre the other triangle holds); both sides are when both hold
  // (intersection).  Otherwise this side receives nothing from the pair.
  float rx = 0.f, ry = 0.f, rq = 0.f;
  unsigned pend = 0;  // bit d: this side receives a term from the pair with neighbour d
  if (want_edge && t >= 0) {
    const bool no_isect = (flags & MER_NO_INTERSECT) != 0;
    const bool in_view[4] = {px > 0, px + 1 < vw.W, py > 0, py + 1 < vw.H};
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int q = nq(d);  // always a slot of the tile or the ring
      const int tn = s_t[q];
      const bool mine = (cm >> d) & 1u;
      const bool theirs = (s_cm[q] >> (d ^ 1)) & 1u;
      const bool take = in_view[d] & (tn != t) & ((tn < 0) | (theirs & !(mine & no_isect)));
      pend |= take ? 1u << d : 0u;
    }
  }
  // the wave takes as many rounds as its busiest lane has such pairs
#pragma unroll 1
  while (__ballot(pend != 0)) {
    if (pend == 0) continue;
    const int dir = __builtin_ctz(pend);
    pend &= pend - 1;
    const int q = nq(dir);
    const int tn = s_t[q];
    const bool selfA = dir == 1 || dir == 3;  // self has the smaller coordinate
    const int axis = dir < 2 ? 0 : 1;
    const int nx = px + (dir == 0 ? -1 : dir == 1 ? 1 : 0), ny = py + (dir == 2 ? -1 : dir == 3 ? 1 : 0);
    const long long pn = vw.px_off + (long long)ny * vw.W + nx;
    const long long pA = selfA ? p : pn, pB = selfA ? pn : p;
    // dL/dp = 1/2 sum_c (g_A + g_B)(I_A - I_B), A before B, four channels a load
    float acc = 0.f;
#pragma unroll 1
    for (int c0 = 0; c0 < C_e; c0 += 4) {
      const int n = min(4, C_e - c0);
      const float4 ia = row4(img + pA * C_e + c0, vimg, n), ib = row4(img + pB * C_e + c0, vimg, n);
      float4 ga, gb;
      if constexpr (L2) {
        const float4 ta = row4(target + pA * C_e + c0, vtar, n), tb = row4(target + pB * C_e + c0, vtar, n);
        ga = make_float4((2.0f * w_l2) * (ia.x - ta.x), (2.0f * w_l2) * (ia.y - ta.y), (2.0f * w_l2) * (ia.z - ta.z),
                         (2.0f * w_l2) * (ia.w - ta.w));
        gb = make_float4((2.0f * w_l2) * (ib.x - tb.x), (2.0f * w_l2) * (ib.y - tb.y), (2.0f * w_l2) * (ib.z - tb.z),
                         (2.0f * w_l2) * (ib.w - tb.w));
      } else {
        ga = row4(g + pA * ld_g + c0, vg, n);
        gb = row4(g + pB * ld_g + c0, vg, n);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (j >= n) break;
        acc += (f4(ga, j) + f4(gb, j)) * (f4(ia, j) - f4(ib, j));
      }
    }
    const float dLdp = 0.5f * acc;
    if (tn < 0 || !((cm >> dir) & 1u)) {
      // overhang over background, or the neighbour's triangle holds this
      // centre and this one does not hold the neighbour's: on top
      if (axis == 0) rx += dLdp;
      else ry += dLdp;
      continue;
    }
    // intersection: both planes' slopes along the pair's axis.  The asm
    // keeps this triangle's slope here, where intersections are rare, rather
    // than hoisted before the loop for every lane.
    const Snap Sn = snap_triangle<false>(v, vw, tri_row(tri, vw, tn));
    Snap So = S;
    asm volatile("" : "+v"(So.z[0]), "+v"(So.z[1]), "+v"(So.z[2]), "+v"(So.X[0]), "+v"(So.X[1]), "+v"(So.X[2]),
                 "+v"(So.Y[0]), "+v"(So.Y[1]), "+v"(So.Y[2]), "+v"(So.D));
    const float sS = plane_slope(So, axis), sN = plane_slope(Sn, axis);
    const float sA = selfA ? sS : sN, sB = selfA ? sN : sS;
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
  const RunMask rm = run_mask(lane & 15, head & 15, t >= 0);  // runs never cross a 16-lane row
  const bool wave_any = __ballot(t >= 0) != 0;

  PixBary pb;
  pb.beta[0] = pb.beta[1] = pb.beta[2] = 0.f;
  pb.b[0] = pb.b[1] = pb.b[2] = 0.f;
  pb.Wq = 1.f;
  pb.d = 1.f;
  if (t >= 0) pb = pixel_bary(S, px, py);

  int slot[3] = {-1, -1, -1};  // the vertices' slots in the table
  if (emit) {
#pragma unroll
    for (int k = 0; k < 3; ++k) slot[k] = slot_of(s_key, s_list, &s_nocc, S.idx[k]);
  }

  auto dispatch = [&](auto&& body) {  // once per wave, with its step count as a constant
    if (!wave_any) return;
    switch (rm.steps) {
      case 0: body(Steps<0>{}); break;
      case 1: body(Steps<1>{}); break;
      case 2: body(Steps<2>{}); break;
      case 3: body(Steps<3>{}); break;
      default: body(Steps<4>{}); break;
    }
  };

  // ---- interpolation adjoint and Omega.  Both terms move vertex k's x and y
  // by beta_k times a per-pixel vector (the fragment gradient, and minus the
  // screen gradient of dL/d(beta) for Omega), so they are summed per pixel
  // first; the 1/z part differs per vertex (dw).  Omega needs dL/d(b_k) =
  // sum_c dL/d(attr_c) attr_k,c over every channel first; the run sums of
  // b_k dL/d(attr_c) come after it, from the same (cached) rows, so that only
  // the sums are live at the table's barrier.
  const long long pg = t >= 0 ? p : 0;
  const int va = row_vec(C_a, attr) == 4 && ((vw.a_off * C_a) & 3) == 0 ? 4 : row_vec(C_a, attr) == 3 ? 3 : 0;
  auto grad_row = [&](int c0, int n) -> float4 {  // dL/d(attr_c0..c0+3) of this pixel (0 for background)
    float4 gc4;
    if constexpr (L2) {
      const float4 i4 = row4(img + pg * C_e + c0, vimg, n), t4 = row4(target + pg * C_e + c0, vtar, n);
      gc4 = make_float4((2.0f * w_l2) * (i4.x - t4.x), (2.0f * w_l2) * (i4.y - t4.y), (2.0f * w_l2) * (i4.z - t4.z),
                        (2.0f * w_l2) * (i4.w - t4.w));
    } else {
      gc4 = row4(g + pg * ld_g + c0, vg, n);
    }
    if (t < 0) gc4 = make_float4(0.f, 0.f, 0.f, 0.f);
    return gc4;
  };
  // run sums of b_k dL/d(attr_c) for channels c0..c0+3: vertex k's channel c0 + j at 4 k + j
  // (the first chunk's row is read once, for both)
  const float4 gc0 = want_interp && wave_any ? grad_row(0, min(4, C_a)) : make_float4(0.f, 0.f, 0.f, 0.f);
  auto attr_sums = [&](auto steps, int c0, float(&sm)[12]) {
    constexpr int ST = decltype(steps)::value;
    const int n = min(4, C_a - c0);
    const float4 gc4 = c0 == 0 ? gc0 : grad_row(c0, n);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (j >= n) break;
        sm[4 * k + j] = seg_sum<ST>(pb.b[k] * f4(gc4, j), rm);
      }
  };
  float fx = rx, fy = ry;
  float dw[3] = {0.f, 0.f, 0.f};
  float gzc = 0.f;  // dL/d(interpolated z)
  if (want_interp && wave_any && t >= 0) {
    float G[3] = {0.f, 0.f, 0.f};
    for (int c0 = 0; c0 < C_a; c0 += 4) {
      const int n = min(4, C_a - c0);
      const float4 gc4 = c0 == 0 ? gc0 : grad_row(c0, n);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float4 a4 = row4(attr + (vw.a_off + S.idx[k]) * C_a + c0, va, n);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (j >= n) break;
          G[k] += f4(gc4, j) * f4(a4, j);
        }
      }
    }
    if (append_z) {
      gzc = L2 ? (2.0f * w_l2) * (img[pg * C_e + C_a] - target[pg * C_e + C_a]) : g[pg * ld_g + C_a];
#pragma unroll
      for (int k = 0; k < 3; ++k) G[k] += gzc * S.z[k];
    }
    const float Gb = (pb.b[0] * G[0] + pb.b[1] * G[1]) + pb.b[2] * G[2];
    const float iW = __builtin_amdgcn_rcpf(pb.Wq);
    float dbeta[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      dw[k] = (G[k] - Gb) * iW;
      dbeta[k] = dw[k] * S.q[k];
    }
    // d beta_i / d v_j = -beta_j * grad_P beta_i;  grad_P beta_i = 256 (-(Yb-Ya), Xb-Xa) / D
    const float invD = 256.0f * __builtin_amdgcn_rcpf(S.D < 0 ? -pb.d : pb.d);  // (float)D, already converted
    float sx = 0.f, sy = 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int a = (i + 1) % 3, b = (i + 2) % 3;
      sx += dbeta[i] * ((float)(-(S.Y[b] - S.Y[a])) * invD);
      sy += dbeta[i] * ((float)(S.X[b] - S.X[a]) * invD);
    }
    fx -= sx;
    fy -= sy;
  }
  const bool attr_tab = want_interp && g_attr;
  if (attr_tab) {
    // channels past the table's go straight to memory
    for (int c0 = kCTab; c0 < C_a; c0 += 4) {
      float sm[12];
#pragma unroll
      for (int i = 0; i < 12; ++i) sm[i] = 0.f;
      dispatch([&](auto steps) { attr_sums(steps, c0, sm); });
      if (emit)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (c0 + j < C_a && sm[4 * k + j] != 0.f)
              atomicAdd(g_attr + (vw.a_off + S.idx[k]) * C_a + c0 + j, sm[4 * k + j]);
    }
  }
  // the run sums the table takes: vertex k's (x, y, z) gradient at 3 k, and
  // its channels 0-3 and 4-7 at 4 k + j
  float sv[9], sa0[12], sa1[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    if (i < 9) sv[i] = 0.f;
    sa0[i] = sa1[i] = 0.f;
  }
  dispatch([&](auto steps) {
    constexpr int ST = decltype(steps)::value;
    if (g_v) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float qk = t >= 0 ? S.q[k] : 0.f;
        // 1/z part: the fragment's rq and Omega's dw, through d(1/z)/dz = -1/z^2;
        // the z channel's own interpolation weight b_k
        const float gzk = (pb.beta[k] * (rq + dw[k])) * (-(qk * qk)) + pb.b[k] * gzc;
        sv[3 * k] = seg_sum<ST>(pb.beta[k] * fx, rm);
        sv[3 * k + 1] = seg_sum<ST>(pb.beta[k] * fy, rm);
        sv[3 * k + 2] = seg_sum<ST>(gzk, rm);
      }
    }
    if (attr_tab) {
      attr_sums(steps, 0, sa0);
      if (C_a > 4) attr_sums(steps, 4, sa1);
    }
  });

  // ---- the vertex table, in fixed point.  A slot holds three groups of
  // values: the coordinates (0-2) and two groups of four attribute channels
  // (3-6, 7-10).  Every run end raises, per slot and group, the largest
  // |run sum| it adds (an integer maximum on the float's bits); after the
  // barrier it adds round(x 2^(22 - E)) as a 32-bit integer, with 2^E above
  // that maximum.  At most 256 run ends add to one value, so a sum stays
  // below 2^30; each run sum is rounded once, by at most 2^-23 of the largest
  // one of its slot and group, and the sums are exact and independent of
  // order.  The flush converts each back with one rounding.  A slot and group
  // whose maximum is not finite sends its run sums straight to memory as
  // floats, so infinities and NaNs reach the gradients as they are.
  const bool grp2 = attr_tab && C_a > 4;  // the second attribute group is in use
  if (emit) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      unsigned m0 = 0u, m1 = 0u, m2 = 0u;
      if (g_v)
#pragma unroll
        for (int j = 0; j < 3; ++j) m0 = max(m0, __float_as_uint(sv[3 * k + j]) & 0x7fffffffu);
      if (attr_tab)
#pragma unroll
        for (int j = 0; j < 4; ++j) m1 = max(m1, __float_as_uint(sa0[4 * k + j]) & 0x7fffffffu);
      if (grp2)
#pragma unroll
        for (int j = 0; j < 4; ++j) m2 = max(m2, __float_as_uint(sa1[4 * k + j]) & 0x7fffffffu);
      if (slot[k] < 0) continue;
      // a maximum with 0 changes nothing: no branch per group
      unsigned* mx = &s_mx[__umul24(slot[k], 3)];
      if (g_v) atomicMax(mx, m0);
      if (attr_tab) atomicMax(mx + 1, m1);
      if (grp2) atomicMax(mx + 2, m2);
    }
  }
  __syncthreads();  // every slot is claimed and zeroed, and its maxima are final
  if (emit) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int sk = slot[k];
#pragma unroll
      for (int grp = 0; grp < 3; ++grp) {
        if (grp == 0 ? !g_v : grp == 1 ? !attr_tab : !grp2) continue;  // groups not in use
        int sh = 0;
        bool fixed = false;
        if (sk >= 0) {
          const unsigned M = s_mx[sk * 3 + grp];
          fixed = M < 0x7f800000u;
          int E = 0;
          (void)frexpf(__uint_as_float(M), &E);
          sh = 22 - E;
        }
        const int col0 = grp == 0 ? 0 : 3 + 4 * (grp - 1);  // the group's first value in the slot
        if (fixed) {
          // every value of the group, zeros included: an integer LDS add
          // costs about the same for any number of active lanes, a branch
          // per value does not (columns past C_a hold zeros and are never
          // flushed)
          int* acc = &s_acc[__umul24(sk, kNV) + col0];
#pragma unroll
          for (int j = 0; j < (grp == 0 ? 3 : 4); ++j) {
            const float x = grp == 0 ? sv[3 * k + j] : grp == 1 ? sa0[4 * k + j] : sa1[4 * k + j];
            atomicAdd(acc + j, round_half_up(ldexpf(x, sh)));
          }
        } else {
#pragma unroll
          for (int j = 0; j < (grp == 0 ? 3 : 4); ++j) {
            const float x = grp == 0 ? sv[3 * k + j] : grp == 1 ? sa0[4 * k + j] : sa1[4 * k + j];
            if (x == 0.f || (grp > 0 && col0 + j - 3 >= C_a)) continue;
            if (grp == 0) atomicAdd(g_v + (vw.v_off + S.idx[k]) * 3 + j, x);
            else atomicAdd(g_attr + (vw.a_off + S.idx[k]) * C_a + col0 + j - 3, x);
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- flush: one global atomic per (vertex, component) of this tile,
  // every lane on one (occupied slot, component) pair: k = i nv + j, with
  // i = k / nv by a multiply and shift (exact for k < 2^16 / nv; here
  // k < 256 nv <= 2816)
  const int nv = 3 + min(C_a, kCTab);
  const int nocc = s_nocc;
  const unsigned mdiv = (65536u + (unsigned)nv - 1u) / (unsigned)nv;
  for (int k = threadIdx.x; k < nocc * nv; k += blockDim.x) {
    const int i = (int)(((unsigned)k * mdiv) >> 16), j = k - i * nv;
    const int s = s_list[i];
    const int qv = s_acc[s * kNV + j];
    if (qv == 0) continue;
    const int key = s_key[s];
    int E = 0;
    (void)frexpf(__uint_as_float(s_mx[s * 3 + (j < 3 ? 0 : j < 7 ? 1 : 2)]), &E);
    const float x = ldexpf((float)qv, E - 22);
    if (j < 3) {
      if (g_v) atomicAdd(g_v + (vw.v_off + key) * 3 + j, x);
    } else if (g_attr) {
      atomicAdd(g_attr + (vw.a_off + key) * C_a + (j - 3), x);
    }
  }
  if constexpr (LOSS) {
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
                    float* g_attr, float* g_v, long long* tab, float* loss_part, hipStream_t st) {
  float* bloss = loss ? loss_part : nullptr;
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
