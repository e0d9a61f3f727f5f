// mer_jvp.hip -- forward mode: the per-pixel image tangent for a tangent of
// the screen vertices (and attributes), i.e. the derivative of every pixel
// with respect to one scene parameter (Sec. 5, "Forward gradients").  It is
// the transpose of the backward sweep: the same micro-edge pairs and
// classification (Sec. 4.2-4.4), with the edge position's tangent in place of
// dL/dp, plus the forward derivative of the interpolation (Sec. 3, the smooth
// term).  One thread per pixel gathers the pairs it belongs to, so every
// output element is written once, with no atomics; the triangles a tile
// needs are snapped once into LDS.
#include "mer_internal.h"
#include "mer_tiletri.h"

namespace mer {

// Screen barycentrics e_k / |D| at pixel (px, py) of snapped triangle s.
__device__ __forceinline__ void screen_beta(const Snap& s, int px, int py, float beta[3]) {
  const Rel32 r = rel32(s, px, py);
  if (r.ok) {  // the same values from 32-bit edge values (|D| = their sum)
    int E[3];
    edge32(s, r, E);
    const float id = __builtin_amdgcn_rcpf((float)(E[0] + E[1] + E[2]));
#pragma unroll
    for (int k = 0; k < 3; ++k) beta[k] = (float)E[k] * id;
    return;
  }
  long long E[3];
  edge_at(s, px, py, E);
  const long long Dabs = s.D < 0 ? -s.D : s.D;
  const float id = __builtin_amdgcn_rcpf((float)Dabs);
#pragma unroll
  for (int k = 0; k < 3; ++k) beta[k] = (float)E[k] * id;
}

// The three vertices' tangent rows (dx, dy, dz) of snapped triangle s, from
// the view's rows dvb; read where needed rather than staged in LDS, which
// keeps the one-wave workgroups small enough for twice the waves per CU.
struct TriTangent {
  float r[9];
};
__device__ __forceinline__ TriTangent tri_tangent(const float* __restrict__ dvb, const Snap& s) {
  TriTangent g;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float* q = dvb + (size_t)(unsigned)s.idx[k] * 3u;
    g.r[3 * k] = q[0];
    g.r[3 * k + 1] = q[1];
    g.r[3 * k + 2] = q[2];
  }
  return g;
}

// Tangent (x, y, 1/z) of the fragment at pixel (px, py) of snapped triangle
// s: the point with that centre's screen barycentrics moves with its
// vertices, and 1/z_k moves by -(1/z_k)^2 dz_k.
__device__ __forceinline__ void frag_tangent(const float* __restrict__ dvb, const Snap& s, int px, int py,
                                             float dr[3]) {
  const TriTangent g = tri_tangent(dvb, s);
  float beta[3];
  screen_beta(s, px, py, beta);
  dr[0] = dr[1] = dr[2] = 0.f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dr[0] += beta[k] * g.r[3 * k];
    dr[1] += beta[k] * g.r[3 * k + 1];
    dr[2] += beta[k] * ((-(s.q[k] * s.q[k])) * g.r[3 * k + 2]);
  }
}

// One workgroup per TS x TS tile of one view, one thread per pixel.  The
// tile's triangles (and its border's) are snapped into LDS with their
// vertices' tangent rows.  For each of the four neighbours whose triangle
// differs, the pair's edge tangent dp (d_dir); then per channel
//   dimg = interior tangent (c < C_out) + 1/2 sum_dir (I_A - I_B) d_dir
// with A the left/upper pixel of each pair.
// Six waves per SIMD (80 registers, a few bytes of spills) rather than the
// five the unbounded allocation allows: the kernel waits on dependent loads
// more than it issues.
template <int TS>
__global__ void __launch_bounds__(TS * TS) __attribute__((amdgpu_waves_per_eu(6))) k_jvp(const mer_view* __restrict__ views, int n_views,
                                             const long long* __restrict__ btile_base,
                                             const float* __restrict__ v, const int32_t* __restrict__ tri,
                                             const int32_t* __restrict__ tri_id, const float* __restrict__ attr,
                                             const float* __restrict__ dattr, int C_a, int append_z,
                                             const float* __restrict__ img, int C_e, const float* __restrict__ dv,
                                             int flags, float* __restrict__ dimg) {
  __shared__ TileTris<TS, false> T;
  // per grid position: bit d when the pixel's triangle holds neighbour d's
  // centre (d: 0 left, 1 right, 2 up, 3 down); a border pixel sets only the
  // bit toward its tile neighbour
  __shared__ unsigned char s_cm[TileDims<TS>::G * TileDims<TS>::G];
  const long long n_tiles = btile_base[n_views];
  if ((long long)blockIdx.x >= n_tiles) return;  // the grid may hold spare workgroups
  const long long tile = xcd_tile(blockIdx.x, n_tiles);
  const int vi = __builtin_amdgcn_readfirstlane(find_bucket(btile_base, n_views, tile));
  const mer_view vw = views[vi];
  const long long local_tile = tile - btile_base[vi];
  const int tiles_x = (vw.W + TS - 1) / TS;
  int x0, y0;
  grid_xy(local_tile, tiles_x, x0, y0);
  x0 *= TS;
  y0 *= TS;
  tile_tris_build<TS, false>(T, vw, x0, y0, tri_id, tri, v, nullptr);
  const float* dvb = dv ? dv + vw.v_off * 3 : nullptr;

  const int lx = threadIdx.x % TS, ly = threadIdx.x / TS;
  const int px = x0 + lx, py = y0 + ly;
  const int t = tile_rec<TS>(T, lx, ly);  // record index, -1 background or outside the view
  Snap S;
  S.ok = false;
  if (t >= 0) S = tile_snap(T, t);
  const bool want_edge = dv && !(flags & MER_SKIP_EDGE);
  if (want_edge) {
    s_cm[tt_pos<TS>(lx, ly)] = t >= 0 ? (unsigned char)cover_mask(S, px, py) : (unsigned char)0;
    if (threadIdx.x < 4 * TS) {  // the border, in tile_tris_build's order: top, bottom, left, right
      const int side = threadIdx.x / TS, j = threadIdx.x % TS;
      const int bx = side < 2 ? j : side == 2 ? -1 : TS, by = side == 0 ? -1 : side == 1 ? TS : j;
      const int ix = side < 2 ? j : side == 2 ? 0 : TS - 1, iy = side == 0 ? 0 : side == 1 ? TS - 1 : j;
      const int back = side == 0 ? 3 : side == 1 ? 2 : side == 2 ? 1 : 0;  // from the border pixel to the tile
      const int tb = tile_rec<TS>(T, bx, by);
      s_cm[tt_pos<TS>(bx, by)] =
          tb >= 0 && contains(tile_snap(T, tb), x0 + ix, y0 + iy) ? (unsigned char)(1u << back) : (unsigned char)0;
    }
    __syncthreads();
  }
  if (px >= vw.W || py >= vw.H) return;
  const long long p = vw.px_off + (long long)py * vw.W + px;

  // ---- micro-edge term: tangent of the edge position of each differing pair
  float d4[4] = {0.f, 0.f, 0.f, 0.f};  // left, right, up, down
  if (want_edge) {
    // A pair of two covered pixels has a term only when one side's
    // triangle holds the other's centre (else the triangles merely touch),
    // and under NO_INTERSECT only when exactly one does: such pairs leave
    // pend before any triangle is read.
    const unsigned cm = s_cm[tt_pos<TS>(lx, ly)];
    unsigned pend = 0, held = 0;  // held bit d: neighbour d's triangle holds this centre
    int tn4[4];
#pragma unroll
    for (int dir = 0; dir < 4; ++dir) {
      const int nx = lx + (dir == 0 ? -1 : dir == 1 ? 1 : 0);
      const int ny = ly + (dir == 2 ? -1 : dir == 3 ? 1 : 0);
      tn4[dir] = tile_rec<TS>(T, nx, ny);  // -1 outside the view too
      const bool inside = px + (nx - lx) >= 0 && px + (nx - lx) < vw.W && py + (ny - ly) >= 0 && py + (ny - ly) < vw.H;
      const unsigned cS = (s_cm[tt_pos<TS>(nx, ny)] >> (dir ^ 1)) & 1u, cN = (cm >> dir) & 1u;
      held |= cS << dir;
      const bool both = t >= 0 && tn4[dir] >= 0;
      const bool term = !both || (cS | cN) && !((flags & MER_NO_INTERSECT) && (cS & cN));
      if (inside && tn4[dir] != t && term) pend |= 1u << dir;
    }
    float drs[3] = {0.f, 0.f, 0.f};  // this pixel's own fragment tangent
    if (t >= 0 && pend) frag_tangent(dvb, S, px, py, drs);
#pragma unroll 1
    while (__ballot(pend != 0)) {
      if (pend == 0) continue;
      const int dir = __builtin_ctz(pend);
      pend &= pend - 1;
      const int tn = dir == 0 ? tn4[0] : dir == 1 ? tn4[1] : dir == 2 ? tn4[2] : tn4[3];
      const int nx = px + (dir == 0 ? -1 : dir == 1 ? 1 : 0);
      const int ny = py + (dir == 2 ? -1 : dir == 3 ? 1 : 0);
      const bool selfA = dir == 1 || dir == 3;  // this pixel has the smaller coordinate
      const int axis = dir < 2 ? 0 : 1;
      float dp;
      if (tn < 0) {
        dp = drs[axis];  // overhang over background: this (covered) side is on top
      } else {
        const Snap Sn = tile_snap(T, tn);
        if (t < 0) {
          float drn[3];
          frag_tangent(dvb, Sn, nx, ny, drn);
          dp = drn[axis];
        } else {
          const bool cS = (held >> dir) & 1u;  // the neighbour's triangle holds this centre
          const bool cN = (cm >> dir) & 1u;    // this triangle holds the neighbour's centre
          if (cS != cN) {
            if (cS) {
              dp = drs[axis];
            } else {
              float drn[3];
              frag_tangent(dvb, Sn, nx, ny, drn);
              dp = drn[axis];
            }
          } else {
            // A = left/upper pixel.  dp = (-sA drA_axis + drA_q + sB drB_axis - drB_q) / (sB - sA)
            const float s_self = plane_slope(S, axis), s_n = plane_slope(Sn, axis);
            const float sA = selfA ? s_self : s_n, sB = selfA ? s_n : s_self;
            const float dlt = sB - sA;
            if (!(dlt > 0.f) || !isfinite(dlt)) continue;
            float drn[3];
            frag_tangent(dvb, Sn, nx, ny, drn);
            const float* drA = selfA ? drs : drn;
            const float* drB = selfA ? drn : drs;
            const float num = ((-sA) * drA[axis] + drA[2]) + (sB * drB[axis] - drB[2]);
            dp = num / dlt;
          }
        }
      }
      if (dir == 0) d4[0] = dp;
      else if (dir == 1) d4[1] = dp;
      else if (dir == 2) d4[2] = dp;
      else d4[3] = dp;
    }
  }

  // ---- interior: forward derivative of sum_k b_k a_kc at the fixed index
  float db[3] = {0.f, 0.f, 0.f}, b[3] = {0.f, 0.f, 0.f};
  float zt = 0.f;  // tangent of the interpolated z
  const bool interior = t >= 0 && !(flags & MER_SKIP_INTERP);
  if (interior) {
    const PixBary pb = pixel_bary(S, px, py);
#pragma unroll
    for (int k = 0; k < 3; ++k) b[k] = pb.b[k];
    if (dv) {
      // the material point at this centre moves by delta = sum_j beta_j dv_j,
      // so beta_i changes by -grad_P beta_i . delta
      const TriTangent gt = tri_tangent(dvb, S);
      float ex = 0.f, ey = 0.f;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        ex += pb.beta[j] * gt.r[3 * j];
        ey += pb.beta[j] * gt.r[3 * j + 1];
      }
      const float invD = 256.0f * __builtin_amdgcn_rcpf(S.D < 0 ? -pb.d : pb.d);  // (float)D, already converted
      float dw[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int a = (i + 1) % 3, c = (i + 2) % 3;
        const float gxi = (float)(-(S.Y[c] - S.Y[a])) * invD;
        const float gyi = (float)(S.X[c] - S.X[a]) * invD;
        const float dbeta = -(gxi * ex + gyi * ey);
        dw[i] = dbeta * S.q[i] + pb.beta[i] * ((-(S.q[i] * S.q[i])) * gt.r[3 * i + 2]);
      }
      const float dW = (dw[0] + dw[1]) + dw[2];
      const float iW = __builtin_amdgcn_rcpf(pb.Wq);
#pragma unroll
      for (int k = 0; k < 3; ++k) db[k] = (dw[k] - b[k] * dW) * iW;
      if (append_z) {
        zt = (db[0] * S.z[0] + db[1] * S.z[1]) + db[2] * S.z[2];
        zt += (b[0] * gt.r[2] + b[1] * gt.r[5]) + b[2] * gt.r[8];
      }
    }
  }
  const int C_out = (flags & MER_SKIP_INTERP) ? 0 : C_a + append_z;

  // ---- per channel
  const bool has_edge = (d4[0] != 0.f) | (d4[1] != 0.f) | (d4[2] != 0.f) | (d4[3] != 0.f);
  const long long W = vw.W;
  const float* i0 = img ? img + p * C_e : nullptr;
  long long arow[3] = {0, 0, 0};
  if (interior) {
#pragma unroll
    for (int k = 0; k < 3; ++k) arow[k] = (vw.a_off + S.idx[k]) * C_a;
  }
  // four channels at a time, rows as vector loads where the channel counts
  // allow (image rows of C_e floats, attribute and tangent rows of C_a);
  // each channel's arithmetic is the same, in the same order, as one at a time
  const int vimg = img ? row_vec(C_e, img) : 0;
  const bool a_al = ((vw.a_off * C_a) & 3) == 0;
  const int va = row_vec(C_a, attr) == 3 ? 3 : row_vec(C_a, attr) == 4 && a_al ? 4 : 0;
  const int vda = !dattr ? 0 : row_vec(C_a, dattr) == 3 ? 3 : row_vec(C_a, dattr) == 4 && a_al ? 4 : 0;
  const int vout = row_vec(C_e, dimg);
  float* out = dimg + p * C_e;
  for (int c0 = 0; c0 < C_e; c0 += 4) {
    const int n = min(4, C_e - c0);
    float xs[4] = {0.f, 0.f, 0.f, 0.f};
    if (interior && c0 < C_out) {
      if (c0 < C_a) {
        const int na = min(4, C_a - c0);
        const float4 a0 = row4(attr + arow[0] + c0, va, na), a1 = row4(attr + arow[1] + c0, va, na),
                     a2 = row4(attr + arow[2] + c0, va, na);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j < na) xs[j] = (db[0] * f4(a0, j) + db[1] * f4(a1, j)) + db[2] * f4(a2, j);
        if (dattr) {
          const float4 e0 = row4(dattr + arow[0] + c0, vda, na), e1 = row4(dattr + arow[1] + c0, vda, na),
                       e2 = row4(dattr + arow[2] + c0, vda, na);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (j < na) xs[j] += (b[0] * f4(e0, j) + b[1] * f4(e1, j)) + b[2] * f4(e2, j);
        }
      }
      if (C_out > C_a && C_a >= c0 && C_a < c0 + n) {  // the z channel
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (c0 + j == C_a) xs[j] = zt;
      }
    }
    if (has_edge) {
      const float4 s0 = row4(i0 + c0, vimg, n);
      float e[4] = {0.f, 0.f, 0.f, 0.f};
      if (d4[0] != 0.f) {
        const float4 q = row4(i0 - C_e + c0, vimg, n);
#pragma unroll
        for (int j = 0; j < 4; ++j) e[j] += (f4(q, j) - f4(s0, j)) * d4[0];
      }
      if (d4[1] != 0.f) {
        const float4 q = row4(i0 + C_e + c0, vimg, n);
#pragma unroll
        for (int j = 0; j < 4; ++j) e[j] += (f4(s0, j) - f4(q, j)) * d4[1];
      }
      if (d4[2] != 0.f) {
        const float4 q = row4(i0 - W * C_e + c0, vimg, n);
#pragma unroll
        for (int j = 0; j < 4; ++j) e[j] += (f4(q, j) - f4(s0, j)) * d4[2];
      }
      if (d4[3] != 0.f) {
        const float4 q = row4(i0 + W * C_e + c0, vimg, n);
#pragma unroll
        for (int j = 0; j < 4; ++j) e[j] += (f4(s0, j) - f4(q, j)) * d4[3];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) xs[j] += 0.5f * e[j];
    }
    if (vout == 4) {
      *reinterpret_cast<float4*>(out + c0) = make_float4(xs[0], xs[1], xs[2], xs[3]);
    } else if (vout == 3) {
      *reinterpret_cast<float3*>(out + c0) = make_float3(xs[0], xs[1], xs[2]);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j < n) out[c0 + j] = xs[j];
    }
  }
}

int launch_jvp(const mer_plan* P, const mer_view* views, const float* v, const int32_t* tri, const int32_t* tri_id,
               const float* attr, const float* dattr, int C_a, int append_z, const float* img, int C_e,
               const float* dv, int flags, float* dimg, void* ws, hipStream_t st) {
  long long* tab = (long long*)((char*)ws + P->off_bviewtab);
  // 8x8 tile prefix per view (one wave per tile); the rasterizer's status
  // words are left alone.  A view has at most 4 times as many of these tiles
  // as 16x16 ones, so 4 workgroups per 16x16 tile cover them all.
  constexpr int TS = 8, lg = 3;
  hipLaunchKernelGGL(k_prep, dim3(1), dim3(1024), 0, st, views, P->n_views, lg, lg, tab, tab + (P->n_views + 1),
                     (long long*)nullptr);
  const long long grid = P->total_btiles * (16 / TS) * (16 / TS);
  if (grid > 0)
    hipLaunchKernelGGL(k_jvp<TS>, dim3((unsigned)grid), dim3(TS * TS), 0, st, views, P->n_views,
                       tab + (P->n_views + 1), v, tri, tri_id, attr, dattr, C_a, append_z, img, C_e, dv, flags, dimg);
  return hipGetLastError() == hipSuccess ? MER_OK : MER_ELAUNCH;
}

}  // namespace mer
