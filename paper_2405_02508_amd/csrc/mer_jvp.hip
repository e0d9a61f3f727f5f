// mer_jvp.hip -- forward mode: the per-pixel image tangent for a tangent of
// the screen vertices (and attributes), i.e. the derivative of every pixel
// with respect to one scene parameter (Sec. 5, "Forward gradients").  It is
// the transpose of the backward sweep: the same micro-edge pairs and
// classification (Sec. 4.2-4.4), with the edge position's tangent in place of
// dL/dp, plus the forward derivative of the interpolation (Sec. 3, the smooth
// term).  One thread per pixel gathers the pairs it belongs to, so every
// output element is written once, with no atomics.
#include "mer_internal.h"

namespace mer {

// Screen barycentrics e_k / |D| at pixel (px, py) of snapped triangle s.
__device__ __forceinline__ void screen_beta(const Snap& s, int px, int py, float beta[3]) {
  long long E[3];
  edge_at(s, px, py, E);
  const long long Dabs = s.D < 0 ? -s.D : s.D;
  const float id = __builtin_amdgcn_rcpf((float)Dabs);
#pragma unroll
  for (int k = 0; k < 3; ++k) beta[k] = (float)E[k] * id;
}

// Tangent (x, y, 1/z) of the fragment at pixel (px, py) of triangle s: the
// point with that centre's screen barycentrics moves with its vertices, and
// 1/z_k moves by -(1/z_k)^2 dz_k.
__device__ __forceinline__ void frag_tangent(const Snap& s, const float* __restrict__ dv, const mer_view& vw, int px,
                                             int py, float dr[3]) {
  float beta[3];
  screen_beta(s, px, py, beta);
  dr[0] = dr[1] = dr[2] = 0.f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float* d = dv + (vw.v_off + s.idx[k]) * 3;
    dr[0] += beta[k] * d[0];
    dr[1] += beta[k] * d[1];
    dr[2] += beta[k] * ((-(s.q[k] * s.q[k])) * d[2]);
  }
}

// One thread per pixel over [px_begin, total_px).  For each of the four
// neighbours whose triangle id differs, the pair's edge tangent dp (d_dir);
// then per channel
//   dimg = interior tangent (c < C_out) + 1/2 sum_dir (I_A - I_B) d_dir
// with A the left/upper pixel of each pair.
__global__ void __launch_bounds__(256) k_jvp(const mer_view* __restrict__ views, int n_views,
                                             const float* __restrict__ v, const int32_t* __restrict__ tri,
                                             const int32_t* __restrict__ tri_id, const float* __restrict__ attr,
                                             const float* __restrict__ dattr, int C_a, int append_z,
                                             const float* __restrict__ img, int C_e, const float* __restrict__ dv,
                                             int flags, float* __restrict__ dimg, long long px_begin,
                                             long long total_px) {
  const long long p = px_begin + (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int wvi = wave_view(views, n_views, p - (threadIdx.x & 63));
  if (p >= total_px) return;
  int vi = wvi;
  if (vi + 1 < n_views && p >= views[vi + 1].px_off) vi = find_view_px(views, n_views, p);
  const mer_view vw = views[vi];
  const long long local = p - vw.px_off;
  if (local < 0 || local >= (long long)vw.H * vw.W) return;  // gap between views
  const int px = (int)(local % vw.W), py = (int)(local / vw.W);

  int t = tri_id[p];
  if (t >= vw.n_t || t < 0) t = -1;
  Snap S;
  S.ok = false;
  if (t >= 0) S = snap_triangle<false>(v, vw, tri_row(tri, vw, t));
  if (t >= 0 && !S.ok) t = -1;  // an id that does not snap counts as background

  // ---- micro-edge term: tangent of the edge position of each differing pair
  float d4[4] = {0.f, 0.f, 0.f, 0.f};  // left, right, up, down
  if (dv && !(flags & MER_SKIP_EDGE)) {
    unsigned pend = 0;
    int tn4[4] = {-1, -1, -1, -1};
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
    float drs[3] = {0.f, 0.f, 0.f};  // this pixel's own fragment tangent
    if (t >= 0 && pend) frag_tangent(S, dv, vw, px, py, drs);
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
      Snap Sn;
      Sn.ok = false;
      if (tn >= 0) Sn = snap_triangle<false>(v, vw, tri_row(tri, vw, tn));
      const bool nfg = Sn.ok;  // neighbour covered by a triangle that snaps
      if (t < 0 && !nfg) continue;
      float dp;
      if (t < 0 || !nfg) {
        // overhang over background: the covered side is on top
        if (t >= 0) {
          dp = drs[axis];
        } else {
          float drn[3];
          frag_tangent(Sn, dv, vw, nx, ny, drn);
          dp = drn[axis];
        }
      } else {
        const bool cS = contains(Sn, px, py);  // the neighbour's triangle holds this centre
        const bool cN = contains(S, nx, ny);   // this triangle holds the neighbour's centre
        if (!cS && !cN) continue;              // adjacent: nothing
        if (cS != cN) {
          if (cS) {
            dp = drs[axis];
          } else {
            float drn[3];
            frag_tangent(Sn, dv, vw, nx, ny, drn);
            dp = drn[axis];
          }
        } else {
          if (flags & MER_NO_INTERSECT) continue;
          // A = left/upper pixel.  dp = (-sA drA_axis + drA_q + sB drB_axis - drB_q) / (sB - sA)
          Snap SA, SB;
          if (selfA) {
            SA = S;
            SB = Sn;
          } else {
            SA = Sn;
            SB = S;
          }
          const float sA = plane_slope(SA, axis), sB = plane_slope(SB, axis);
          const float dlt = sB - sA;
          if (!(dlt > 0.f) || !isfinite(dlt)) continue;
          float drn[3];
          frag_tangent(Sn, dv, vw, nx, ny, drn);
          const float* drA = selfA ? drs : drn;
          const float* drB = selfA ? drn : drs;
          const float num = ((-sA) * drA[axis] + drA[2]) + (sB * drB[axis] - drB[2]);
          dp = num / dlt;
        }
      }
      if (dir == 0) d4[0] = dp;
      else if (dir == 1) d4[1] = dp;
      else if (dir == 2) d4[2] = dp;
      else d4[3] = dp;
    }
  }

  // ---- interior: forward derivative of sum_k b_k a_kc at the fixed index
  float db[3] = {0.f, 0.f, 0.f}, b[3] = {0.f, 0.f, 0.f}, dz[3] = {0.f, 0.f, 0.f};
  const bool interior = t >= 0 && !(flags & MER_SKIP_INTERP);
  if (interior) {
    const PixBary pb = pixel_bary(S, px, py);
#pragma unroll
    for (int k = 0; k < 3; ++k) b[k] = pb.b[k];
    if (dv) {
      // the material point at this centre moves by delta = sum_j beta_j dv_j,
      // so beta_i changes by -grad_P beta_i . delta
      float ex = 0.f, ey = 0.f;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float* d = dv + (vw.v_off + S.idx[j]) * 3;
        ex += pb.beta[j] * d[0];
        ey += pb.beta[j] * d[1];
        dz[j] = d[2];
      }
      const float invD = 256.0f * __builtin_amdgcn_rcpf((float)S.D);
      float dw[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int a = (i + 1) % 3, c = (i + 2) % 3;
        const float gxi = (float)(-(S.Y[c] - S.Y[a])) * invD;
        const float gyi = (float)(S.X[c] - S.X[a]) * invD;
        const float dbeta = -(gxi * ex + gyi * ey);
        dw[i] = dbeta * S.q[i] + pb.beta[i] * ((-(S.q[i] * S.q[i])) * dz[i]);
      }
      const float dW = (dw[0] + dw[1]) + dw[2];
      const float iW = __builtin_amdgcn_rcpf(pb.Wq);
#pragma unroll
      for (int k = 0; k < 3; ++k) db[k] = (dw[k] - b[k] * dW) * iW;
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
  float* out = dimg + p * C_e;
  for (int c = 0; c < C_e; ++c) {
    float x = 0.f;
    if (interior && c < C_out) {
      if (c < C_a) {
        x = (db[0] * attr[arow[0] + c] + db[1] * attr[arow[1] + c]) + db[2] * attr[arow[2] + c];
        if (dattr) x += (b[0] * dattr[arow[0] + c] + b[1] * dattr[arow[1] + c]) + b[2] * dattr[arow[2] + c];
      } else {
        x = (db[0] * S.z[0] + db[1] * S.z[1]) + db[2] * S.z[2];
        x += (b[0] * dz[0] + b[1] * dz[1]) + b[2] * dz[2];
      }
    }
    if (has_edge) {
      const float s0 = i0[c];
      float e = 0.f;
      if (d4[0] != 0.f) e += (i0[c - C_e] - s0) * d4[0];
      if (d4[1] != 0.f) e += (s0 - i0[c + C_e]) * d4[1];
      if (d4[2] != 0.f) e += (i0[c - W * C_e] - s0) * d4[2];
      if (d4[3] != 0.f) e += (s0 - i0[c + W * C_e]) * d4[3];
      x += 0.5f * e;
    }
    out[c] = x;
  }
}

int launch_jvp(const mer_plan* P, const mer_view* views, const float* v, const int32_t* tri, const int32_t* tri_id,
               const float* attr, const float* dattr, int C_a, int append_z, const float* img, int C_e,
               const float* dv, int flags, float* dimg, hipStream_t st) {
  const long long n = P->total_px - P->px_begin;
  if (n > 0)
    hipLaunchKernelGGL(k_jvp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, views, P->n_views, v, tri, tri_id,
                       attr, dattr, C_a, append_z, img, C_e, dv, flags, dimg, P->px_begin, P->total_px);
  return hipGetLastError() == hipSuccess ? MER_OK : MER_ELAUNCH;
}

}  // namespace mer
