// mer_backward.hip -- attribute interpolation (forward) and the fused
// backward pass: the micro-edge term of EdgeGrad (Sec. 4.2-4.4) plus the
// interpolation adjoint with the smooth term Omega (Sec. 3), one sweep over
// the pixels.
#include "mer_internal.h"

namespace mer {

// ---------------------------------------------------------- interpolate
__global__ void __launch_bounds__(256) k_interp(const mer_view* __restrict__ views, int n_views,
                                                const float* __restrict__ attr, int C_a,
                                                const float* __restrict__ v, const int32_t* __restrict__ tri,
                                                const int32_t* __restrict__ tri_id, const float* __restrict__ bary,
                                                int append_z, float* __restrict__ out, long long px_begin,
                                                long long total_px) {
  const long long p = px_begin + (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total_px) return;
  const int vi = find_view_px(views, n_views, p);
  const mer_view vw = views[vi];
  const long long local = p - vw.px_off;
  if (local < 0 || local >= (long long)vw.H * vw.W) return;
  const int C = C_a + append_z;
  float* o = out + p * C;
  int t = tri_id[p];
  if (t >= vw.n_t) t = -1;
  float b0 = 0.f, b1 = 0.f, b2 = 0.f;
  int idx[3] = {0, 0, 0};
  bool ok = false;
  if (t >= 0) {
    const int32_t* row = tri + (vw.t_off + t) * 3;
    idx[0] = row[0];
    idx[1] = row[1];
    idx[2] = row[2];
    ok = idx[0] >= 0 && idx[0] < vw.n_v && idx[1] >= 0 && idx[1] < vw.n_v && idx[2] >= 0 && idx[2] < vw.n_v;
    if (ok) {
      if (bary) {
        b0 = bary[2 * p];
        b1 = bary[2 * p + 1];
        b2 = (1.0f - b0) - b1;
      } else {
        const Snap s = snap_triangle(v, vw, row);
        ok = s.ok;
        if (ok) {
          const PixBary pb = pixel_bary(s, (int)(local % vw.W), (int)(local / vw.W));
          b0 = pb.b[0];
          b1 = pb.b[1];
          b2 = pb.b[2];
        }
      }
    }
  }
  if (!ok) {
    for (int c = 0; c < C; ++c) o[c] = 0.f;
    return;
  }
  const float* a0 = attr + (vw.a_off + idx[0]) * C_a;
  const float* a1 = attr + (vw.a_off + idx[1]) * C_a;
  const float* a2 = attr + (vw.a_off + idx[2]) * C_a;
  for (int c = 0; c < C_a; ++c) o[c] = (b0 * a0[c] + b1 * a1[c]) + b2 * a2[c];
  if (append_z) {
    const float z0 = v[(vw.v_off + idx[0]) * 3 + 2], z1 = v[(vw.v_off + idx[1]) * 3 + 2],
                z2 = v[(vw.v_off + idx[2]) * 3 + 2];
    o[C_a] = (b0 * z0 + b1 * z1) + b2 * z2;
  }
}

// ------------------------------------------------------------- backward
__device__ __forceinline__ Snap snap_id(const float* v, const int32_t* tri, const mer_view& vw, int t) {
  return snap_triangle(v, vw, tri + (vw.t_off + t) * 3);
}

// Segmented inclusive sum over lanes [head, lane] of a wave64.
__device__ __forceinline__ float seg_sum(float x, int lane, int head) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const float y = __shfl_up(x, off, 64);
    if (lane - off >= head) x += y;
  }
  return x;
}

// One thread per pixel; a wave covers 64 consecutive pixels of the packed
// buffer, so along one image row.  A triangle meets a row in one run of
// pixels (it is convex), so after the per-pixel work the wave sums each
// run's contributions with a segmented reduction and only the last lane of
// the run issues the global float atomics.
__global__ void __launch_bounds__(256) k_backward(const mer_view* __restrict__ views, int n_views,
                                                  const float* __restrict__ v, const int32_t* __restrict__ tri,
                                                  const int32_t* __restrict__ tri_id, const float* __restrict__ attr,
                                                  int C_a, int append_z, const float* __restrict__ img,
                                                  const float* __restrict__ g, int C_e, int ld_g, int flags,
                                                  float* __restrict__ g_attr, float* __restrict__ g_v,
                                                  long long px_begin, long long total_px) {
  const long long p = px_begin + (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int vi = -1, px = 0, py = -1, t = -1;
  mer_view vw;
  vw.v_off = vw.a_off = 0;
  vw.n_v = vw.n_t = vw.H = vw.W = 0;
  const int wvi = wave_view(views, n_views, p - lane);
  if (p < total_px) {
    vi = wvi;
    if (vi + 1 < n_views && p >= views[vi + 1].px_off) vi = find_view_px(views, n_views, p);
    vw = views[vi];
    const long long local = p - vw.px_off;
    if (local >= 0 && local < (long long)vw.H * vw.W) {
      px = (int)(local % vw.W);
      py = (int)(local / vw.W);
      t = tri_id[p];
      if (t >= vw.n_t || t < 0) t = -1;
    } else {
      vi = -1;
    }
  }
  Snap S;
  S.ok = false;
  if (t >= 0) S = snap_id(v, tri, vw, t);
  if (t >= 0 && !S.ok) t = -1;

  // ---- micro-edge term: fragment gradient (r_x, r_y, r_q) of this pixel
  float rx = 0.f, ry = 0.f, rq = 0.f;
  // a background pixel is never the top side of a pair, so it receives nothing
  if (t >= 0 && !(flags & MER_SKIP_EDGE)) {
#pragma unroll 1
    for (int dir = 0; dir < 4; ++dir) {
      const int nx = px + (dir == 0 ? -1 : dir == 1 ? 1 : 0);
      const int ny = py + (dir == 2 ? -1 : dir == 3 ? 1 : 0);
      if (nx < 0 || ny < 0 || nx >= vw.W || ny >= vw.H) continue;
      const long long pn = vw.px_off + (long long)ny * vw.W + nx;
      int tn = tri_id[pn];
      if (tn >= vw.n_t || tn < 0) tn = -1;
      if (tn == t) continue;
      const bool selfA = dir == 1 || dir == 3;  // self has the smaller coordinate
      const int axis = dir < 2 ? 0 : 1;
      const long long pA = selfA ? p : pn, pB = selfA ? pn : p;
      float acc = 0.f;
      for (int c = 0; c < C_e; ++c) {
        const float gs = g[pA * ld_g + c] + g[pB * ld_g + c];
        const float di = img[pA * C_e + c] - img[pB * C_e + c];
        acc += gs * di;
      }
      const float dLdp = 0.5f * acc;
      const int tA = selfA ? t : tn, tB = selfA ? tn : t;
      if (tA < 0 || tB < 0) {
        // overhang over background: the covered side is on top
        if ((tA < 0) != selfA) {
          if (axis == 0) rx += dLdp;
          else ry += dLdp;
        }
        continue;
      }
      const Snap Sn = snap_id(v, tri, vw, tn);
      const Snap& SA = selfA ? S : Sn;
      const Snap& SB = selfA ? Sn : S;
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
  }

  // ---- runs of equal (view, row, triangle) inside the wave
  const int t_prev = __shfl_up(t, 1, 64), py_prev = __shfl_up(py, 1, 64), vi_prev = __shfl_up(vi, 1, 64);
  const bool head_flag = lane == 0 || t != t_prev || py != py_prev || vi != vi_prev;
  const unsigned long long F = __ballot(head_flag);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int head = 63 - __clzll((long long)(F & upto));
  const bool tail = lane == 63 || ((F >> (lane + 1)) & 1ull);
  const bool emit = tail && t >= 0;

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

  // ---- interpolation adjoint and Omega
  if (!(flags & MER_SKIP_INTERP)) {
    const float* gp = g + (t >= 0 ? p : 0) * ld_g;
    long long arow[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) arow[k] = t >= 0 ? (vw.a_off + S.idx[k]) * C_a : 0;
    float G[3] = {0.f, 0.f, 0.f};
    for (int c = 0; c < C_a; ++c) {  // uniform trip count: every lane joins the reductions
      const float gc = t >= 0 ? gp[c] : 0.f;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (t >= 0) G[k] += gc * attr[arow[k] + c];
        if (g_attr) {
          const float s = seg_sum(pb.b[k] * gc, lane, head);
          if (emit) atomicAdd(g_attr + arow[k] + c, s);
        }
      }
    }
    if (t >= 0) {
      if (append_z) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          G[k] += gp[C_a] * S.z[k];
          gz[k] += pb.b[k] * gp[C_a];
        }
      }
      const float Gb = (pb.b[0] * G[0] + pb.b[1] * G[1]) + pb.b[2] * G[2];
      float dbeta[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float dw = (G[k] - Gb) / pb.Wq;
        dbeta[k] = dw * S.q[k];
        gz[k] += (dw * pb.beta[k]) * (-(S.q[k] * S.q[k]));
      }
      // d beta_i / d v_j = -beta_j * grad_P beta_i;  grad_P beta_i = 256 (-(Yb-Ya), Xb-Xa) / D
      const float invD = 256.0f / (float)S.D;
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
      const float sx = seg_sum(gx[k], lane, head);
      const float sy = seg_sum(gy[k], lane, head);
      const float sz = seg_sum(gz[k], lane, head);
      if (emit) {
        float* gvk = g_v + (vw.v_off + S.idx[k]) * 3;
        if (sx != 0.f) atomicAdd(gvk + 0, sx);
        if (sy != 0.f) atomicAdd(gvk + 1, sy);
        if (sz != 0.f) atomicAdd(gvk + 2, sz);
      }
    }
  }
}

int launch_interpolate(const mer_plan* P, const mer_view* views, const float* attr, int C_a, const float* v,
                       const int32_t* tri, const int32_t* tri_id, const float* bary, int append_z, float* out,
                       hipStream_t st) {
  const long long n = P->total_px - P->px_begin;
  hipLaunchKernelGGL(k_interp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, views, P->n_views, attr, C_a, v,
                     tri, tri_id, bary, append_z, out, P->px_begin, P->total_px);
  return hipGetLastError() == hipSuccess ? MER_OK : MER_ELAUNCH;
}

int launch_backward(const mer_plan* P, const mer_view* views, const float* v, const int32_t* tri,
                    const int32_t* tri_id, const float* attr, int C_a, int append_z, const float* img,
                    const float* g, int C_e, int ld_g, int flags, float* g_attr, float* g_v, hipStream_t st) {
  const long long n = P->total_px - P->px_begin;
  hipLaunchKernelGGL(k_backward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, views, P->n_views, v, tri,
                     tri_id, attr, C_a, append_z, img, g, C_e, ld_g, flags, g_attr, g_v, P->px_begin, P->total_px);
  return hipGetLastError() == hipSuccess ? MER_OK : MER_ELAUNCH;
}

}  // namespace mer
