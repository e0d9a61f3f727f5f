// mer_device.h -- device-side pieces shared by the raster and backward kernels.
//
// Triangle set-up follows the rasterizer's contract (mer.h): vertices snapped
// to 1/256 px, exact integer edge functions, top-left rule on edges, depth key
// = interpolated 1/z in binary32 with a fixed operation order (the library is
// built with -ffp-contract=off, so nothing below is fused).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mer.h"

namespace mer {

constexpr float kGuard = 1048576.0f;  // |x|,|y| beyond 2^20 px -> culled
constexpr float kZNear = 1.0e-3f;     // z at or below -> culled

// Per (view, triangle) set-up record, 64 bytes.  For edge k (opposite vertex
// k) and pixel (px, py):  E'_k = A[k] * (256 px) + B[k] * (256 py) + C[k]
// equals sign(D) * orient(v_{k+1}, v_{k+2}, centre) + tl_k, so the centre is
// covered iff all three E'_k > 0; e_k = E'_k - tl_k is the exact value.
struct __align__(16) Rec {
  long long C[3];
  int A[3];
  int B[3];
  float q[3];  // 1/z of the three vertices, binary32
  int tl;      // bit k < 3: edge k is a top or left edge; bit 3: the 32-bit raster path
               // applies; bit 4: bits 16-31 hold the binning pass's tile mask
};
static_assert(sizeof(Rec) == 64, "record layout");

// Snapped triangle in fixed point plus 1/z; ok == false when culled.
struct Snap {
  int X[3], Y[3];
  float q[3];
  float z[3];
  long long D;  // twice the signed area, fixed point squared
  int idx[3];
  bool ok;
};

// EXACT_Q: 1/z correctly rounded (the depth key and plane slopes need it);
// otherwise a hardware reciprocal, for gradient arithmetic only.
// Branch-free over the three vertices: the nine coordinates are loaded
// together (only when all three indices are in range) and every check is
// folded into ok, so a culled triangle costs the same as a kept one.
template <bool EXACT_Q = true>
__device__ __forceinline__ Snap snap_triangle(const float* __restrict__ v, const mer_view& vw,
                                              const int32_t* __restrict__ row) {
  Snap s;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    s.idx[k] = row[k];
    ok &= (unsigned)s.idx[k] < (unsigned)vw.n_v;
  }
  float p[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) p[j] = 0.f;
  if (ok) {
    const float* vb = v + vw.v_off * 3;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float* q = vb + (size_t)(unsigned)s.idx[k] * 3u;
      p[3 * k] = q[0];
      p[3 * k + 1] = q[1];
      p[3 * k + 2] = q[2];
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float x = p[3 * k], y = p[3 * k + 1], z = p[3 * k + 2];
    // z > near is false for NaN; |x|, |y| <= guard is false for NaN and inf
    ok &= (z > kZNear) & (z < INFINITY) & (fabsf(x) <= kGuard) & (fabsf(y) <= kGuard);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float x = ok ? p[3 * k] : 0.f, y = ok ? p[3 * k + 1] : 0.f, z = ok ? p[3 * k + 2] : 1.f;
    s.X[k] = (int)rintf(x * 256.0f);
    s.Y[k] = (int)rintf(y * 256.0f);
    s.q[k] = ok ? (EXACT_Q ? 1.0f / z : __builtin_amdgcn_rcpf(z)) : 0.f;
    s.z[k] = ok ? z : 0.f;
  }
  s.D = (long long)(s.X[1] - s.X[0]) * (long long)(s.Y[2] - s.Y[0]) -
        (long long)(s.X[2] - s.X[0]) * (long long)(s.Y[1] - s.Y[0]);
  s.ok = ok && s.D != 0;
  return s;
}

// Row of view-local triangle t (0 <= t < n_t): per-view base plus a 32x32-bit offset.
__device__ __forceinline__ const int32_t* tri_row(const int32_t* tri, const mer_view& vw, int t) {
  return tri + vw.t_off * 3 + (size_t)(unsigned)t * 3u;
}

// Build the coverage record from a snapped triangle.
__device__ __forceinline__ Rec make_rec(const Snap& s) {
  Rec r;
  const long long sg = s.D > 0 ? 1 : -1;
  r.tl = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int a = (k + 1) % 3, b = (k + 2) % 3;
    // orient(va, vb, P) = A * Px + B * Py + C0 with P in fixed point
    const long long A = -(long long)(s.Y[b] - s.Y[a]);
    const long long B = (long long)(s.X[b] - s.X[a]);
    const long long C0 = (long long)(s.Y[b] - s.Y[a]) * s.X[a] - (long long)(s.X[b] - s.X[a]) * s.Y[a];
    const long long As = sg * A, Bs = sg * B;
    // inward normal (As, Bs): left edge iff As > 0, top edge iff As == 0 && Bs > 0
    const int tl = (As > 0 || (As == 0 && Bs > 0)) ? 1 : 0;
    r.A[k] = (int)As;
    r.B[k] = (int)Bs;
    r.C[k] = sg * (C0 + 128 * A + 128 * B) + tl;
    r.tl |= tl << k;
    r.q[k] = s.q[k];
  }
  // bit 3: every |A|, |B| < 2^17, so offsets of up to 46 pixels from a tile
  // origin, 256 * (A dx + B dy), fit in 31 bits (the tile raster's 32-bit path)
  bool small = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) small = small && abs(r.A[k]) < (1 << 17) && abs(r.B[k]) < (1 << 17);
  if (small) r.tl |= 8;
  return r;
}

// Biased edge functions at pixel (px, py).
__device__ __forceinline__ void edge_eval(const Rec& r, int px, int py, long long E[3]) {
  const int PX = px * 256, PY = py * 256;  // |.| < 2^23: both factors are 32-bit
#pragma unroll
  for (int k = 0; k < 3; ++k) E[k] = (long long)r.A[k] * (long long)PX + (long long)r.B[k] * (long long)PY + r.C[k];
}

__device__ __forceinline__ bool covered(const long long E[3]) { return E[0] > 0 && E[1] > 0 && E[2] > 0; }

// Can any pixel centre in [x0, x1] x [y0, y1] be covered?  Each edge function
// is linear, so its maximum over the box of centres sits at the corner its
// inward normal points to; if one edge is <= 0 there, no centre is covered.
__device__ __forceinline__ bool box_may_cover(const Rec& r, int x0, int y0, int x1, int y1) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int X = (r.A[k] > 0 ? x1 : x0) * 256, Y = (r.B[k] > 0 ? y1 : y0) * 256;
    if ((long long)r.A[k] * (long long)X + (long long)r.B[k] * (long long)Y + r.C[k] <= 0) return false;
  }
  return true;
}

// Exact unbiased edge values as binary32, and d = (float)(|D|).
__device__ __forceinline__ void edge_values(const Rec& r, const long long E[3], float e[3], float& d) {
  long long u0 = E[0] - (r.tl & 1), u1 = E[1] - ((r.tl >> 1) & 1), u2 = E[2] - ((r.tl >> 2) & 1);
  e[0] = (float)u0;
  e[1] = (float)u1;
  e[2] = (float)u2;
  d = (float)(u0 + u1 + u2);
}

// Depth key: ((e0 q0 + e1 q1) + e2 q2) / d, one rounding per operation.
__device__ __forceinline__ float depth_key(const Rec& r, const float e[3], float d) {
  float a = e[0] * r.q[0];
  float b = e[1] * r.q[1];
  float c = e[2] * r.q[2];
  float n = a + b;
  n = n + c;
  return n / d;
}

// 64-bit visibility key: larger 1/z wins, then smaller triangle id.  1/z > 0,
// so its IEEE bits order like the value.
__device__ __forceinline__ unsigned long long vis_key(float q, int t) {
  return ((unsigned long long)__float_as_uint(q) << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)t);
}
__device__ __forceinline__ int key_tri(unsigned long long k) {
  return k == 0ull ? -1 : (int)(0xFFFFFFFFu - (unsigned)(k & 0xFFFFFFFFull));
}
__device__ __forceinline__ float key_q(unsigned long long k) { return __uint_as_float((unsigned)(k >> 32)); }

// Exact sign(D) * orient(v_{k+1}, v_{k+2}, centre of (px, py)) straight from
// the snapped vertices: every factor is a 32-bit integer.
__device__ __forceinline__ void edge_at(const Snap& s, int px, int py, long long E[3]) {
  const int Px = px * 256 + 128, Py = py * 256 + 128;
  const bool neg = s.D < 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int a = (k + 1) % 3, b = (k + 2) % 3;
    const long long e = (long long)(s.X[b] - s.X[a]) * (long long)(Py - s.Y[a]) -
                        (long long)(s.Y[b] - s.Y[a]) * (long long)(Px - s.X[a]);
    E[k] = neg ? -e : e;
  }
}

// The same edge values in 32-bit arithmetic.  With the vertices taken
// relative to the pixel centre, (x_k, y_k) = (X_k - Px, Y_k - Py), the
// orientation of edge (a, b) at the centre is x_a y_b - x_b y_a.  When every
// |x_k|, |y_k| is at most 2^14 (the triangle lies within 64 pixels of the
// centre) each product is at most 2^28 in magnitude, so the 24-bit multiplier
// gives it exactly, and the edge values, their sum |D| and the steps to the
// neighbouring centres (below 2^23) fit in 32 bits: bit for bit the 64-bit
// values.  ok is false when the bound does not hold.
struct Rel32 {
  int x[3], y[3];
  bool ok;
};
__device__ __forceinline__ Rel32 rel32(const Snap& s, int px, int py) {
  const unsigned Px = (unsigned)px * 256u + 128u, Py = (unsigned)py * 256u + 128u;
  Rel32 r;
  unsigned m = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r.x[k] = (int)((unsigned)s.X[k] - Px);
    r.y[k] = (int)((unsigned)s.Y[k] - Py);
    m |= ((unsigned)r.x[k] + (1u << 14)) | ((unsigned)r.y[k] + (1u << 14));
  }
  r.ok = m <= (1u << 15);
  return r;
}
// The 24-bit multiply as one instruction: its operands are in range here,
// so the sign extension __mul24 would add is not needed.
__device__ __forceinline__ int mul_i24(int a, int b) {
  int r;
  asm("v_mul_i32_i24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ void edge32(const Snap& s, const Rel32& r, int E[3]) {
  const bool neg = s.D < 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int a = (k + 1) % 3, b = (k + 2) % 3;
    const int e = mul_i24(r.x[a], r.y[b]) - mul_i24(r.x[b], r.y[a]);
    E[k] = neg ? -e : e;
  }
}
// Inward normal (A_k, B_k) of edge k and its top-left bit.
__device__ __forceinline__ int inward_tl(const Snap& s, int k, int& A, int& B) {
  const bool neg = s.D < 0;
  const int a = (k + 1) % 3, b = (k + 2) % 3;
  const int dy = s.Y[a] - s.Y[b], dx = s.X[b] - s.X[a];
  A = neg ? -dy : dy;
  B = neg ? -dx : dx;
  return (A > 0 || (A == 0 && B > 0)) ? 1 : 0;
}

// Coverage rule on exact edge values: E_k > 0, or E_k == 0 on a top/left edge.
__device__ __forceinline__ bool covered_at(const Snap& s, const long long E[3]) {
  const bool neg = s.D < 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (E[k] > 0) continue;
    if (E[k] < 0) return false;
    const int a = (k + 1) % 3, b = (k + 2) % 3;
    const int A = neg ? (s.Y[b] - s.Y[a]) : -(s.Y[b] - s.Y[a]);  // inward normal, x
    const int B = neg ? -(s.X[b] - s.X[a]) : (s.X[b] - s.X[a]);  // inward normal, y
    if (!(A > 0 || (A == 0 && B > 0))) return false;
  }
  return true;
}

// Is pixel (px, py)'s centre inside snapped triangle s by the coverage rule?
__device__ __forceinline__ bool contains(const Snap& s, int px, int py) {
  if (!s.ok) return false;
  const Rel32 r = rel32(s, px, py);
  if (r.ok) {
    int E[3];
    edge32(s, r, E);
    bool in = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      int A, B;
      in &= E[k] + inward_tl(s, k, A, B) > 0;
    }
    return in;
  }
  long long E[3];
  edge_at(s, px, py, E);
  return covered_at(s, E);
}

// Exact edge values of snapped triangle s at the centre of pixel (px, py),
// with their steps to the neighbouring centres.  Ep[k] = sign(D) *
// orient(v_{k+1}, v_{k+2}, centre) + tl_k, biased by the top-left rule so
// that a centre is covered iff all three are > 0; one pixel to the right
// adds dx[k] = 256 A_k, one pixel down dy[k] = 256 B_k, with (A_k, B_k) the
// inward normal of edge k.
struct PixEdges {
  long long Ep[3];
  long long dx[3], dy[3];
  int tl;  // bit k: edge k is a top or left edge
};

__device__ __forceinline__ PixEdges pix_edges(const Snap& s, int px, int py) {
  PixEdges o;
  long long E[3];
  edge_at(s, px, py, E);
  const bool neg = s.D < 0;
  o.tl = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int a = (k + 1) % 3, b = (k + 2) % 3;
    const int A = neg ? (s.Y[b] - s.Y[a]) : -(s.Y[b] - s.Y[a]);
    const int B = neg ? -(s.X[b] - s.X[a]) : (s.X[b] - s.X[a]);
    const int tl = (A > 0 || (A == 0 && B > 0)) ? 1 : 0;
    o.tl |= tl << k;
    o.Ep[k] = E[k] + tl;
    o.dx[k] = (long long)A * 256;
    o.dy[k] = (long long)B * 256;
  }
  return o;
}

// Which of the four neighbouring centres the triangle covers: bit d for
// neighbour d = 0 left, 1 right, 2 up, 3 down (same rule as the rasterizer).
__device__ __forceinline__ unsigned neighbour_cover(const PixEdges& e) {
  bool l = true, r = true, u = true, d = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    l &= e.Ep[k] - e.dx[k] > 0;
    r &= e.Ep[k] + e.dx[k] > 0;
    u &= e.Ep[k] - e.dy[k] > 0;
    d &= e.Ep[k] + e.dy[k] > 0;
  }
  return (l ? 1u : 0u) | (r ? 2u : 0u) | (u ? 4u : 0u) | (d ? 8u : 0u);
}

// neighbour_cover(pix_edges(s, px, py)), in 32 bits where rel32 allows.
__device__ __forceinline__ unsigned cover_mask(const Snap& s, int px, int py) {
  const Rel32 r = rel32(s, px, py);
  if (r.ok) {
    int E[3];
    edge32(s, r, E);
    bool l = true, rt = true, u = true, d = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      int A, B;
      const int Ep = E[k] + inward_tl(s, k, A, B);
      const int dx = A * 256, dy = B * 256;
      l &= Ep - dx > 0;
      rt &= Ep + dx > 0;
      u &= Ep - dy > 0;
      d &= Ep + dy > 0;
    }
    return (l ? 1u : 0u) | (rt ? 2u : 0u) | (u ? 4u : 0u) | (d ? 8u : 0u);
  }
  return neighbour_cover(pix_edges(s, px, py));
}

// Screen barycentrics beta_k = e_k / |D| from the exact edge values,
// perspective-correct b_k = beta_k q_k / W with W = sum_k beta_k q_k (the
// interpolated 1/z), using hardware reciprocals (about 1 ulp each).  Inside a
// triangle with |D| < 2^31 every e_k lies in [0, |D|] and converts to binary32
// in one instruction; otherwise the 64-bit conversion is used.
struct PixBary {
  float beta[3];
  float b[3];
  float Wq;
  float d;  // (float)|D|
};

__device__ __forceinline__ bool fits_i32(long long x) { return x == (long long)(int)x; }

__device__ __forceinline__ PixBary bary_from(const Snap& s, const float e[3], float d) {
  const float id = __builtin_amdgcn_rcpf(d);
  PixBary o;
  float w[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    o.beta[k] = e[k] * id;
    w[k] = o.beta[k] * s.q[k];
  }
  const float W = (w[0] + w[1]) + w[2];
  const float iW = __builtin_amdgcn_rcpf(W);
  o.b[0] = w[0] * iW;
  o.b[1] = w[1] * iW;
  o.b[2] = w[2] * iW;
  o.Wq = W;
  o.d = d;
  return o;
}

__device__ __forceinline__ PixBary pixel_bary_e(const Snap& s, const long long E[3]) {
  const long long Dabs = s.D < 0 ? -s.D : s.D;  // = E[0] + E[1] + E[2]
  float e[3], d;
  if (fits_i32(E[0]) && fits_i32(E[1]) && fits_i32(E[2]) && Dabs < 2147483648ll) {
#pragma unroll
    for (int k = 0; k < 3; ++k) e[k] = (float)(int)E[k];
    d = (float)(int)Dabs;
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) e[k] = (float)E[k];
    d = (float)Dabs;
  }
  return bary_from(s, e, d);
}

__device__ __forceinline__ PixBary pixel_bary(const Snap& s, int px, int py) {
  const Rel32 r = rel32(s, px, py);
  if (r.ok) {
    // |D| = E[0] + E[1] + E[2] < 2^31: the 32-bit conversions of pixel_bary_e
    int E[3];
    edge32(s, r, E);
    const float e[3] = {(float)E[0], (float)E[1], (float)E[2]};
    return bary_from(s, e, (float)(E[0] + E[1] + E[2]));
  }
  long long E[3];
  edge_at(s, px, py, E);
  return pixel_bary_e(s, E);
}

// Depth-key products at pixel (px, py) of snapped triangle s (EXACT_Q):
// a = e0 q0, b = e1 q1 and n = (a + b) + e2 q2 from the exact edge values and
// correctly rounded 1/z.  n / |D| is the depth key, and (a, b) / n are the
// perspective-correct barycentrics b0, b1 (beta_k q_k / W with |D| cancelled);
// the rasterizer keeps these products for the winning candidate.
__device__ __forceinline__ void resolve_products(const Snap& s, int px, int py, float& a, float& b, float& n) {
  long long E[3];
  edge_at(s, px, py, E);
  a = (float)E[0] * s.q[0];
  b = (float)E[1] * s.q[1];
  const float c = (float)E[2] * s.q[2];
  n = a + b;
  n = n + c;
}

// Slope of the plane through (x_k, y_k, 1/z_k) along axis 0 (x) or 1 (y),
// binary32 from the snapped vertices, fixed order.
__device__ __forceinline__ float plane_slope(const Snap& s, int axis) {
  const float q0 = 1.0f / s.z[0], q1 = 1.0f / s.z[1], q2 = 1.0f / s.z[2];  // correctly rounded
  float dq1 = q1 - q0;
  float dq2 = q2 - q0;
  float num;
  // snapped coordinates are at most 2^28 in magnitude: differences fit 32 bits
  if (axis == 0) {
    float a = dq1 * (float)(s.Y[2] - s.Y[0]);
    float b = dq2 * (float)(s.Y[1] - s.Y[0]);
    num = a - b;
  } else {
    float a = dq2 * (float)(s.X[1] - s.X[0]);
    float b = dq1 * (float)(s.X[2] - s.X[0]);
    num = a - b;
  }
  float n256 = num * 256.0f;
  return n256 / (float)s.D;
}

// Up to four consecutive floats of a row, with one vector load where the
// channel count allows it (vec: 4 = rows of a multiple of 4 floats at a
// 16-byte aligned base, 3 = rows of 3 floats, 0 = one load per float).
__device__ __forceinline__ float4 row4(const float* __restrict__ a, int vec, int n) {
  if (vec == 4) return *reinterpret_cast<const float4*>(a);
  if (vec == 3) {
    const float3 x = *reinterpret_cast<const float3*>(a);
    return make_float4(x.x, x.y, x.z, 0.f);
  }
  float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
  x.x = a[0];
  if (n > 1) x.y = a[1];
  if (n > 2) x.z = a[2];
  if (n > 3) x.w = a[3];
  return x;
}
__device__ __forceinline__ int row_vec(int C, const void* base) {
  return C == 3 ? 3 : ((C & 3) == 0 && ((uintptr_t)base & 15) == 0) ? 4 : 0;
}
__device__ __forceinline__ float f4(const float4& x, int j) { return j == 0 ? x.x : j == 1 ? x.y : j == 2 ? x.z : x.w; }
// Workgroups are dealt to the chip's 8 XCDs round-robin (workgroup b to XCD
// b % 8), and each XCD has its own L2.  Neighbouring tiles share data (halo
// pixels, triangles, vertices), so this maps workgroup b to a tile such that
// each XCD sweeps one contiguous run of tiles: XCD x takes tiles
// [x q + min(x, r), ...) with q = n / 8, r = n % 8 (a bijection on [0, n)).
__device__ __forceinline__ long long xcd_tile(long long b, long long n) {
  const long long q = n >> 3, r = n & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// Column and row of cell `local` of a grid `w` cells wide, in 32-bit unsigned
// division (a view has fewer than 2^31 pixels, so fewer tiles).
__device__ __forceinline__ void grid_xy(long long local, int w, int& x, int& y) {
  const unsigned l = (unsigned)local, uw = (unsigned)w;
  const unsigned q = l / uw;
  y = (int)q;
  x = (int)(l - q * uw);
}

// Largest i in [0, n) with base[i] <= g (base non-decreasing, base[0] <= g).
template <typename T>
__device__ __forceinline__ int find_bucket(const T* base, int n, long long g) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if ((long long)base[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int find_view_px(const mer_view* views, int n, long long p) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (views[mid].px_off <= p) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Bucket of g (see find_bucket), searched once per wave with a wave-uniform
// index (scalar loads) and per lane only where the wave crosses a bucket end.
template <typename T>
__device__ __forceinline__ int wave_bucket(const T* base, int n, long long g) {
  const long long g0 = g - (threadIdx.x & 63);
  const long long u = ((long long)__builtin_amdgcn_readfirstlane((int)(g0 >> 32)) << 32) |
                      (unsigned)__builtin_amdgcn_readfirstlane((int)(g0 & 0xffffffff));
  int b = __builtin_amdgcn_readfirstlane(find_bucket(base, n, u));
  if (b + 1 < n && g >= (long long)base[b + 1]) b = find_bucket(base, n, g);
  return b;
}

// View of the wave's first pixel, searched with a wave-uniform index so the
// loads go through the scalar cache.
__device__ __forceinline__ int wave_view(const mer_view* views, int n, long long p0) {
  const long long u = ((long long)__builtin_amdgcn_readfirstlane((int)(p0 >> 32)) << 32) |
                      (unsigned)__builtin_amdgcn_readfirstlane((int)(p0 & 0xffffffff));
  return __builtin_amdgcn_readfirstlane(find_view_px(views, n, u));
}

}  // namespace mer
