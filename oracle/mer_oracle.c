/*
 * mer_oracle.c -- plain, slow CPU oracle for the micro-edge path.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  It shares no code,
 * header, table or constant with the GPU library; the two were written
 * separately from the same statement of the method.
 *
 * What it computes (one view at a time, every loop written out):
 *   - rasterisation (Implementation detail, "Rasterization module"): the
 *     nearest triangle whose interior contains each pixel centre, with a
 *     z-buffer.  Coverage uses exact integer edge functions on vertices
 *     snapped to 1/256 px and a top-left tie rule; the depth key is the
 *     interpolated 1/z in binary32, ties going to the smaller triangle id.
 *     Two loop orders: triangle-major over each bounding box, and plain
 *     every-triangle-at-every-pixel (brute force).
 *   - barycentrics and depth at a given triangle-id image, in binary64
 *     (Implementation detail, "Barycentrics module").
 *   - attribute interpolation and its adjoint, including the smooth term
 *     Omega through the barycentrics (Sec. 3 "Preliminaries", the second
 *     product-rule term; Implementation detail, "straightforward
 *     differentiation of the forward pass").
 *   - the micro-edge term (Sec. 4.2 Pixel Pairs, boxed Eq. chain_new;
 *     Sec. 4.3 Edge Classification; Sec. 4.4 Geometry Intersections,
 *     Eq. grad_int; supplement Eq. b_vec .. Eq. prd): for every pair of
 *     4-neighbours with different triangle ids, dL/dp = 1/2 (gA + gB)(IA - IB)
 *     summed over channels, classification by testing each pixel centre
 *     against the other pixel's triangle, dp/dr = 1 for the triangle on top
 *     of an overhang, and for an intersection dp/dr from the slopes of the
 *     two planes in the (axis, 1/z) slice; then fragment gradients go to the
 *     vertices through the screen-space barycentric weights.
 *   - the texture sampler (supplement, "Implementation detail": uv
 *     interpolated per pixel, a neural texture sampled there): bilinear,
 *     clamp-to-edge, and its adjoint to the texture and to uv.
 *   - forward mode (Sec. 5, "Forward gradients"): the per-pixel image tangent
 *     for a tangent of the screen vertices (and attributes), the transpose of
 *     the two reverse-mode parts above.
 *
 * Precision: binary64 throughout, except the two places where a floating
 * point result decides a discrete outcome, which are taken in binary32 in a
 * fixed operation order (the precision the GPU path decides them in):
 *   (1) the depth key that picks the visible triangle, and
 *   (2) the slopes of the two planes at an intersection pair, whose
 *       difference decides whether the pair scatters at all.
 * Build with -ffp-contract=off so no multiply-add is fused.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_SUB 256            /* fixed-point steps per pixel              */
#define ORC_HALF 128           /* pixel centre offset in fixed point       */
#define ORC_GUARD 1048576.0f   /* |x|,|y| above this (px) -> culled        */
#define ORC_ZNEAR 1.0e-3f      /* z at or below this -> culled             */

typedef struct {
  int ok;
  int32_t idx[3];     /* view-local vertex indices                    */
  int64_t X[3], Y[3]; /* snapped fixed-point positions                */
  int64_t D;          /* twice the signed fixed-point area            */
  int s;              /* sign of D                                    */
  float q32[3];       /* 1/z in binary32 (depth key, slopes)          */
  double q[3];        /* 1/z in binary64                              */
  double z[3];
} orc_tri;

/* ---------------------------------------------------------------- setup */
static void orc_setup(const float *v, int n_v, const int32_t *tri, int t, orc_tri *T) {
  T->ok = 0;
  for (int k = 0; k < 3; ++k) {
    int32_t i = tri[3 * t + k];
    T->idx[k] = i;
    if (i < 0 || i >= n_v) return;
    float x = v[3 * i + 0], y = v[3 * i + 1], z = v[3 * i + 2];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) return;
    if (!(z > ORC_ZNEAR)) return;
    if (fabsf(x) > ORC_GUARD || fabsf(y) > ORC_GUARD) return;
    T->X[k] = (int64_t)rintf(x * 256.0f);
    T->Y[k] = (int64_t)rintf(y * 256.0f);
    T->q32[k] = 1.0f / z;
    T->z[k] = (double)z;
    T->q[k] = 1.0 / (double)z;
  }
  T->D = (T->X[1] - T->X[0]) * (T->Y[2] - T->Y[0]) - (T->X[2] - T->X[0]) * (T->Y[1] - T->Y[0]);
  if (T->D == 0) return;
  T->s = T->D > 0 ? 1 : -1;
  T->ok = 1;
}

/* Edge k runs between vertices k+1 and k+2 and is opposite vertex k.
 * Top edge: horizontal with the opposite vertex below it (y grows down).
 * Left edge: not horizontal, opposite vertex strictly right of its line. */
static int orc_top_left(const orc_tri *T, int k) {
  int a = (k + 1) % 3, b = (k + 2) % 3, c = k;
  if (T->Y[a] == T->Y[b]) return T->Y[c] > T->Y[a];
  if (T->Y[a] > T->Y[b]) { int w = a; a = b; b = w; }
  int64_t cr = (T->X[c] - T->X[a]) * (T->Y[b] - T->Y[a]) - (T->X[b] - T->X[a]) * (T->Y[c] - T->Y[a]);
  return cr > 0;
}

/* E_k(P) = orient(v_{k+1}, v_{k+2}, P) times sign(D); covered iff every
 * E_k > 0, or E_k == 0 on a top-left edge. */
static int orc_cover(const orc_tri *T, int px, int py, int64_t E[3]) {
  int64_t Px = (int64_t)ORC_SUB * px + ORC_HALF, Py = (int64_t)ORC_SUB * py + ORC_HALF;
  int inside = 1;
  for (int k = 0; k < 3; ++k) {
    int a = (k + 1) % 3, b = (k + 2) % 3;
    int64_t e = (T->X[b] - T->X[a]) * (Py - T->Y[a]) - (T->Y[b] - T->Y[a]) * (Px - T->X[a]);
    e *= T->s;
    E[k] = e;
    if (e < 0 || (e == 0 && !orc_top_left(T, k))) inside = 0;
  }
  return inside;
}

/* Depth key: interpolated 1/z in binary32, fixed order, one rounding each. */
static float orc_qkey(const orc_tri *T, const int64_t E[3]) {
  float e0 = (float)E[0], e1 = (float)E[1], e2 = (float)E[2];
  float d = (float)(T->D * T->s);
  float a = e0 * T->q32[0];
  float b = e1 * T->q32[1];
  float c = e2 * T->q32[2];
  float n = a + b;
  n = n + c;
  return n / d;
}

static int64_t orc_floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

/* ------------------------------------------------------------ rasterise */
/* tri_id[H*W] (-1 = background); qkey[H*W] (nullable) the winning key.
 * brute = 1 tests every triangle at every pixel; 0 walks each triangle's
 * bounding box of pixel centres.  Returns the number of culled triangles. */
int orc_rasterize(const float *v, int n_v, const int32_t *tri, int n_t, int H, int W,
                  int brute, int32_t *tri_id, float *qkey) {
  float *best = (float *)malloc(sizeof(float) * (size_t)H * W);
  for (int64_t p = 0; p < (int64_t)H * W; ++p) { tri_id[p] = -1; best[p] = 0.0f; }
  int culled = 0;
  orc_tri T;
  int64_t E[3];
  if (brute) {
    orc_tri *all = (orc_tri *)malloc(sizeof(orc_tri) * (size_t)(n_t > 0 ? n_t : 1));
    for (int t = 0; t < n_t; ++t) { orc_setup(v, n_v, tri, t, &all[t]); culled += !all[t].ok; }
    for (int py = 0; py < H; ++py)
      for (int px = 0; px < W; ++px) {
        int64_t p = (int64_t)py * W + px;
        for (int t = 0; t < n_t; ++t) {
          if (!all[t].ok || !orc_cover(&all[t], px, py, E)) continue;
          float q = orc_qkey(&all[t], E);
          if (tri_id[p] < 0 || q > best[p] || (q == best[p] && t < tri_id[p])) { tri_id[p] = t; best[p] = q; }
        }
      }
    free(all);
  } else {
    for (int t = 0; t < n_t; ++t) {
      orc_setup(v, n_v, tri, t, &T);
      if (!T.ok) { ++culled; continue; }
      int64_t x0 = T.X[0], x1 = T.X[0], y0 = T.Y[0], y1 = T.Y[0];
      for (int k = 1; k < 3; ++k) {
        if (T.X[k] < x0) x0 = T.X[k];
        if (T.X[k] > x1) x1 = T.X[k];
        if (T.Y[k] < y0) y0 = T.Y[k];
        if (T.Y[k] > y1) y1 = T.Y[k];
      }
      /* pixel centres 256 p + 128 inside [x0, x1] */
      int64_t pxa = -orc_floordiv(-(x0 - ORC_HALF), ORC_SUB), pxb = orc_floordiv(x1 - ORC_HALF, ORC_SUB);
      int64_t pya = -orc_floordiv(-(y0 - ORC_HALF), ORC_SUB), pyb = orc_floordiv(y1 - ORC_HALF, ORC_SUB);
      if (pxa < 0) pxa = 0;
      if (pya < 0) pya = 0;
      if (pxb > W - 1) pxb = W - 1;
      if (pyb > H - 1) pyb = H - 1;
      for (int64_t py = pya; py <= pyb; ++py)
        for (int64_t px = pxa; px <= pxb; ++px) {
          if (!orc_cover(&T, (int)px, (int)py, E)) continue;
          float q = orc_qkey(&T, E);
          int64_t p = py * W + px;
          if (tri_id[p] < 0 || q > best[p] || (q == best[p] && t < tri_id[p])) { tri_id[p] = t; best[p] = q; }
        }
    }
  }
  if (qkey) memcpy(qkey, best, sizeof(float) * (size_t)H * W);
  free(best);
  return culled;
}

/* Brute-force visibility at a list of pixels (px[i], py[i]). */
void orc_raster_sample(const float *v, int n_v, const int32_t *tri, int n_t, int n_s,
                       const int32_t *px, const int32_t *py, int32_t *tri_id) {
  orc_tri T;
  int64_t E[3];
  float *best = (float *)malloc(sizeof(float) * (size_t)(n_s > 0 ? n_s : 1));
  for (int i = 0; i < n_s; ++i) { tri_id[i] = -1; best[i] = 0.0f; }
  for (int t = 0; t < n_t; ++t) {
    orc_setup(v, n_v, tri, t, &T);
    if (!T.ok) continue;
    for (int i = 0; i < n_s; ++i) {
      if (!orc_cover(&T, px[i], py[i], E)) continue;
      float q = orc_qkey(&T, E);
      if (tri_id[i] < 0 || q > best[i] || (q == best[i] && t < tri_id[i])) { tri_id[i] = t; best[i] = q; }
    }
  }
  free(best);
}

/* Number of (non-culled) triangles whose closed-by-rule interior holds each
 * pixel centre; used to check that a planar mesh covers every centre once. */
void orc_cover_count(const float *v, int n_v, const int32_t *tri, int n_t, int H, int W, int32_t *count) {
  orc_tri T;
  int64_t E[3];
  for (int64_t p = 0; p < (int64_t)H * W; ++p) count[p] = 0;
  for (int t = 0; t < n_t; ++t) {
    orc_setup(v, n_v, tri, t, &T);
    if (!T.ok) continue;
    for (int py = 0; py < H; ++py)
      for (int px = 0; px < W; ++px)
        if (orc_cover(&T, px, py, E)) count[(int64_t)py * W + px] += 1;
  }
}

/* Is pixel centre (px,py) inside triangle t by the coverage rule? */
int orc_cover_query(const float *v, int n_v, const int32_t *tri, int t, int px, int py) {
  orc_tri T;
  int64_t E[3];
  orc_setup(v, n_v, tri, t, &T);
  return T.ok && orc_cover(&T, px, py, E);
}

/* ------------------------------------------------------------- resolve */
/* Screen barycentrics beta_k = E_k / D at the pixel centre, from the exact
 * integer edge functions (exactly representable in binary64 here). */
static void orc_beta(const orc_tri *T, int px, int py, double beta[3]) {
  int64_t Px = (int64_t)ORC_SUB * px + ORC_HALF, Py = (int64_t)ORC_SUB * py + ORC_HALF;
  for (int k = 0; k < 3; ++k) {
    int a = (k + 1) % 3, b = (k + 2) % 3;
    int64_t e = (T->X[b] - T->X[a]) * (Py - T->Y[a]) - (T->Y[b] - T->Y[a]) * (Px - T->X[a]);
    beta[k] = (double)e / (double)T->D;
  }
}

/* depth[H*W] = 1/(sum beta_k q_k); bary[H*W*3] perspective-correct
 * b_k = beta_k q_k / sum_j beta_j q_j; beta[H*W*3] screen barycentrics.
 * Background: depth 0, bary 0, beta 0.  Any output may be NULL. */
void orc_resolve(const float *v, int n_v, const int32_t *tri, int H, int W, const int32_t *tri_id,
                 double *depth, double *bary, double *beta) {
  orc_tri T;
  for (int py = 0; py < H; ++py)
    for (int px = 0; px < W; ++px) {
      int64_t p = (int64_t)py * W + px;
      int t = tri_id[p];
      double bt[3] = {0, 0, 0}, b[3] = {0, 0, 0}, d = 0.0;
      if (t >= 0) {
        orc_setup(v, n_v, tri, t, &T);
        if (T.ok) {
          orc_beta(&T, px, py, bt);
          double w[3], Wsum = 0.0;
          for (int k = 0; k < 3; ++k) { w[k] = bt[k] * T.q[k]; Wsum += w[k]; }
          for (int k = 0; k < 3; ++k) b[k] = w[k] / Wsum;
          d = 1.0 / Wsum;
        }
      }
      if (depth) depth[p] = d;
      for (int k = 0; k < 3; ++k) {
        if (bary) bary[3 * p + k] = b[k];
        if (beta) beta[3 * p + k] = bt[k];
      }
    }
}

/* ---------------------------------------------------------- back faces */
/* out[H*W]: 1 where the visible triangle shows its back side, else 0
 * (supplement, "Implementation detail": the image that is 1 where the wrong
 * side of a triangle is visible, fed through EdgeGrad for the back-face
 * loss).  Orientation: pixel y points down, so a triangle whose vertices run
 * counter-clockwise on screen -- the front of a closed mesh wound with
 * outward normals -- has snapped D < 0; its back shows where D > 0.
 * Background, and an index that names a triangle that does not snap, give 0. */
void orc_backface(const float *v, int n_v, const int32_t *tri, int n_t, int H, int W, const int32_t *tri_id,
                  double *out) {
  orc_tri T;
  for (int64_t p = 0; p < (int64_t)H * W; ++p) {
    int t = tri_id[p];
    out[p] = 0.0;
    if (t < 0 || t >= n_t) continue;
    orc_setup(v, n_v, tri, t, &T);
    if (T.ok && T.D > 0) out[p] = 1.0;
  }
}

/* --------------------------------------------------------- interpolate */
/* out[H*W*(C_a+append_z)]: sum_k b_k a_kc over the visible triangle's
 * vertices; optional last channel interpolates the vertices' screen z. */
void orc_interpolate(const float *attr, int C_a, const float *v, int n_v, const int32_t *tri, int H, int W,
                     const int32_t *tri_id, int append_z, double *out) {
  int C = C_a + (append_z ? 1 : 0);
  orc_tri T;
  double *bary = (double *)malloc(sizeof(double) * 3 * (size_t)H * W);
  orc_resolve(v, n_v, tri, H, W, tri_id, NULL, bary, NULL);
  for (int64_t p = 0; p < (int64_t)H * W; ++p) {
    for (int c = 0; c < C; ++c) out[p * C + c] = 0.0;
    int t = tri_id[p];
    if (t < 0) continue;
    orc_setup(v, n_v, tri, t, &T);
    if (!T.ok) continue;
    for (int c = 0; c < C_a; ++c) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += bary[3 * p + k] * (double)attr[(int64_t)T.idx[k] * C_a + c];
      out[p * C + c] = acc;
    }
    if (append_z) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += bary[3 * p + k] * T.z[k];
      out[p * C + C_a] = acc;
    }
  }
  free(bary);
}

/* Adjoint of orc_interpolate, with Omega.  g_out[H*W*(C_a+append_z)].
 * g_attr[n_v*C_a] += dL/d attr; g_v[n_v*3] += dL/d(x, y, z) of the screen
 * vertices through the barycentrics (and the interpolated z channel). */
void orc_interpolate_bwd(const float *attr, int C_a, const float *v, int n_v, const int32_t *tri, int H, int W,
                         const int32_t *tri_id, int append_z, const double *g_out, double *g_attr, double *g_v) {
  int C = C_a + (append_z ? 1 : 0);
  orc_tri T;
  for (int py = 0; py < H; ++py)
    for (int px = 0; px < W; ++px) {
      int64_t p = (int64_t)py * W + px;
      int t = tri_id[p];
      if (t < 0) continue;
      orc_setup(v, n_v, tri, t, &T);
      if (!T.ok) continue;
      double bt[3], w[3], b[3], Wsum = 0.0;
      orc_beta(&T, px, py, bt);
      for (int k = 0; k < 3; ++k) { w[k] = bt[k] * T.q[k]; Wsum += w[k]; }
      for (int k = 0; k < 3; ++k) b[k] = w[k] / Wsum;
      const double *g = g_out + p * C;
      /* dL/d attr and dL/d b_k */
      double G[3] = {0, 0, 0};
      for (int k = 0; k < 3; ++k) {
        int64_t vi = T.idx[k];
        for (int c = 0; c < C_a; ++c) {
          if (g_attr) g_attr[vi * C_a + c] += b[k] * g[c];
          G[k] += g[c] * (double)attr[vi * C_a + c];
        }
        if (append_z) {
          G[k] += g[C_a] * T.z[k];
          if (g_v) g_v[3 * vi + 2] += b[k] * g[C_a];
        }
      }
      if (!g_v) continue;
      /* b_k = w_k / W  ->  dL/dw_k = (G_k - sum_j b_j G_j) / W */
      double Gb = b[0] * G[0] + b[1] * G[1] + b[2] * G[2];
      double dbeta[3];
      for (int k = 0; k < 3; ++k) {
        double dw = (G[k] - Gb) / Wsum;
        dbeta[k] = dw * T.q[k];
        double dq = dw * bt[k];
        g_v[3 * (int64_t)T.idx[k] + 2] += dq * (-(T.q[k] * T.q[k])); /* q = 1/z */
      }
      /* beta_i = E_i / D: d beta_i / d v_j = -beta_j grad_P beta_i */
      double gx = 0.0, gy = 0.0;
      for (int i = 0; i < 3; ++i) {
        int a = (i + 1) % 3, bb = (i + 2) % 3;
        double dxi = -256.0 * (double)(T.Y[bb] - T.Y[a]) / (double)T.D;
        double dyi = 256.0 * (double)(T.X[bb] - T.X[a]) / (double)T.D;
        gx += dbeta[i] * dxi;
        gy += dbeta[i] * dyi;
      }
      for (int j = 0; j < 3; ++j) {
        g_v[3 * (int64_t)T.idx[j] + 0] += -bt[j] * gx;
        g_v[3 * (int64_t)T.idx[j] + 1] += -bt[j] * gy;
      }
    }
}

/* --------------------------------------------------------- edge term */
/* Slope of triangle T's plane in (x, y, 1/z) along axis (0: x, 1: y), in
 * binary32 from the snapped vertices, fixed order, one rounding per op. */
static float orc_slope32(const orc_tri *T, int axis) {
  float dq1 = T->q32[1] - T->q32[0];
  float dq2 = T->q32[2] - T->q32[0];
  float num;
  if (axis == 0) {
    float a = dq1 * (float)(T->Y[2] - T->Y[0]);
    float b = dq2 * (float)(T->Y[1] - T->Y[0]);
    num = a - b;
  } else {
    float a = dq2 * (float)(T->X[1] - T->X[0]);
    float b = dq1 * (float)(T->X[2] - T->X[0]);
    num = a - b;
  }
  float n256 = num * 256.0f;
  return n256 / (float)T->D;
}

#define ORC_NO_INTERSECT 1   /* ablation: intersection pairs scatter nothing   */
#define ORC_PAIRS_H_ONLY 2   /* test aid: only horizontal neighbour pairs      */
#define ORC_PAIRS_V_ONLY 4   /* test aid: only vertical neighbour pairs        */

/* img, g: [H*W*C] per-pixel image and dL/dimage.  g_v[n_v*3] += edge term.
 * frag[H*W*3] (nullable) receives the fragment gradient (r_x, r_y, r_q) of
 * every pixel.  counts[4] (nullable) += pairs that were: overhang,
 * intersection, adjacent, intersection skipped by the slope guard. */
void orc_edge_grad(const float *v, int n_v, const int32_t *tri, int H, int W, const int32_t *tri_id,
                   const double *img, const double *g, int C, int flags, double *g_v, double *frag,
                   int64_t *counts) {
  double *r = (double *)calloc((size_t)H * W * 3, sizeof(double));
  orc_tri TA, TB;
  int64_t E[3];
  for (int py = 0; py < H; ++py)
    for (int px = 0; px < W; ++px)
      for (int axis = 0; axis < 2; ++axis) {
        if ((flags & ORC_PAIRS_H_ONLY) && axis != 0) continue;
        if ((flags & ORC_PAIRS_V_ONLY) && axis != 1) continue;
        int qx = px + (axis == 0), qy = py + (axis == 1);
        if (qx >= W || qy >= H) continue;
        int64_t A = (int64_t)py * W + px, B = (int64_t)qy * W + qx;
        int tA = tri_id[A], tB = tri_id[B];
        if (tA == tB) continue;
        double acc = 0.0;
        for (int c = 0; c < C; ++c) acc += (g[A * C + c] + g[B * C + c]) * (img[A * C + c] - img[B * C + c]);
        double dLdp = 0.5 * acc;
        int64_t fg = -1;
        int inter = 0;
        if (tA < 0) fg = B;
        else if (tB < 0) fg = A;
        else {
          orc_setup(v, n_v, tri, tA, &TA);
          orc_setup(v, n_v, tri, tB, &TB);
          int cA = TB.ok && orc_cover(&TB, px, py, E);  /* B's triangle holds A's centre */
          int cB = TA.ok && orc_cover(&TA, qx, qy, E);  /* A's triangle holds B's centre */
          if (!cA && !cB) { if (counts) counts[2]++; continue; }
          if (cA && !cB) fg = A;
          else if (!cA && cB) fg = B;
          else inter = 1;
        }
        if (!inter) {
          if (counts) counts[0]++;
          r[3 * fg + axis] += dLdp;
          continue;
        }
        if (flags & ORC_NO_INTERSECT) continue;
        float sA = orc_slope32(&TA, axis), sB = orc_slope32(&TB, axis);
        float dlt = sB - sA;
        if (!(dlt > 0.0f) || !isfinite(dlt)) { if (counts) counts[3]++; continue; }
        if (counts) counts[1]++;
        double u = dLdp / (double)dlt;
        r[3 * A + axis] += -(double)sA * u;
        r[3 * A + 2] += u;
        r[3 * B + axis] += (double)sB * u;
        r[3 * B + 2] += -u;
      }
  /* fragment -> vertices through the screen barycentrics of the pixel's own
   * triangle at its own centre; 1/z moves z by d(1/z)/dz = -1/z^2 */
  orc_tri T;
  for (int py = 0; py < H; ++py)
    for (int px = 0; px < W; ++px) {
      int64_t p = (int64_t)py * W + px;
      double *rp = r + 3 * p;
      if (frag) { frag[3 * p] = rp[0]; frag[3 * p + 1] = rp[1]; frag[3 * p + 2] = rp[2]; }
      if (rp[0] == 0.0 && rp[1] == 0.0 && rp[2] == 0.0) continue;
      int t = tri_id[p];
      if (t < 0) continue;
      orc_setup(v, n_v, tri, t, &T);
      if (!T.ok) continue;
      double bt[3];
      orc_beta(&T, px, py, bt);
      for (int k = 0; k < 3; ++k) {
        int64_t vi = T.idx[k];
        g_v[3 * vi + 0] += bt[k] * rp[0];
        g_v[3 * vi + 1] += bt[k] * rp[1];
        g_v[3 * vi + 2] += bt[k] * rp[2] * (-(T.q[k] * T.q[k]));
      }
    }
  free(r);
}

/* -------------------------------------------------------- forward mode */
/* Forward-mode (per-pixel) derivatives of the image with respect to a
 * tangent dv[n_v*3] of the screen vertices (Sec. 5 "Forward gradients": the
 * derivative of every pixel with respect to one scene parameter).  Each part
 * is the transpose of its reverse-mode counterpart above, so that for any g
 * the sum over pixels of g . dimg equals the sum over vertices of
 * (dL/dv) . dv computed by the backward functions. */

/* Tangent of the fragment seen at pixel (px, py) on triangle T: the point
 * with the fixed screen barycentrics of that centre, whose (x, y) move by
 * sum_k beta_k (dx_k, dy_k) and whose 1/z moves by sum_k beta_k d(1/z_k),
 * with d(1/z_k) = -(1/z_k)^2 dz_k. */
static void orc_frag_tangent(const orc_tri *T, int px, int py, const double *dv, double dr[3]) {
  double bt[3];
  orc_beta(T, px, py, bt);
  dr[0] = dr[1] = dr[2] = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double *d = dv + 3 * (int64_t)T->idx[k];
    dr[0] += bt[k] * d[0];
    dr[1] += bt[k] * d[1];
    dr[2] += bt[k] * (-(T->q[k] * T->q[k])) * d[2];
  }
}

/* dimg[H*W*C] += the micro-edge term: for every pair of 4-neighbours A, B
 * (B right of or below A) with different triangle ids, classified exactly as
 * in orc_edge_grad, the edge position p moves by dp (overhang: the axis
 * component of the foreground fragment's tangent; intersection: the
 * slope-form combination of both fragments' tangents), and both pixels of the
 * pair change by 1/2 (IA - IB) dp, channel by channel. */
void orc_edge_jvp(const float *v, int n_v, const int32_t *tri, int H, int W, const int32_t *tri_id,
                  const double *img, int C, int flags, const double *dv, double *dimg, int64_t *counts) {
  orc_tri TA, TB;
  int64_t E[3];
  for (int py = 0; py < H; ++py)
    for (int px = 0; px < W; ++px)
      for (int axis = 0; axis < 2; ++axis) {
        if ((flags & ORC_PAIRS_H_ONLY) && axis != 0) continue;
        if ((flags & ORC_PAIRS_V_ONLY) && axis != 1) continue;
        int qx = px + (axis == 0), qy = py + (axis == 1);
        if (qx >= W || qy >= H) continue;
        int64_t A = (int64_t)py * W + px, B = (int64_t)qy * W + qx;
        int tA = tri_id[A], tB = tri_id[B];
        if (tA == tB) continue;
        int fg = -1; /* 0: A, 1: B */
        int inter = 0;
        if (tA >= 0) orc_setup(v, n_v, tri, tA, &TA);
        if (tB >= 0) orc_setup(v, n_v, tri, tB, &TB);
        if (tA < 0) fg = 1;
        else if (tB < 0) fg = 0;
        else {
          int cA = TB.ok && orc_cover(&TB, px, py, E);
          int cB = TA.ok && orc_cover(&TA, qx, qy, E);
          if (!cA && !cB) { if (counts) counts[2]++; continue; }
          if (cA && !cB) fg = 0;
          else if (!cA && cB) fg = 1;
          else inter = 1;
        }
        double dp;
        if (!inter) {
          if (counts) counts[0]++;
          const orc_tri *T = fg == 0 ? &TA : &TB;
          if (!T->ok) continue;
          double dr[3];
          orc_frag_tangent(T, fg == 0 ? px : qx, fg == 0 ? py : qy, dv, dr);
          dp = dr[axis];
        } else {
          if (flags & ORC_NO_INTERSECT) continue;
          float sA = orc_slope32(&TA, axis), sB = orc_slope32(&TB, axis);
          float dlt = sB - sA;
          if (!(dlt > 0.0f) || !isfinite(dlt)) { if (counts) counts[3]++; continue; }
          if (counts) counts[1]++;
          double drA[3], drB[3];
          orc_frag_tangent(&TA, px, py, dv, drA);
          orc_frag_tangent(&TB, qx, qy, dv, drB);
          dp = ((-(double)sA) * drA[axis] + drA[2] + (double)sB * drB[axis] - drB[2]) / (double)dlt;
        }
        for (int c = 0; c < C; ++c) {
          double h = 0.5 * (img[A * C + c] - img[B * C + c]) * dp;
          dimg[A * C + c] += h;
          dimg[B * C + c] += h;
        }
      }
}

/* dout[H*W*(C_a+append_z)] = tangent of orc_interpolate at a fixed index
 * image when the screen vertices move by dv (nullable) and the attributes by
 * dattr[n_v*C_a] (nullable): the forward derivative of b_k = w_k / sum_j w_j
 * with w_k = beta_k / z_k, beta_k = E_k / D (continuous; snapping is taken as
 * the identity), and of sum_k b_k a_kc.  Background pixels get 0. */
void orc_interpolate_jvp(const float *attr, int C_a, const double *dattr, const float *v, int n_v,
                         const int32_t *tri, int H, int W, const int32_t *tri_id, int append_z,
                         const double *dv, double *dout) {
  int C = C_a + (append_z ? 1 : 0);
  orc_tri T;
  for (int py = 0; py < H; ++py)
    for (int px = 0; px < W; ++px) {
      int64_t p = (int64_t)py * W + px;
      for (int c = 0; c < C; ++c) dout[p * C + c] = 0.0;
      int t = tri_id[p];
      if (t < 0) continue;
      orc_setup(v, n_v, tri, t, &T);
      if (!T.ok) continue;
      double bt[3], w[3], b[3], Wsum = 0.0;
      orc_beta(&T, px, py, bt);
      for (int k = 0; k < 3; ++k) { w[k] = bt[k] * T.q[k]; Wsum += w[k]; }
      for (int k = 0; k < 3; ++k) b[k] = w[k] / Wsum;
      double db[3] = {0, 0, 0}, dz[3] = {0, 0, 0};
      if (dv) {
        /* moving every vertex by dv_j moves the material point at this
         * centre by delta = sum_j beta_j dv_j (xy), so beta_i changes by
         * -grad_P beta_i . delta */
        double ex = 0.0, ey = 0.0;
        for (int j = 0; j < 3; ++j) {
          ex += bt[j] * dv[3 * (int64_t)T.idx[j] + 0];
          ey += bt[j] * dv[3 * (int64_t)T.idx[j] + 1];
          dz[j] = dv[3 * (int64_t)T.idx[j] + 2];
        }
        double dw[3], dW = 0.0;
        for (int i = 0; i < 3; ++i) {
          int a = (i + 1) % 3, bb = (i + 2) % 3;
          double gxi = -256.0 * (double)(T.Y[bb] - T.Y[a]) / (double)T.D;
          double gyi = 256.0 * (double)(T.X[bb] - T.X[a]) / (double)T.D;
          double dbeta = -(gxi * ex + gyi * ey);
          double dq = -(T.q[i] * T.q[i]) * dz[i];
          dw[i] = dbeta * T.q[i] + bt[i] * dq;
          dW += dw[i];
        }
        for (int k = 0; k < 3; ++k) db[k] = (dw[k] - b[k] * dW) / Wsum;
      }
      for (int c = 0; c < C_a; ++c) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) {
          int64_t vi = T.idx[k];
          acc += db[k] * (double)attr[vi * C_a + c];
          if (dattr) acc += b[k] * dattr[vi * C_a + c];
        }
        dout[p * C + c] = acc;
      }
      if (append_z) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += db[k] * T.z[k] + b[k] * dz[k];
        dout[p * C + C_a] = acc;
      }
    }
}

/* ------------------------------------------------------ texture sampler */
/* Deferred texturing (supplement, "Implementation detail": uv coordinates
 * are interpolated per pixel and a neural texture is sampled at them; Sec. 3
 * names the texture sampler among the parts the smooth term differentiates
 * through).  tex[(y * tw + x) * C + c], texel (x, y) centred at
 * ((x + 1/2) / tw, (y + 1/2) / th).  Bilinear filtering with clamp-to-edge
 * addressing: s = u tw - 1/2 and t = v th - 1/2 (first clamped to
 * [-1, tw] and [-1, th]), x0 = floor(s), fx = s - x0, likewise y0, fy, and
 * the four texels (x0 + i, y0 + j), i, j in {0, 1}, each index clamped to the
 * texture, weighted (1 - fx or fx) (1 - fy or fy).  A pixel is sampled
 * where tri_id >= 0 (all pixels when tri_id is NULL) and its uv is finite;
 * other pixels give 0 and take no gradient. */
static int orc_tex_setup(const double *uvp, int th, int tw, int64_t xi[2], int64_t yi[2], double *fx,
                         double *fy) {
  double u = uvp[0], w = uvp[1];
  if (!isfinite(u) || !isfinite(w)) return 0;
  double s = u * tw - 0.5, t = w * th - 0.5;
  if (s < -1.0) s = -1.0;
  if (s > (double)tw) s = (double)tw;
  if (t < -1.0) t = -1.0;
  if (t > (double)th) t = (double)th;
  double x0 = floor(s), y0 = floor(t);
  *fx = s - x0;
  *fy = t - y0;
  for (int i = 0; i < 2; ++i) {
    int64_t x = (int64_t)x0 + i, y = (int64_t)y0 + i;
    xi[i] = x < 0 ? 0 : (x > tw - 1 ? tw - 1 : x);
    yi[i] = y < 0 ? 0 : (y > th - 1 ? th - 1 : y);
  }
  return 1;
}

/* out[n*C] = bilinear samples; uv[n*ld_uv] holds (u, v) in its first two columns. */
void orc_texture(const double *tex, int th, int tw, int C, int64_t n, const double *uv, int ld_uv,
                 const int32_t *tri_id, double *out) {
  for (int64_t p = 0; p < n; ++p) {
    for (int c = 0; c < C; ++c) out[p * C + c] = 0.0;
    if (tri_id && tri_id[p] < 0) continue;
    int64_t xi[2], yi[2];
    double fx, fy;
    if (!orc_tex_setup(uv + p * ld_uv, th, tw, xi, yi, &fx, &fy)) continue;
    double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy};
    for (int j = 0; j < 2; ++j)
      for (int i = 0; i < 2; ++i) {
        const double *tp = tex + (yi[j] * tw + xi[i]) * C;
        for (int c = 0; c < C; ++c) out[p * C + c] += wx[i] * wy[j] * tp[c];
      }
  }
}

/* Adjoint: g_tex[th*tw*C] += the transpose of the sampling applied to
 * g_out[n*C]; g_uv[n*2] (written) = sum_c g_out[p,c] d out[p,c] / d(u, v),
 * the derivative of the bilinear interpolant inside the cell (tw times the
 * difference of the two horizontally neighbouring texel pairs, blended by
 * fy, and likewise for v), 0 for pixels that are not sampled.  Either
 * output may be NULL. */
void orc_texture_bwd(const double *tex, int th, int tw, int C, int64_t n, const double *uv, int ld_uv,
                     const int32_t *tri_id, const double *g_out, double *g_tex, double *g_uv) {
  for (int64_t p = 0; p < n; ++p) {
    if (g_uv) g_uv[2 * p] = g_uv[2 * p + 1] = 0.0;
    if (tri_id && tri_id[p] < 0) continue;
    int64_t xi[2], yi[2];
    double fx, fy;
    const double *uvp = uv + p * ld_uv;
    if (!orc_tex_setup(uvp, th, tw, xi, yi, &fx, &fy)) continue;
    double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy};
    const double *g = g_out + p * C;
    if (g_tex)
      for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 2; ++i) {
          double *gp = g_tex + (yi[j] * tw + xi[i]) * C;
          for (int c = 0; c < C; ++c) gp[c] += wx[i] * wy[j] * g[c];
        }
    if (!g_uv) continue;
    /* where a coordinate is clamped, or in the half texel next to the edge,
     * both texels along that axis are the same and the difference is 0 */
    double du = 0.0, dvv = 0.0;
    for (int c = 0; c < C; ++c) {
      double t00 = tex[(yi[0] * tw + xi[0]) * C + c], t10 = tex[(yi[0] * tw + xi[1]) * C + c];
      double t01 = tex[(yi[1] * tw + xi[0]) * C + c], t11 = tex[(yi[1] * tw + xi[1]) * C + c];
      du += g[c] * (wy[0] * (t10 - t00) + wy[1] * (t11 - t01));
      dvv += g[c] * (wx[0] * (t01 - t00) + wx[1] * (t11 - t10));
    }
    g_uv[2 * p] = du * tw;
    g_uv[2 * p + 1] = dvv * th;
  }
}
