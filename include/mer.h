/*
 * mer.h -- C ABI of the micro-edge rasterize / interpolate / edge-gradient
 * library for AMD Instinct MI355X (gfx950).
 *
 * The calls follow the module boundaries of the method (supplement,
 * "Implementation detail"): a rasterizer that writes an index image (visible
 * triangle per pixel) and a depth image, a barycentrics stage, an attribute
 * interpolator with its backward pass, and the EdgeGrad backward pass that
 * turns dL/d(image) into dL/d(vertex position) through micro-edges between
 * neighbouring pixels (Sec. 4.2 Pixel Pairs, Eq. chain_new; Sec. 4.3 Edge
 * Classification and Gradient Scattering; Sec. 4.4 Geometry Intersections,
 * Eq. grad_int).  The EdgeGrad forward pass is the identity and has no call.
 *
 * Conventions (all calls):
 *   - Every data pointer is DEVICE memory owned by the caller.  The library
 *     allocates nothing and frees nothing.  Scratch memory is the caller's
 *     workspace, sized by mer_plan_init.
 *   - Every call enqueues work on `stream` (a hipStream_t; NULL = the null
 *     stream) and returns without waiting, except mer_status which waits.
 *     No call allocates or synchronises, so sequences of calls can be
 *     captured into a HIP graph.
 *   - Return value: MER_OK (0) or a negative MER_E* code from the synchronous
 *     argument checks; on error nothing is enqueued.
 *   - Screen vertices v: float [sum n_v, 3] rows (x_px, y_px, z) -- pixel
 *     coordinates with y down and the origin at the image corner, z the
 *     camera depth along the principal axis (> 0 in front of the camera).
 *     Pixel (x, y) covers [x, x+1) x [y, y+1); its centre is (x+1/2, y+1/2).
 *   - Triangles tri: int32 [sum n_t, 3] of view-local vertex indices.
 *   - Per-pixel buffers are packed over views (view i starts at px_off) and
 *     row-major inside a view (index px_off + y * W + x), channels last.
 *   - Index image tri_id: int32, view-local triangle index, -1 = background.
 *   - Gradient outputs (g_v, g_attr) are ACCUMULATED (+=); the caller clears
 *     them.  Float atomics make the last bits order-dependent.
 */
#ifndef MER_H
#define MER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MER_OK 0
#define MER_EINVAL (-1)     /* null required pointer, bad size or bad view   */
#define MER_EWORKSPACE (-2) /* workspace pointer null / plan inconsistent    */
#define MER_ELAUNCH (-3)    /* a kernel launch failed (hipGetLastError)      */
#define MER_ETUNING (-4)    /* unsupported tile shape                        */
#define MER_EINTERNAL (-5)  /* mer_status: an integrity check of the last
                               mer_rasterize failed (a library defect)      */
#define MER_ESCRATCH (-6)   /* mer_backward_l2_noalloc: the plan needs more
                               than MER_NOALLOC_SCRATCH_BYTES of scratch    */

/* Size of the fixed device scratch of mer_backward_l2_noalloc. */
#define MER_NOALLOC_SCRATCH_BYTES (8u << 20)

/* edge-gradient flags */
#define MER_NO_INTERSECT 1  /* ablation: intersection pairs scatter nothing   */
#define MER_SKIP_EDGE 2     /* fused backward: skip the micro-edge term       */
#define MER_SKIP_INTERP 4   /* fused backward: skip the interpolation adjoint */

/* One rasterization job: one view of one mesh.  Views may share triangles
 * (t_off) and attributes (a_off); each view has its own screen vertices. */
typedef struct mer_view {
  int64_t v_off;  /* first row of this view's vertices in v[]                */
  int64_t t_off;  /* first row of this view's triangles in tri[]             */
  int64_t a_off;  /* first row of this view's vertex attributes in attr[]   */
  int64_t px_off; /* first pixel of this view in the per-pixel buffers       */
  int32_t n_v, n_t, H, W;
} mer_view;       /* 48 bytes, no padding */

/* Tile shape (pixels), bin pool capacity (triangle-tile entries, at most
 * INT_MAX - 1; 0 picks a default from the triangle and tile counts; tiles
 * whose entries do not fit are rasterized by a slower path that scans every
 * triangle of their view) and the small-triangle limit:
 * a triangle whose box of pixel centres holds at most small_px centres is
 * rasterized by its set-up thread directly into the per-pixel z-buffer key
 * instead of being binned (0 picks the default 16, a negative value bins
 * every triangle).  The results do not depend on any of these. */
typedef struct mer_tuning {
  int32_t tile_w, tile_h; /* supported: 8x8, 16x16, 32x8, 16x8 */
  int64_t bin_cap;
  int32_t small_px;
  int32_t big_tiles; /* a triangle whose box spans more tiles is binned by a
                        whole wave (0: default 16; negative: never) */
} mer_tuning;

/* Host-side plan: totals over the view table and the workspace layout.
 * Filled by mer_plan_init; treat as opaque apart from ws_bytes. */
typedef struct mer_plan {
  int32_t n_views, tile_w, tile_h, small_px;
  int64_t total_tris, total_tiles, total_px, bin_cap;
  int64_t px_begin; /* first pixel of the first view (pixel kernels cover [px_begin, total_px)) */
  int64_t ws_bytes;
  int64_t off_viewtab, off_rec, off_bbox, off_count, off_offs, off_part, off_bins, off_status, off_key;
  int64_t n_part;
  int64_t total_btiles, off_bviewtab; /* 16x16 tiles of the backward sweep */
  int64_t total_v, off_vbase;         /* screen vertices over all views, their per-view prefix */
  int64_t off_bloss;                  /* per-wave partial sums of the fused L2 loss */
  int64_t off_big, off_bign;          /* per-workgroup lists of large triangles, lengths + offsets */
  int64_t big_tiles;                  /* see mer_tuning */
  int64_t n_bingroups, off_bigflat;   /* workgroups of the binning passes; the packed list */
  int64_t off_bigpart;                /* scan partials of the list lengths */
} mer_plan;

/* One pinhole camera per view for the vertex transform: the rows of R are
 * the camera axes in world coordinates (x right, y down, z forward), C the
 * camera centre, f the focal length and (cx, cy) the principal point in
 * pixels.  The view's n_v screen rows v_off .. v_off + n_v - 1 are its world
 * rows w_off .. w_off + n_v - 1 (views of one mesh share w_off). */
typedef struct mer_camera {
  float R[9];       /* row-major */
  float C[3];
  float f, cx, cy;
  int32_t reserved; /* set to 0 */
  int64_t w_off;
} mer_camera;       /* 72 bytes */

/* Validate the host copy of the view table (H, W in [1, 32767], n_v, n_t >= 0,
 * offsets >= 0, views packed in order; sum n_t <= INT_MAX and fewer than
 * INT_MAX raster tiles over all views) and fill *plan.  tun may be NULL (8x8
 * tiles, default pool).
 * Reads host memory only.  MER_EINVAL on a bad view, MER_ETUNING on an
 * unsupported tile shape. */
int mer_plan_init(const mer_view *views_host, int n_views, const mer_tuning *tun, mer_plan *plan);

/* Vertex transform module (supplement, "Implementation detail": vertices
 * to the camera frame, then projected onto the image plane).  For view i and
 * j < n_v, with p = R (v_world[w_off + j] - C) in binary32 (no fused
 * multiply-add): v_screen[v_off + j] = (f p_x / p_z + cx, f p_y / p_z + cy, p_z).
 * A vertex behind the camera gets p_z <= 0 and is culled by the rasterizer.
 *   cams_dev: device copy of n_views mer_camera.  v_world: float [*, 3], at
 *   least max_i(w_off + n_v) rows.  v_screen: float [*, 3] rows as the view
 *   table lays them out.  ws: the plan's workspace. */
int mer_transform(const mer_plan *plan, const mer_view *views_dev, const mer_camera *cams_dev, const float *v_world,
                  float *v_screen, void *ws, void *stream);

/* Backward of mer_transform (the derivative of the forward map):
 * g_world[w_off + j] += J^T g_screen[v_off + j] with J = d(v_screen)/d(v_world)
 * at the vertex, summed over every view that uses the vertex (float atomics). */
int mer_transform_bwd(const mer_plan *plan, const mer_view *views_dev, const mer_camera *cams_dev,
                      const float *v_world, const float *g_screen, float *g_world, void *ws, void *stream);

/* Rasterization module + barycentrics (supplement, "Rasterization module",
 * "Barycentrics module"; the z-buffer of the Rasterization module).
 * For every pixel centre: the visible triangle is the one with the largest
 * interpolated 1/z among triangles whose interior contains the centre
 * (vertices snapped to 1/256 px; exact integer edge functions; top-left rule
 * on edges; equal binary32 1/z -> smaller triangle id).  Triangles with an
 * index outside [0, n_v), a non-finite coordinate, z <= 1e-3 or |x|, |y| >
 * 2^20 px are culled (counted in mer_status).
 *   views_dev: device copy of the same view table given to mer_plan_init.
 *   tri_id: int32 [total_px] out.  depth: float [total_px] out, 1/(1/z) of
 *   the visible surface, 0 on background; NULL to skip.  bary: float
 *   [total_px, 2] out, perspective-correct (b0, b1) for tri[t][0], tri[t][1]
 *   (b2 = 1 - b0 - b1), (0, 0) on background; NULL to skip.
 *   ws: device workspace of plan->ws_bytes bytes. */
int mer_rasterize(const mer_plan *plan, const mer_view *views_dev, const float *v, const int32_t *tri,
                  int32_t *tri_id, float *depth, float *bary, void *ws, void *stream);

/* mer_rasterize and mer_interpolate in one pass: the rasterizer's resolve
 * also writes the interpolated attributes, with the arithmetic of
 * mer_interpolate on this call's index image and barycentrics, so `out` is
 * bit-identical to rasterizing then interpolating.  depth and bary may be
 * NULL; attr, C_a, append_z and out as mer_interpolate. */
int mer_rasterize_interpolate(const mer_plan *plan, const mer_view *views_dev, const float *v, const int32_t *tri,
                              int32_t *tri_id, float *depth, float *bary, const float *attr, int C_a, int append_z,
                              float *out, void *ws, void *stream);

/* Interpolation module (supplement, "Interpolation module"):
 * out[p, c] = sum_k b_k attr[a_off + tri[t][k], c] for c < C_a and, if
 * append_z, out[p, C_a] = sum_k b_k z_k (screen z of the view's vertices);
 * 0 on background.  bary may be NULL: the barycentrics are then recomputed
 * from tri_id and v exactly as mer_rasterize computes them.
 *   attr: float [*, C_a] (1 <= C_a, C_a + append_z <= 64).
 *   out: float [total_px, C_a+append_z]. */
int mer_interpolate(const mer_plan *plan, const mer_view *views_dev, const float *attr, int C_a,
                    const float *v, const int32_t *tri, const int32_t *tri_id, const float *bary,
                    int append_z, float *out, void *stream);

/* Back-face image (supplement, "Implementation detail": an image that is 1
 * where the wrong side of a triangle is visible, passed through EdgeGrad so
 * that a loss on it moves the geometry).  out[p] = 1.0f where tri_id[p]
 * names a triangle whose snapped vertices run clockwise on screen as the
 * viewer sees it, i.e. twice its signed fixed-point area D > 0 with pixel y
 * pointing down (the front of a closed mesh wound counter-clockwise seen
 * from outside has D < 0); 0.0f on background, for ids outside [0, n_t)
 * and for triangles that do not snap (culled).  Pixels in gaps between
 * views are not written.
 *   out: float [total_px] (one channel). */
int mer_backface(const mer_plan *plan, const mer_view *views_dev, const float *v, const int32_t *tri,
                 const int32_t *tri_id, float *out, void *stream);

/* EdgeGrad backward (Sec. 4.2-4.4): for every horizontal and vertical pair of
 * neighbouring pixels inside a view whose triangle ids differ,
 *   dL/dp = 1/2 sum_c (g[A,c] + g[B,c]) (img[A,c] - img[B,c])
 * with p increasing from A (left/upper) to B.  Pairs are classified by
 * testing each pixel centre against the other pixel's triangle (same rule as
 * the rasterizer): one side background -> overhang, neither contained ->
 * adjacent (nothing), one contained -> overhang with the containing side's
 * pixel on top, both -> intersection.  Overhang: the top fragment's axis
 * coordinate gets dL/dp.  Intersection: with s_A, s_B the slopes of the two
 * triangles' planes in (axis, 1/z), d = s_B - s_A (pair skipped unless
 * d > 0), u = dL/dp / d: fragment A gets (-s_A u, +u), fragment B
 * (+s_B u, -u) on (axis, 1/z).  Fragment gradients go to the three vertices
 * of the pixel's triangle with its screen-space barycentrics at the pixel
 * centre; the 1/z part reaches z through d(1/z)/dz = -1/z^2.
 *   img, g_img: float [total_px, C_e] (1 <= C_e <= 64).  g_v: float
 *   [sum n_v, 3], accumulated.  flags: MER_NO_INTERSECT. */
int mer_edge_grad(const mer_plan *plan, const mer_view *views_dev, const float *v, const int32_t *tri,
                  const int32_t *tri_id, const float *img, const float *g_img, int C_e, int flags,
                  float *g_v, void *ws, void *stream);

/* Backward of mer_interpolate (supplement: "straightforward differentiation
 * of the forward pass"), the smooth term Omega of Sec. 3:
 *   g_attr[a_off + tri[t][k], c] += b_k g_out[p, c]
 *   g_v (x, y, z) += the derivative through the perspective-correct
 *   barycentrics (screen barycentrics E_k/D of snapped vertices, snapping
 *   taken as the identity) and, if append_z, through the z channel.
 *   g_out: float [total_px, ld_out] with the C_a (+append_z) channels first.
 *   g_attr: float [*, C_a] accumulated, may be NULL; g_v may be NULL. */
int mer_interpolate_bwd(const mer_plan *plan, const mer_view *views_dev, const float *attr, int C_a,
                        const float *v, const int32_t *tri, const int32_t *tri_id, int append_z,
                        const float *g_out, int ld_out, float *g_attr, float *g_v, void *ws, void *stream);

/* Both backward passes in one sweep over the pixels: the EdgeGrad term on
 * (img, g_img, C_e) and the interpolation adjoint on the first C_a+append_z
 * channels of g_img (so the interpolated attributes must be the first
 * channels of the image).  flags: MER_NO_INTERSECT, MER_SKIP_EDGE,
 * MER_SKIP_INTERP.
 *
 * The three backward calls sweep 16x16 pixel tiles; each workgroup sums its
 * contributions per vertex in LDS before the global float atomics.  They use
 * the plan's workspace `ws` only for a small view/tile table (rewritten on
 * every call), so a backward call may follow mer_rasterize on the same
 * stream with the same workspace. */
int mer_backward_fused(const mer_plan *plan, const mer_view *views_dev, const float *v, const int32_t *tri,
                       const int32_t *tri_id, const float *attr, int C_a, int append_z, const float *img,
                       const float *g_img, int C_e, int flags, float *g_attr, float *g_v, void *ws,
                       void *stream);

/* mer_backward_fused for the L2 image loss L = w sum_p sum_c (img - target)^2
 * (supplement, "Implementation detail": an l2 photometric loss on the
 * rendered images): dL/d(img) = 2 w (img - target) is formed inside the
 * sweep instead of being read from memory, and when `loss` (one device
 * float, accumulated) is not NULL, L over every pixel of every view is added
 * to it (partial sums per wave of pixels, then one atomic).  target: float
 * [total_px, C_e], the same layout as img.  Other arguments as
 * mer_backward_fused. */
int mer_backward_l2(const mer_plan *plan, const mer_view *views_dev, const float *v, const int32_t *tri,
                    const int32_t *tri_id, const float *attr, int C_a, int append_z, const float *img,
                    const float *target, float weight, int C_e, int flags, float *g_attr, float *g_v, float *loss,
                    void *ws, void *stream);

/* mer_backward_l2 without a workspace, for callers that cannot allocate
 * one (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments and results as mer_backward_l2 minus
 * `ws`; the small scratch the backward needs (the per-view tile prefix,
 * 2 (n_views + 1) int64, and, when `loss` is not NULL, one float per wave of
 * 64 pixels) lives in a fixed array of MER_NOALLOC_SCRATCH_BYTES bytes in
 * the library's device memory, one per GPU, kept until the process ends.
 * The call allocates nothing: it uses the current device's array (the
 * stream must belong to the current device), whose address is looked up on
 * the first call on each device.  Every call on one GPU shares that array,
 * so calls that overlap on one GPU (different streams, no ordering) race;
 * calls on one stream are ordered and safe.  Nothing in the array needs to
 * start at zero: each call writes what it reads.  MER_ESCRATCH when the
 * plan needs more scratch than the array holds (about 2 million 16x16
 * tiles, i.e. ~500 M pixels, with `loss`; ~500 k views without). */
int mer_backward_l2_noalloc(const mer_plan *plan, const mer_view *views_dev, const float *v, const int32_t *tri,
                            const int32_t *tri_id, const float *attr, int C_a, int append_z, const float *img,
                            const float *target, float weight, int C_e, int flags, float *g_attr, float *g_v,
                            float *loss, void *stream);

/* Forward mode (Sec. 5, "Forward gradients": per-pixel derivatives of the
 * image with respect to a scene parameter).  For a tangent dv of the screen
 * vertices and dattr of the attributes, writes the image tangent
 *   dimg[p, c] = interior[p, c] + edge[p, c]
 * for every pixel p of every view (pixels in gaps between views are not
 * written), the transpose of mer_backward_fused: for any g,
 * sum g . dimg = (dL/dv) . dv + (dL/dattr) . dattr with dL/dv, dL/dattr what
 * mer_backward_fused returns for dL/d(img) = g.
 *   interior (c < C_a + append_z, unless MER_SKIP_INTERP; 0 on background
 *   and on the channels beyond): the derivative of sum_k b_k a_kc (and of
 *   the interpolated z) at the fixed index image, through the perspective
 *   barycentrics b_k = (beta_k / z_k) / sum_j (beta_j / z_j), beta_k = E_k / D
 *   (fixed-point snapping taken as the identity), plus sum_k b_k dattr_kc.
 *   edge (all C_e channels, unless MER_SKIP_EDGE): each pair of neighbouring
 *   pixels A (left/upper), B with different triangle ids, classified as in
 *   mer_edge_grad, moves its edge position p by dp: an overhang's dp is the
 *   axis component of the top fragment's tangent, sum_k beta_k dv_k with the
 *   fragment's own screen barycentrics beta at its centre; an intersection's
 *   dp = (-s_A dr_A + dq_A + s_B dr_B - dq_B) / (s_B - s_A), with dr the
 *   fragments' axis tangents, dq = sum_k beta_k (-1/z_k^2) dz_k their 1/z
 *   tangents and the pair skipped unless s_B - s_A > 0.  Both pixels of the
 *   pair change by 1/2 (img[A,c] - img[B,c]) dp.
 * An id naming a triangle that does not snap (culled) counts as background.
 *   dv: float [sum n_v, 3] or NULL (no geometry tangent: only dattr acts);
 *   dattr: float [*, C_a] like attr, or NULL.  attr is required unless
 *   MER_SKIP_INTERP, img [total_px, C_e] unless MER_SKIP_EDGE (with dv).
 *   dimg: float [total_px, C_e], written.  1 <= C_e <= 64; C_a + append_z
 *   <= C_e when the interior term is on.  flags: MER_NO_INTERSECT,
 *   MER_SKIP_EDGE, MER_SKIP_INTERP.  One wave per 8x8 pixel tile, one
 *   thread per pixel, no atomics: the result is deterministic.  Uses the
 *   workspace's view-tile table (rebuilt for 8x8 tiles; the backward calls
 *   rebuild it for theirs). */
int mer_jvp(const mer_plan *plan, const mer_view *views_dev, const float *v, const int32_t *tri,
            const int32_t *tri_id, const float *attr, const float *dattr, int C_a, int append_z,
            const float *img, int C_e, const float *dv, int flags, float *dimg, void *ws, void *stream);

/* Texture sampler (supplement, "Implementation detail": uv coordinates are
 * interpolated per pixel, then a neural texture is sampled at them in a
 * deferred shading step; Sec. 3 lists the texture sampler among the parts
 * the smooth term differentiates through).  Bilinear filtering with
 * clamp-to-edge addressing: texel (x, y) of the tex_h x tex_w texture is
 * centred at ((x + 1/2) / tex_w, (y + 1/2) / tex_h); s = u tex_w - 1/2 and
 * t = v tex_h - 1/2 (formed in binary64, clamped to [-1, tex_w] and
 * [-1, tex_h]), x0 = floor(s), fx = s - x0, likewise y0, fy; texels
 * (x0 + i, y0 + j), i, j in {0, 1}, each index clamped into the texture,
 * weighted (1 - fx or fx)(1 - fy or fy).  A pixel is sampled where
 * tri_id >= 0 (every pixel when tri_id is NULL) and its uv is finite; other
 * pixels of the views get 0 (gaps between views are not written).
 *   uv: float, row p holds (u, v) in its first two of ld_uv >= 2 columns
 *   (so it can be a slice of an interpolated image).  tex: float
 *   [tex_h, tex_w, C_t], channels last, 1 <= C_t <= 64.  out: float
 *   [total_px, C_t], written.  The workspace is not used. */
int mer_texture(const mer_plan *plan, const mer_view *views_dev, const int32_t *tri_id, const float *uv,
                int ld_uv, const float *tex, int tex_h, int tex_w, int C_t, float *out, void *stream);

/* Adjoint of mer_texture for dL/d(out) g_out [total_px, C_t]:
 *   g_tex [tex_h, tex_w, C_t] += the transpose of the sampling (each sampled
 *   pixel adds weight * g_out to its four texels; a workgroup sums its 16x16
 *   pixels' contributions in LDS, in 64-bit fixed point scaled to the
 *   tile's largest |g_out| (exact sums, rounded once to binary32), when the
 *   box of texels they touch holds at most 3072 values, else adds them
 *   straight to memory with float atomics);
 *   g_uv [total_px, 2] (written, every pixel of the views) = sum_c g_out[p,c]
 *   d out[p,c] / d(u, v) inside the texel cell: tex_w times the fy-blend of
 *   the two horizontal texel differences, tex_h times the fx-blend of the two
 *   vertical ones (0 where a coordinate is clamped, and for pixels that are
 *   not sampled).  g_uv then feeds mer_interpolate_bwd as the gradient of the
 *   interpolated uv.  Either output may be NULL.  tex_h * tex_w must not
 *   exceed 2^31 - 1.  Uses the workspace's view-tile table. */
int mer_texture_bwd(const mer_plan *plan, const mer_view *views_dev, const int32_t *tri_id, const float *uv,
                    int ld_uv, const float *tex, int tex_h, int tex_w, int C_t, const float *g_out, float *g_tex,
                    float *g_uv, void *ws, void *stream);

/* Wait for `stream`, then read the workspace status of the last
 * mer_rasterize: out[0] tiles whose triangle list overflowed the bin pool
 * (they were rasterized by the slower fallback, results unchanged),
 * out[1] culled triangles, out[2] triangle-tile entries needed, out[3]
 * bin pool capacity, and two integrity counts that are 0 unless the library
 * is defective: out[4] bin entries that did not name a triangle of their
 * tile's view (skipped, not read), out[5] tiles whose counter the binning
 * passes did not take back to 0 (their list has an unwritten position).
 * Returns MER_EINTERNAL, with out[] filled, when out[4] or out[5] is not 0. */
int mer_status(const mer_plan *plan, const void *ws, void *stream, int64_t out[6]);

const char *mer_strerror(int code);
int mer_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MER_H */
