"""CPU oracle for the micro-edge path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It wraps ``mer_oracle.c`` (plain C, built with gcc,
no code shared with the GPU library) and walks a multi-view scene one view at
a time, in float64 unless a discrete outcome is decided (see the C file).

Functions follow the paper's modules (supplement, "Implementation detail"):
rasterisation -> index image, barycentrics/depth at the index image,
interpolation and its adjoint (the smooth term Omega), the EdgeGrad
backward (Sec. 4.2-4.4), the forward-mode image tangents of both (Sec. 5,
"Forward gradients"), and the bilinear texture sampler with its adjoint
(deferred texturing of interpolated uv).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mer_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

NO_INTERSECT = 1
PAIRS_H_ONLY = 2   # test aid: horizontal neighbour pairs only
PAIRS_V_ONLY = 4   # test aid: vertical neighbour pairs only


def build() -> str:
    """Compile the oracle with gcc (no fused multiply-add, IEEE semantics)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i, i64 = ctypes.c_int, ctypes.c_int64
        L.orc_rasterize.argtypes = [P, i, P, i, i, i, i, P, P]
        L.orc_rasterize.restype = i
        L.orc_raster_sample.argtypes = [P, i, P, i, i, P, P, P]
        L.orc_cover_count.argtypes = [P, i, P, i, i, i, P]
        L.orc_cover_query.argtypes = [P, i, P, i, i, i]
        L.orc_cover_query.restype = i
        L.orc_resolve.argtypes = [P, i, P, i, i, P, P, P, P]
        L.orc_interpolate.argtypes = [P, i, P, i, P, i, i, P, i, P]
        L.orc_interpolate_bwd.argtypes = [P, i, P, i, P, i, i, P, i, P, P, P]
        L.orc_edge_grad.argtypes = [P, i, P, i, i, P, P, P, i, i, P, P, P]
        L.orc_backface.argtypes = [P, i, P, i, i, i, P, P]
        L.orc_texture.argtypes = [P, i, i, i, i64, P, i, P, P]
        L.orc_texture_bwd.argtypes = [P, i, i, i, i64, P, i, P, P, P, P]
        L.orc_edge_jvp.argtypes = [P, i, P, i, i, P, P, i, i, P, P, P]
        L.orc_interpolate_jvp.argtypes = [P, i, P, P, i, P, i, i, P, i, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- one view
def rasterize(v, tri, H, W, brute=False, with_key=False):
    v, tri = _f32(v), _i32(tri)
    tid = np.empty(H * W, np.int32)
    key = np.empty(H * W, np.float32) if with_key else None
    culled = lib().orc_rasterize(_p(v), v.shape[0], _p(tri), tri.shape[0], H, W, int(brute), _p(tid), _p(key))
    return (tid, key, culled) if with_key else tid


def raster_sample(v, tri, px, py):
    v, tri, px, py = _f32(v), _i32(tri), _i32(px), _i32(py)
    out = np.empty(px.shape[0], np.int32)
    lib().orc_raster_sample(_p(v), v.shape[0], _p(tri), tri.shape[0], px.shape[0], _p(px), _p(py), _p(out))
    return out


def cover_count(v, tri, H, W):
    v, tri = _f32(v), _i32(tri)
    out = np.empty(H * W, np.int32)
    lib().orc_cover_count(_p(v), v.shape[0], _p(tri), tri.shape[0], H, W, _p(out))
    return out


def cover_query(v, tri, t, px, py):
    v, tri = _f32(v), _i32(tri)
    return bool(lib().orc_cover_query(_p(v), v.shape[0], _p(tri), int(t), int(px), int(py)))


def backface(v, tri, H, W, tri_id):
    """1.0 where the visible triangle shows its back side (snapped D > 0 with
    pixel y down), else 0.0; f64 [H*W]."""
    v, tri, tid = _f32(v), _i32(tri), _i32(tri_id)
    out = np.zeros(H * W)
    lib().orc_backface(_p(v), v.shape[0], _p(tri), tri.shape[0], H, W, _p(tid), _p(out))
    return out


def resolve(v, tri, H, W, tri_id):
    v, tri, tri_id = _f32(v), _i32(tri), _i32(tri_id)
    depth = np.empty(H * W)
    bary = np.empty((H * W, 3))
    beta = np.empty((H * W, 3))
    lib().orc_resolve(_p(v), v.shape[0], _p(tri), H, W, _p(tri_id), _p(depth), _p(bary), _p(beta))
    return depth, bary, beta


def interpolate(attr, v, tri, H, W, tri_id, append_z=False):
    attr, v, tri, tri_id = _f32(attr), _f32(v), _i32(tri), _i32(tri_id)
    C_a = attr.shape[1]
    out = np.empty((H * W, C_a + int(append_z)))
    lib().orc_interpolate(_p(attr), C_a, _p(v), v.shape[0], _p(tri), H, W, _p(tri_id), int(append_z), _p(out))
    return out


def interpolate_bwd(attr, v, tri, H, W, tri_id, g_out, append_z=False, g_attr=None, g_v=None):
    attr, v, tri, tri_id, g_out = _f32(attr), _f32(v), _i32(tri), _i32(tri_id), _f64(g_out)
    C_a = attr.shape[1]
    if g_attr is None:
        g_attr = np.zeros((v.shape[0], C_a))
    if g_v is None:
        g_v = np.zeros((v.shape[0], 3))
    assert g_attr.dtype == np.float64 and g_attr.flags.c_contiguous
    assert g_v.dtype == np.float64 and g_v.flags.c_contiguous
    lib().orc_interpolate_bwd(_p(attr), C_a, _p(v), v.shape[0], _p(tri), H, W, _p(tri_id), int(append_z),
                              _p(g_out), _p(g_attr), _p(g_v))
    return g_attr, g_v


def edge_grad(v, tri, H, W, tri_id, img, g, flags=0, g_v=None, want_frag=False, counts=None):
    v, tri, tri_id, img, g = _f32(v), _i32(tri), _i32(tri_id), _f64(img), _f64(g)
    C = img.shape[1]
    assert g.shape == img.shape
    if g_v is None:
        g_v = np.zeros((v.shape[0], 3))
    frag = np.zeros((H * W, 3)) if want_frag else None
    if counts is None:
        counts = np.zeros(4, np.int64)
    lib().orc_edge_grad(_p(v), v.shape[0], _p(tri), H, W, _p(tri_id), _p(img), _p(g), C, int(flags),
                        _p(g_v), _p(frag), _p(counts))
    return (g_v, frag) if want_frag else g_v


def edge_jvp(v, tri, H, W, tri_id, img, dv, flags=0, dimg=None, counts=None):
    """Forward-mode micro-edge term: dimg [H*W, C] += per-pixel image
    tangent for the screen-vertex tangent dv [n_v, 3]."""
    v, tri, tri_id, img, dv = _f32(v), _i32(tri), _i32(tri_id), _f64(img), _f64(dv)
    C = img.shape[1]
    assert dv.shape == (v.shape[0], 3)
    if dimg is None:
        dimg = np.zeros((H * W, C))
    assert dimg.dtype == np.float64 and dimg.flags.c_contiguous and dimg.shape == img.shape
    if counts is None:
        counts = np.zeros(4, np.int64)
    lib().orc_edge_jvp(_p(v), v.shape[0], _p(tri), H, W, _p(tri_id), _p(img), C, int(flags), _p(dv),
                       _p(dimg), _p(counts))
    return dimg


def interpolate_jvp(attr, v, tri, H, W, tri_id, dv=None, dattr=None, append_z=False):
    """Tangent of the interpolated image [H*W, C_a + append_z] at a fixed
    index image, for vertex tangent dv [n_v, 3] and attribute tangent dattr
    [n_v, C_a] (either may be None)."""
    attr, v, tri, tri_id = _f32(attr), _f32(v), _i32(tri), _i32(tri_id)
    C_a = attr.shape[1]
    dv = None if dv is None else _f64(dv)
    dattr = None if dattr is None else _f64(dattr)
    out = np.empty((H * W, C_a + int(append_z)))
    lib().orc_interpolate_jvp(_p(attr), C_a, _p(dattr), _p(v), v.shape[0], _p(tri), H, W, _p(tri_id),
                              int(append_z), _p(dv), _p(out))
    return out


def texture(tex, uv, tri_id=None):
    """Bilinear, clamp-to-edge samples of tex [th, tw, C] at uv [n, >=2]
    (first two columns); 0 where tri_id < 0 or uv is not finite.  [n, C]."""
    tex, uv = _f64(tex), _f64(uv)
    th, tw, C = tex.shape
    n = uv.shape[0]
    tid = None if tri_id is None else _i32(tri_id)
    out = np.empty((n, C))
    lib().orc_texture(_p(tex), th, tw, C, n, _p(uv), uv.shape[1], _p(tid), _p(out))
    return out


def texture_bwd(tex, uv, g_out, tri_id=None):
    """Adjoint of ``texture``: (g_tex [th, tw, C], g_uv [n, 2])."""
    tex, uv, g_out = _f64(tex), _f64(uv), _f64(g_out)
    th, tw, C = tex.shape
    n = uv.shape[0]
    assert g_out.shape == (n, C)
    tid = None if tri_id is None else _i32(tri_id)
    g_tex = np.zeros_like(tex)
    g_uv = np.empty((n, 2))
    lib().orc_texture_bwd(_p(tex), th, tw, C, n, _p(uv), uv.shape[1], _p(tid), _p(g_out), _p(g_tex), _p(g_uv))
    return g_tex, g_uv


# ------------------------------------------------------- whole scene (views)
def _view_slices(scene, i):
    vw = scene.view(i)
    vs = scene.v[vw["v_off"]: vw["v_off"] + vw["n_v"]]
    ts = scene.tri[vw["t_off"]: vw["t_off"] + vw["n_t"]]
    ats = scene.attr[vw["a_off"]: vw["a_off"] + vw["n_v"]]
    return vw, vs, ts, ats


def _each_view(fn, views, threads):
    """fn(i) for every view, in view order; with threads > 1 the views run on
    a pool of threads (the C calls release the interpreter lock).  The results
    come back in view order, so whatever is summed from them is summed in the
    same order for any thread count."""
    if threads <= 1:
        for i in views:
            yield fn(i)
        return
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        yield from ex.map(fn, views)


def forward(scene, views=None, threads=1):
    """Per-pixel outputs over all views, packed like the GPU buffers.

    Returns dict: tri_id i32 [n_px], depth f64 [n_px], bary f64 [n_px,3],
    interp f64 [n_px, C_out], image f64 [n_px, C_e] (interp + optional mask),
    backface f64 [n_px] (1 where the visible triangle shows its back side).
    """
    n_px = scene.n_px
    out = dict(tri_id=np.full(n_px, -1, np.int32), depth=np.zeros(n_px), bary=np.zeros((n_px, 3)),
               interp=np.zeros((n_px, scene.C_out)), image=np.zeros((n_px, scene.C_e)), backface=np.zeros(n_px))

    def one(i):
        vw, vs, ts, ats = _view_slices(scene, i)
        H, W, o = vw["H"], vw["W"], vw["px_off"]
        tid = rasterize(vs, ts, H, W)
        d, b, _ = resolve(vs, ts, H, W, tid)
        it = interpolate(ats, vs, ts, H, W, tid, scene.append_z)
        sl = slice(o, o + H * W)
        out["tri_id"][sl] = tid
        out["depth"][sl] = d
        out["bary"][sl] = b
        out["interp"][sl] = it
        out["backface"][sl] = backface(vs, ts, H, W, tid)
        out["image"][sl, :scene.C_out] = it
        if scene.mask_channel:
            out["image"][sl, scene.C_out] = (tid >= 0).astype(np.float64)

    for _ in _each_view(one, range(scene.n_views) if views is None else views, threads):
        pass
    return out


def backward(scene, fwd, g_img, flags=0, edge=True, interp=True, views=None, threads=1):
    """Fused backward over all views: g_v [sum V_view, 3], g_attr [sum V_attr, C_a].

    ``g_img`` is dL/d(image) [n_px, C_e]; its first C_out channels are also
    dL/d(interpolated attributes).  Per-view sums are added in view order.
    """
    g_img = np.asarray(g_img, np.float64)
    g_v = np.zeros((scene.v.shape[0], 3))
    g_attr = np.zeros((scene.attr.shape[0], scene.C_a))

    def one(i):
        vw, vs, ts, ats = _view_slices(scene, i)
        H, W, o = vw["H"], vw["W"], vw["px_off"]
        sl = slice(o, o + H * W)
        gv = np.zeros((vw["n_v"], 3))
        ga = np.zeros((vw["n_v"], scene.C_a))
        tid = fwd["tri_id"][sl]
        if edge:
            edge_grad(vs, ts, H, W, tid, fwd["image"][sl], g_img[sl], flags=flags, g_v=gv)
        if interp:
            interpolate_bwd(ats, vs, ts, H, W, tid, np.ascontiguousarray(g_img[sl, :scene.C_out]),
                            scene.append_z, g_attr=ga, g_v=gv)
        return vw, gv, ga

    for vw, gv, ga in _each_view(one, range(scene.n_views) if views is None else views, threads):
        g_v[vw["v_off"]: vw["v_off"] + vw["n_v"]] += gv
        g_attr[vw["a_off"]: vw["a_off"] + vw["n_v"]] += ga
    return g_v, g_attr


def jvp(scene, fwd, dv, dattr=None, flags=0, edge=True, interp=True, views=None):
    """Forward-mode image tangent over all views, [n_px, C_e]: the
    interpolated channels' tangent at the fixed index image (first C_out
    channels; the mask channel has none) plus the micro-edge term over every
    channel of the image.  dv [sum V_view, 3] screen-vertex tangent, dattr
    [sum V_attr, C_a] attribute tangent (optional)."""
    dv = np.asarray(dv, np.float64)
    dimg = np.zeros((scene.n_px, scene.C_e))
    for i in (range(scene.n_views) if views is None else views):
        vw, vs, ts, ats = _view_slices(scene, i)
        H, W, o = vw["H"], vw["W"], vw["px_off"]
        sl = slice(o, o + H * W)
        tid = fwd["tri_id"][sl]
        dvs = dv[vw["v_off"]: vw["v_off"] + vw["n_v"]]
        d = np.zeros((H * W, scene.C_e))
        if interp:
            da = None if dattr is None else np.asarray(dattr, np.float64)[vw["a_off"]: vw["a_off"] + vw["n_v"]]
            d[:, :scene.C_out] = interpolate_jvp(ats, vs, ts, H, W, tid, dvs, da, scene.append_z)
        if edge:
            edge_jvp(vs, ts, H, W, tid, fwd["image"][sl], dvs, flags=flags, dimg=d)
        dimg[sl] = d
    return dimg


def step_view(scene, i, target_value=0.5):
    """Forward + backward of one view with view-local buffers (for timing):
    rasterize, resolve, interpolate, L2 gradient against a constant target,
    edge term and interpolation adjoint.  Returns the view's pixel count."""
    vw, vs, ts, ats = _view_slices(scene, i)
    H, W = vw["H"], vw["W"]
    tid = rasterize(vs, ts, H, W)
    resolve(vs, ts, H, W, tid)
    it = interpolate(ats, vs, ts, H, W, tid, scene.append_z)
    img = it
    if scene.mask_channel:
        img = np.concatenate([it, (tid >= 0).astype(np.float64)[:, None]], 1)
    g = 2.0 * (img - target_value)
    gv = np.zeros((vw["n_v"], 3))
    ga = np.zeros((vw["n_v"], scene.C_a))
    edge_grad(vs, ts, H, W, tid, img, g, g_v=gv)
    interpolate_bwd(ats, vs, ts, H, W, tid, np.ascontiguousarray(g[:, :scene.C_out]), scene.append_z,
                    g_attr=ga, g_v=gv)
    return H * W


# ------------------------------------------------ vertex transform (numpy)
# Supplement, "Implementation detail": the vertex transform module takes the
# vertices to the camera frame and projects them onto the image plane; its
# backward pass is the derivative of that map.  Camera: rows of R are the
# camera axes in world coordinates (x right, y down, z forward), C the centre,
# f the focal length and (cx, cy) the principal point in pixels.  View i maps
# world rows w_off[i] .. w_off[i] + n_v to screen rows v_off .. v_off + n_v.
def transform(v_world, R, C, f, cx, cy, w_off, views):
    """Screen vertices (x_px, y_px, z) [sum n_v, 3], binary64."""
    V = np.asarray(views, np.int64)
    vw = np.asarray(v_world, np.float64)
    out = np.zeros((max([int(r[0] + r[4]) for r in V] + [0]), 3))
    for i, r in enumerate(V):
        v_off, n_v = int(r[0]), int(r[4])
        pw = vw[int(w_off[i]): int(w_off[i]) + n_v]
        pc = (pw - np.asarray(C[i], np.float64)) @ np.asarray(R[i], np.float64).T  # camera frame
        z = pc[:, 2]
        out[v_off: v_off + n_v, 0] = f[i] * pc[:, 0] / z + cx[i]
        out[v_off: v_off + n_v, 1] = f[i] * pc[:, 1] / z + cy[i]
        out[v_off: v_off + n_v, 2] = z
    return out


def transform32(v_world, R, C, f, cx, cy, w_off, views):
    """The same map in binary32, one rounding per operation in the order the
    library documents for its transform (camera parameters rounded to
    binary32 first): d = p_world - C, p_cam,r = (R_r0 d_0 + R_r1 d_1) + R_r2 d_2,
    x = (f p_x) / p_z + cx, y = (f p_y) / p_z + cy, z = p_z.  Snapping the
    screen vertices to 1/256 px is an integer decision taken on these values,
    so a chain that feeds the rasterizer from the transform compares its
    index image against this form.  [sum n_v, 3] float32."""
    V = np.asarray(views, np.int64)
    vw = np.asarray(v_world, np.float32)
    out = np.zeros((max([int(r[0] + r[4]) for r in V] + [0]), 3), np.float32)
    for i, r in enumerate(V):
        v_off, n_v = int(r[0]), int(r[4])
        Ri = np.asarray(R[i], np.float64).astype(np.float32)
        Ci = np.asarray(C[i], np.float64).astype(np.float32)
        fi, cxi, cyi = np.float32(f[i]), np.float32(cx[i]), np.float32(cy[i])
        d = vw[int(w_off[i]): int(w_off[i]) + n_v] - Ci
        pc = [((Ri[k, 0] * d[:, 0]) + (Ri[k, 1] * d[:, 1])) + (Ri[k, 2] * d[:, 2]) for k in range(3)]
        out[v_off: v_off + n_v, 0] = (fi * pc[0]) / pc[2] + cxi
        out[v_off: v_off + n_v, 1] = (fi * pc[1]) / pc[2] + cyi
        out[v_off: v_off + n_v, 2] = pc[2]
    return out


def transform_bwd(v_world, R, C, f, cx, cy, w_off, views, g_screen):
    """dL/d(world vertices) [n_world, 3]: for every view and vertex, the
    transpose of the projection's Jacobian applied to dL/d(screen vertex),
    summed over the views that use the vertex.  binary64."""
    V = np.asarray(views, np.int64)
    vw = np.asarray(v_world, np.float64)
    gs = np.asarray(g_screen, np.float64)
    g = np.zeros_like(vw)
    for i, r in enumerate(V):
        v_off, n_v = int(r[0]), int(r[4])
        Ri = np.asarray(R[i], np.float64)
        pc = (vw[int(w_off[i]): int(w_off[i]) + n_v] - np.asarray(C[i], np.float64)) @ Ri.T
        x, y, z = pc[:, 0], pc[:, 1], pc[:, 2]
        gx, gy, gz = gs[v_off: v_off + n_v, 0], gs[v_off: v_off + n_v, 1], gs[v_off: v_off + n_v, 2]
        # d(screen)/d(camera frame): x_px = f x / z + cx, y_px = f y / z + cy, z_out = z
        g_cam = np.stack([gx * f[i] / z, gy * f[i] / z, gz - gx * f[i] * x / (z * z) - gy * f[i] * y / (z * z)], 1)
        g[int(w_off[i]): int(w_off[i]) + n_v] += g_cam @ Ri  # camera frame = R (world - C)
    return g
