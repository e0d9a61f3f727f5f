"""Thin Python binding of ``libmer.so`` (include/mer.h) -- argument marshalling only.

Every step of the path runs in the HIP kernels behind the C ABI; this module
only checks tensor dtypes/devices, passes ``data_ptr()`` and the current
stream, and turns error codes into exceptions.  If the library has not been
built it raises: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmer.so")

NO_INTERSECT = 1
SKIP_EDGE = 2
SKIP_INTERP = 4

SYMBOLS = ("mer_plan_init", "mer_transform", "mer_transform_bwd", "mer_rasterize", "mer_rasterize_interpolate",
           "mer_interpolate", "mer_backface", "mer_edge_grad", "mer_interpolate_bwd", "mer_backward_fused",
           "mer_backward_l2", "mer_backward_l2_noalloc", "mer_jvp", "mer_texture", "mer_texture_bwd", "mer_status",
           "mer_strerror", "mer_version")


class View(ctypes.Structure):
    _fields_ = [("v_off", ctypes.c_int64), ("t_off", ctypes.c_int64), ("a_off", ctypes.c_int64),
                ("px_off", ctypes.c_int64), ("n_v", ctypes.c_int32), ("n_t", ctypes.c_int32),
                ("H", ctypes.c_int32), ("W", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("bin_cap", ctypes.c_int64),
                ("small_px", ctypes.c_int32), ("big_tiles", ctypes.c_int32)]


class Plan(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int32), ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("small_px", ctypes.c_int32), ("total_tris", ctypes.c_int64), ("total_tiles", ctypes.c_int64),
                ("total_px", ctypes.c_int64), ("bin_cap", ctypes.c_int64), ("px_begin", ctypes.c_int64),
                ("ws_bytes", ctypes.c_int64),
                ("off_viewtab", ctypes.c_int64), ("off_rec", ctypes.c_int64), ("off_bbox", ctypes.c_int64),
                ("off_count", ctypes.c_int64), ("off_offs", ctypes.c_int64), ("off_part", ctypes.c_int64),
                ("off_bins", ctypes.c_int64), ("off_status", ctypes.c_int64), ("off_key", ctypes.c_int64),
                ("n_part", ctypes.c_int64), ("total_btiles", ctypes.c_int64), ("off_bviewtab", ctypes.c_int64),
                ("total_v", ctypes.c_int64), ("off_vbase", ctypes.c_int64), ("off_bloss", ctypes.c_int64),
                ("off_big", ctypes.c_int64), ("off_bign", ctypes.c_int64),
                ("big_tiles", ctypes.c_int64), ("n_bingroups", ctypes.c_int64), ("off_bigflat", ctypes.c_int64),
                ("off_bigpart", ctypes.c_int64)]


class Camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("C", ctypes.c_float * 3), ("f", ctypes.c_float), ("cx", ctypes.c_float),
                ("cy", ctypes.c_float), ("reserved", ctypes.c_int32), ("w_off", ctypes.c_int64)]


class MerError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libmer.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MerError(f"{LIB_PATH} is missing: build the HIP library first (__graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, i, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        L.mer_plan_init.argtypes = [ctypes.POINTER(View), i, ctypes.POINTER(Tuning), ctypes.POINTER(Plan)]
        L.mer_rasterize.argtypes = [ctypes.POINTER(Plan), P, P, P, P, P, P, P, P]
        L.mer_rasterize_interpolate.argtypes = [ctypes.POINTER(Plan), P, P, P, P, P, P, P, i, i, P, P, P]
        L.mer_interpolate.argtypes = [ctypes.POINTER(Plan), P, P, i, P, P, P, P, i, P, P]
        L.mer_backface.argtypes = [ctypes.POINTER(Plan), P, P, P, P, P, P]
        L.mer_transform.argtypes = [ctypes.POINTER(Plan), P, P, P, P, P, P]
        L.mer_transform_bwd.argtypes = [ctypes.POINTER(Plan), P, P, P, P, P, P, P]
        L.mer_edge_grad.argtypes = [ctypes.POINTER(Plan), P, P, P, P, P, P, i, i, P, P, P]
        L.mer_interpolate_bwd.argtypes = [ctypes.POINTER(Plan), P, P, i, P, P, P, i, P, i, P, P, P, P]
        L.mer_backward_fused.argtypes = [ctypes.POINTER(Plan), P, P, P, P, P, i, i, P, P, i, i, P, P, P, P]
        L.mer_backward_l2.argtypes = [ctypes.POINTER(Plan), P, P, P, P, P, i, i, P, P, ctypes.c_float, i, i, P, P,
                                      P, P, P]
        L.mer_backward_l2_noalloc.argtypes = [ctypes.POINTER(Plan), P, P, P, P, P, i, i, P, P, ctypes.c_float, i, i, P,
                                              P, P, P]
        L.mer_jvp.argtypes = [ctypes.POINTER(Plan), P, P, P, P, P, P, i, i, P, i, P, i, P, P, P]
        L.mer_texture.argtypes = [ctypes.POINTER(Plan), P, P, P, i, P, i, i, i, P, P]
        L.mer_texture_bwd.argtypes = [ctypes.POINTER(Plan), P, P, P, i, P, i, i, i, P, P, P, P, P]
        L.mer_status.argtypes = [ctypes.POINTER(Plan), P, P, ctypes.POINTER(i64)]
        L.mer_strerror.argtypes = [i]
        L.mer_strerror.restype = ctypes.c_char_p
        L.mer_version.restype = i
        for name in SYMBOLS:
            getattr(L, name).restype = getattr(L, name).restype or i
        L.mer_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise MerError(f"mer error {rc}: {lib().mer_strerror(rc).decode()}")


def views_struct(views_i64: np.ndarray):
    """int64 [n, 8] table (v_off, t_off, a_off, px_off, n_v, n_t, H, W) -> ctypes array of View."""
    views_i64 = np.asarray(views_i64, np.int64)
    arr = (View * views_i64.shape[0])()
    for i, r in enumerate(views_i64):
        arr[i] = View(*[int(x) for x in r])
    return arr


def plan_init(views_i64, tile=(8, 8), bin_cap=0, small_px=0, big_tiles=0) -> Plan:
    vs = views_struct(views_i64)
    tun = Tuning(int(tile[0]), int(tile[1]), int(bin_cap), int(small_px), int(big_tiles))
    P = Plan()
    _check(lib().mer_plan_init(vs, len(vs), ctypes.byref(tun), ctypes.byref(P)))
    return P


# ------------------------------------------------------------------ torch side
def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, name):
    import torch
    if t is None:
        raise MerError(f"{name} is required")
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise MerError(f"{name} must be a contiguous {dtype} CUDA tensor (got {t.dtype}, {t.device})")
    return t


class Context:
    """Plan + device view table + workspace for one batch of views.

    Owns nothing but torch tensors; every method is one C-ABI call on the
    current torch stream.
    """

    def __init__(self, views_i64, device="cuda", tile=(8, 8), bin_cap=0, small_px=0, big_tiles=0):
        import torch
        self.views_i64 = np.asarray(views_i64, np.int64)
        self.plan = plan_init(self.views_i64, tile, bin_cap, small_px, big_tiles)
        raw = bytes(views_struct(self.views_i64))
        self.views_dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)
        self.ws = torch.empty(int(self.plan.ws_bytes), dtype=torch.uint8, device=device)
        self.n_px = int(self.plan.total_px)
        self.tile = tuple(tile)
        V = self.views_i64
        self.need_v = int((V[:, 0] + V[:, 4]).max())
        self.need_t = int((V[:, 1] + V[:, 5]).max())
        self.need_a = int((V[:, 2] + V[:, 4]).max())
        self.n_views = int(V.shape[0])

    def _rows(self, t, n, name, cols=None):
        if t is None:
            return
        if t.shape[0] < n or (cols is not None and (t.dim() != 2 or t.shape[1] != cols)):
            raise MerError(f"{name} has shape {tuple(t.shape)}; the view table needs {n} rows"
                           + (f" x {cols}" if cols else ""))

    def _geom(self, v, tri, attr=None):
        import torch
        _need(v, torch.float32, "v")
        _need(tri, torch.int32, "tri")
        if attr is not None:
            _need(attr, torch.float32, "attr")
        self._rows(v, self.need_v, "v", 3)
        self._rows(tri, self.need_t, "tri", 3)
        self._rows(attr, self.need_a, "attr")

    def _px(self, t, name, cols=None):
        if t is not None:
            if t.shape[0] < self.n_px or (cols is not None and (t.dim() != 2 or t.shape[1] != cols)):
                raise MerError(f"{name} has shape {tuple(t.shape)}; needs {self.n_px} pixel rows"
                               + (f" x {cols}" if cols else ""))

    # forward --------------------------------------------------------------
    def rasterize(self, v, tri, tri_id, depth=None, bary=None):
        import torch
        _need(v, torch.float32, "v")
        _need(tri, torch.int32, "tri")
        _need(tri_id, torch.int32, "tri_id")
        if depth is not None:
            _need(depth, torch.float32, "depth")
        if bary is not None:
            _need(bary, torch.float32, "bary")
        self._geom(v, tri)
        self._px(tri_id, "tri_id")
        self._px(depth, "depth")
        self._px(bary, "bary", 2)
        _check(lib().mer_rasterize(ctypes.byref(self.plan), _ptr(self.views_dev), _ptr(v), _ptr(tri), _ptr(tri_id),
                                   _ptr(depth), _ptr(bary), _ptr(self.ws), _stream()))

    def interpolate(self, attr, v, tri, tri_id, out, bary=None, append_z=False):
        import torch
        _need(attr, torch.float32, "attr")
        _need(out, torch.float32, "out")
        _need(tri_id, torch.int32, "tri_id")
        self._geom(v, tri, attr)
        self._px(tri_id, "tri_id")
        self._px(out, "out", int(attr.shape[1]) + int(bool(append_z)))
        if bary is not None:
            _need(bary, torch.float32, "bary")
            self._px(bary, "bary", 2)
        _check(lib().mer_interpolate(ctypes.byref(self.plan), _ptr(self.views_dev), _ptr(attr), int(attr.shape[1]),
                                     _ptr(v), _ptr(tri), _ptr(tri_id), _ptr(bary), int(bool(append_z)), _ptr(out),
                                     _stream()))

    def rasterize_interpolate(self, v, tri, tri_id, attr, out, depth=None, bary=None, append_z=False):
        """rasterize + interpolate in one pass (out bit-identical to the two calls)."""
        import torch
        _need(v, torch.float32, "v")
        _need(tri, torch.int32, "tri")
        _need(tri_id, torch.int32, "tri_id")
        _need(attr, torch.float32, "attr")
        _need(out, torch.float32, "out")
        if depth is not None:
            _need(depth, torch.float32, "depth")
        if bary is not None:
            _need(bary, torch.float32, "bary")
        self._geom(v, tri, attr)
        self._px(tri_id, "tri_id")
        self._px(depth, "depth")
        self._px(bary, "bary", 2)
        self._px(out, "out", int(attr.shape[1]) + int(bool(append_z)))
        _check(lib().mer_rasterize_interpolate(ctypes.byref(self.plan), _ptr(self.views_dev), _ptr(v), _ptr(tri),
                                               _ptr(tri_id), _ptr(depth), _ptr(bary), _ptr(attr), int(attr.shape[1]),
                                               int(bool(append_z)), _ptr(out), _ptr(self.ws), _stream()))

    # vertex transform ---------------------------------------------------
    def transform(self, cams, v_world, v_screen):
        """Screen vertices of every view from world vertices (``cams``: Cameras)."""
        import torch
        _need(v_world, torch.float32, "v_world")
        _need(v_screen, torch.float32, "v_screen")
        self._cams(cams, v_world)
        self._rows(v_screen, self.need_v, "v_screen", 3)
        _check(lib().mer_transform(ctypes.byref(self.plan), _ptr(self.views_dev), _ptr(cams.dev), _ptr(v_world),
                                   _ptr(v_screen), _ptr(self.ws), _stream()))

    def transform_bwd(self, cams, v_world, g_screen, g_world):
        """g_world += dL/d(world vertices) from dL/d(screen vertices)."""
        import torch
        _need(v_world, torch.float32, "v_world")
        _need(g_screen, torch.float32, "g_screen")
        _need(g_world, torch.float32, "g_world")
        self._rows(g_world, self._cams(cams, v_world), "g_world", 3)
        self._rows(g_screen, self.need_v, "g_screen", 3)
        _check(lib().mer_transform_bwd(ctypes.byref(self.plan), _ptr(self.views_dev), _ptr(cams.dev),
                                       _ptr(v_world), _ptr(g_screen), _ptr(g_world), _ptr(self.ws), _stream()))

    def _cams(self, cams, v_world):
        """Check the camera table against the views; world rows needed."""
        if cams.n != self.n_views:
            raise MerError(f"{cams.n} cameras for {self.n_views} views")
        need = cams.need_for(self.views_i64)
        self._rows(v_world, need, "v_world", 3)
        return need

    def backface(self, v, tri, tri_id, out):
        """out[p] = 1 where the visible triangle shows its back side, else 0."""
        import torch
        _need(out, torch.float32, "out")
        _need(tri_id, torch.int32, "tri_id")
        self._geom(v, tri)
        self._px(tri_id, "tri_id")
        self._px(out, "out")
        _check(lib().mer_backface(ctypes.byref(self.plan), _ptr(self.views_dev), _ptr(v), _ptr(tri), _ptr(tri_id),
                                  _ptr(out), _stream()))

    def edge_grad(self, v, tri, tri_id, img, g_img, g_v, flags=0):
        import torch
        _need(img, torch.float32, "img")
        _need(g_img, torch.float32, "g_img")
        _need(g_v, torch.float32, "g_v")
        _need(tri_id, torch.int32, "tri_id")
        self._geom(v, tri)
        self._rows(g_v, self.need_v, "g_v", 3)
        self._px(tri_id, "tri_id")
        self._px(img, "img")
        self._px(g_img, "g_img", int(img.shape[1]))
        _check(lib().mer_edge_grad(ctypes.byref(self.plan), _ptr(self.views_dev), _ptr(v), _ptr(tri), _ptr(tri_id),
                                   _ptr(img), _ptr(g_img), int(img.shape[1]), int(flags), _ptr(g_v), _ptr(self.ws),
                                   _stream()))

    def interpolate_bwd(self, attr, v, tri, tri_id, g_out, g_attr=None, g_v=None, append_z=False):
        import torch
        _need(g_out, torch.float32, "g_out")
        _need(attr, torch.float32, "attr")
        _need(tri_id, torch.int32, "tri_id")
        self._geom(v, tri, attr)
        self._px(tri_id, "tri_id")
        self._px(g_out, "g_out")
        if g_attr is not None:
            _need(g_attr, torch.float32, "g_attr")
            self._rows(g_attr, self.need_a, "g_attr", int(attr.shape[1]))
        if g_v is not None:
            _need(g_v, torch.float32, "g_v")
            self._rows(g_v, self.need_v, "g_v", 3)
        _check(lib().mer_interpolate_bwd(ctypes.byref(self.plan), _ptr(self.views_dev), _ptr(attr),
                                         int(attr.shape[1]), _ptr(v), _ptr(tri), _ptr(tri_id), int(bool(append_z)),
                                         _ptr(g_out), int(g_out.shape[1]), _ptr(g_attr), _ptr(g_v), _ptr(self.ws),
                                         _stream()))

    def backward(self, v, tri, tri_id, attr, img, g_img, g_attr, g_v, append_z=False, flags=0):
        import torch
        _need(img, torch.float32, "img")
        _need(g_img, torch.float32, "g_img")
        _need(attr, torch.float32, "attr")
        _need(tri_id, torch.int32, "tri_id")
        self._geom(v, tri, attr)
        self._px(tri_id, "tri_id")
        self._px(img, "img")
        self._px(g_img, "g_img", int(img.shape[1]))
        if g_attr is not None:
            _need(g_attr, torch.float32, "g_attr")
            self._rows(g_attr, self.need_a, "g_attr", int(attr.shape[1]))
        if g_v is not None:
            _need(g_v, torch.float32, "g_v")
            self._rows(g_v, self.need_v, "g_v", 3)
        _check(lib().mer_backward_fused(ctypes.byref(self.plan), _ptr(self.views_dev), _ptr(v), _ptr(tri),
                                        _ptr(tri_id), _ptr(attr), int(attr.shape[1]), int(bool(append_z)), _ptr(img),
                                        _ptr(g_img), int(img.shape[1]), int(flags), _ptr(g_attr), _ptr(g_v),
                                        _ptr(self.ws), _stream()))

    def backward_l2(self, v, tri, tri_id, attr, img, target, g_attr, g_v, weight=1.0, loss=None, append_z=False,
                    flags=0):
        """backward for L = weight * sum (img - target)^2, dL/dimg formed in the
        kernel; ``loss`` (one float, accumulated) receives L when given."""
        import torch
        _need(img, torch.float32, "img")
        _need(target, torch.float32, "target")
        _need(attr, torch.float32, "attr")
        _need(tri_id, torch.int32, "tri_id")
        self._geom(v, tri, attr)
        self._px(tri_id, "tri_id")
        self._px(img, "img")
        self._px(target, "target", int(img.shape[1]))
        if g_attr is not None:
            _need(g_attr, torch.float32, "g_attr")
            self._rows(g_attr, self.need_a, "g_attr", int(attr.shape[1]))
        if g_v is not None:
            _need(g_v, torch.float32, "g_v")
            self._rows(g_v, self.need_v, "g_v", 3)
        if loss is not None:
            _need(loss, torch.float32, "loss")
            if loss.numel() < 1:
                raise MerError("loss needs one float")
        _check(lib().mer_backward_l2(ctypes.byref(self.plan), _ptr(self.views_dev), _ptr(v), _ptr(tri),
                                     _ptr(tri_id), _ptr(attr), int(attr.shape[1]), int(bool(append_z)), _ptr(img),
                                     _ptr(target), float(weight), int(img.shape[1]), int(flags), _ptr(g_attr),
                                     _ptr(g_v), _ptr(loss), _ptr(self.ws), _stream()))

    def backward_l2_noalloc(self, v, tri, tri_id, attr, img, target, g_attr, g_v, weight=1.0, loss=None,
                            append_z=False, flags=0):
        """backward_l2 without the workspace: the call's scratch is the
        library's fixed per-GPU array (calls that overlap on one GPU race)."""
        import torch
        _need(img, torch.float32, "img")
        _need(target, torch.float32, "target")
        _need(attr, torch.float32, "attr")
        _need(tri_id, torch.int32, "tri_id")
        self._geom(v, tri, attr)
        self._px(tri_id, "tri_id")
        self._px(img, "img")
        self._px(target, "target", int(img.shape[1]))
        if g_attr is not None:
            _need(g_attr, torch.float32, "g_attr")
            self._rows(g_attr, self.need_a, "g_attr", int(attr.shape[1]))
        if g_v is not None:
            _need(g_v, torch.float32, "g_v")
            self._rows(g_v, self.need_v, "g_v", 3)
        if loss is not None:
            _need(loss, torch.float32, "loss")
            if loss.numel() < 1:
                raise MerError("loss needs one float")
        _check(lib().mer_backward_l2_noalloc(ctypes.byref(self.plan), _ptr(self.views_dev), _ptr(v), _ptr(tri),
                                             _ptr(tri_id), _ptr(attr), int(attr.shape[1]), int(bool(append_z)),
                                             _ptr(img), _ptr(target), float(weight), int(img.shape[1]), int(flags),
                                             _ptr(g_attr), _ptr(g_v), _ptr(loss), _stream()))

    def jvp(self, v, tri, tri_id, attr, img, dv, dimg, dattr=None, append_z=False, flags=0):
        """Forward mode: dimg [px, C_e] = image tangent for the screen-vertex
        tangent ``dv`` [sum n_v, 3] (or None) and attribute tangent ``dattr``
        (like attr, or None): the interpolated channels' derivative at the
        fixed index image plus the micro-edge term on every channel of
        ``img``.  ``attr`` may be None with MER_SKIP_INTERP."""
        import torch
        _need(tri_id, torch.int32, "tri_id")
        _need(dimg, torch.float32, "dimg")
        self._px(tri_id, "tri_id")
        self._px(dimg, "dimg")
        C_e = int(dimg.shape[1])
        C_a = 0
        if attr is not None:
            _need(attr, torch.float32, "attr")
            self._geom(v, tri, attr)
            C_a = int(attr.shape[1])
        else:
            self._geom(v, tri, None)
        if img is not None:
            _need(img, torch.float32, "img")
            self._px(img, "img", C_e)
        if dv is not None:
            _need(dv, torch.float32, "dv")
            self._rows(dv, self.need_v, "dv", 3)
        if dattr is not None:
            _need(dattr, torch.float32, "dattr")
            self._rows(dattr, self.need_a, "dattr", C_a)
        _check(lib().mer_jvp(ctypes.byref(self.plan), _ptr(self.views_dev), _ptr(v), _ptr(tri), _ptr(tri_id),
                             _ptr(attr), _ptr(dattr), C_a, int(bool(append_z)), _ptr(img), C_e, _ptr(dv),
                             int(flags), _ptr(dimg), _ptr(self.ws), _stream()))

    def _tex_args(self, tri_id, uv, tex):
        import torch
        if tri_id is not None:
            _need(tri_id, torch.int32, "tri_id")
            self._px(tri_id, "tri_id")
        if uv is None or uv.dtype != torch.float32 or not uv.is_cuda or uv.dim() != 2 or uv.shape[1] < 2 \
                or uv.stride(1) != 1:
            raise MerError("uv must be a float32 CUDA tensor [px, >= 2] with unit column stride")
        if uv.shape[0] < self.n_px:
            raise MerError(f"uv has {uv.shape[0]} rows; needs {self.n_px}")
        _need(tex, torch.float32, "tex")
        if tex.dim() != 3:
            raise MerError("tex must be [tex_h, tex_w, C_t]")
        return int(uv.stride(0)), int(tex.shape[0]), int(tex.shape[1]), int(tex.shape[2])

    def texture(self, tri_id, uv, tex, out):
        """out [px, C_t] = bilinear clamp-to-edge samples of tex [th, tw, C_t]
        at uv (the first two columns of a [px, >= 2] tensor, e.g. a slice of
        an interpolated image); 0 where tri_id < 0 (tri_id may be None)."""
        import torch
        ld, th, tw, C = self._tex_args(tri_id, uv, tex)
        _need(out, torch.float32, "out")
        self._px(out, "out", C)
        _check(lib().mer_texture(ctypes.byref(self.plan), _ptr(self.views_dev), _ptr(tri_id), _ptr(uv), ld,
                                 _ptr(tex), th, tw, C, _ptr(out), _stream()))

    def texture_bwd(self, tri_id, uv, tex, g_out, g_tex=None, g_uv=None):
        """g_tex [th, tw, C_t] += adjoint to the texture; g_uv [px, 2]
        (written) = gradient to uv.  Either may be None."""
        import torch
        ld, th, tw, C = self._tex_args(tri_id, uv, tex)
        _need(g_out, torch.float32, "g_out")
        self._px(g_out, "g_out", C)
        if g_tex is not None:
            _need(g_tex, torch.float32, "g_tex")
            if tuple(g_tex.shape) != (th, tw, C):
                raise MerError("g_tex must have the texture's shape")
        if g_uv is not None:
            _need(g_uv, torch.float32, "g_uv")
            self._px(g_uv, "g_uv", 2)
        _check(lib().mer_texture_bwd(ctypes.byref(self.plan), _ptr(self.views_dev), _ptr(tri_id), _ptr(uv), ld,
                                     _ptr(tex), th, tw, C, _ptr(g_out), _ptr(g_tex), _ptr(g_uv), _ptr(self.ws),
                                     _stream()))

    def status(self):
        """Status of the last rasterize on this workspace (waits for the
        stream).  Raises MerError if an integrity count is not zero."""
        out = (ctypes.c_int64 * 6)()
        rc = lib().mer_status(ctypes.byref(self.plan), _ptr(self.ws), _stream(), out)
        st = dict(overflow_tiles=out[0], culled=out[1], entries=out[2], bin_cap=out[3], bad_entries=out[4],
                  unbalanced_tiles=out[5])
        if rc != 0:
            raise MerError(f"mer error {rc}: {lib().mer_strerror(rc).decode()} {st}")
        return st


class Cameras:
    """Device copy of one pinhole camera per view (mer_camera): rows of R are
    the camera axes in world coordinates (x right, y down, z forward), C the
    centre, f the focal length and (cx, cy) the principal point in pixels;
    view i reads world rows w_off[i] .. w_off[i] + n_v - 1."""

    def __init__(self, views_i64, R, C, f, cx, cy, w_off, device="cuda"):
        import torch
        V = np.asarray(views_i64, np.int64)
        n = V.shape[0]
        arr = (Camera * n)()
        R, C = np.asarray(R, np.float64).reshape(n, 9), np.asarray(C, np.float64).reshape(n, 3)
        for i in range(n):
            arr[i].R[:] = [float(x) for x in R[i]]
            arr[i].C[:] = [float(x) for x in C[i]]
            arr[i].f, arr[i].cx, arr[i].cy = float(f[i]), float(cx[i]), float(cy[i])
            arr[i].reserved = 0
            arr[i].w_off = int(w_off[i])
        self.n = n
        self.w_off = np.asarray(w_off, np.int64)
        self.dev = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).to(device)

    def need_for(self, V):
        V = np.asarray(V, np.int64)
        return int(max([int(self.w_off[i] + V[i, 4]) for i in range(V.shape[0])] + [0]))
