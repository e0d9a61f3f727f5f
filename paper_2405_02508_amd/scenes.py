"""Seeded synthetic inputs: meshes, cameras and screen-space vertex buffers.

This module produces the *inputs* of the rasterize / interpolate / edge-gradient
path and nothing else: it holds none of the method's arithmetic (no coverage,
no depth test, no barycentrics, no gradients).  Both the HIP path and the CPU
oracle consume what it returns, so it is the only code they share.

Meshes are frequency-nu geodesic icospheres (V = 10 nu^2 + 2, T = 20 nu^2),
built from an icosahedron whose faces are subdivided on an integer lattice.
Lattice points are keyed by their integer weights on the icosahedron corners,
so a point shared by two faces gets one index and bit-identical coordinates:
the meshes are watertight by construction.

Screen-space vertices follow the paper's vertex transform (camera frame, then
pinhole projection): v = (x_px, y_px, z) with x, y in pixels, y pointing down,
origin at the image corner, and z the camera-space depth along the principal
axis (supplement, "Implementation detail").

Each ``make_config(k)`` reproduces one of the five workload shapes of the
micro-edge method (a single small view; a 512^2 view of two interpenetrating
displaced spheres; a 64-view head-like mesh; 256 ragged scenes; a 2M-triangle
pair at 2048^2).  ``small=True`` gives reduced versions that a slow CPU
reference finishes in seconds but that still span several tiles and ragged
image edges.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# view-table column order (all int64 on the host side)
VIEW_COLS = ("v_off", "t_off", "a_off", "px_off", "n_v", "n_t", "H", "W")


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
def _icosahedron():
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array(
        [[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
         [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
         [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array(
        [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
         [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
         [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
         [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    return v, f


def icosphere(nu: int):
    """Unit geodesic sphere of frequency ``nu``: (verts f64 [V,3], faces i32 [T,3]).

    Faces are wound counter-clockwise seen from outside.
    """
    nu = int(nu)
    if nu < 1 or nu > 300:
        raise ValueError("nu must be in [1, 300]")
    V0, F0 = _icosahedron()
    ii, jj = np.meshgrid(np.arange(nu + 1), np.arange(nu + 1), indexing="ij")
    m = (ii + jj) <= nu
    ii, jj = ii[m], jj[m]                          # lattice points of one face
    lidx = -np.ones((nu + 1, nu + 1), dtype=np.int64)
    lidx[ii, jj] = np.arange(ii.size)
    P = ii.size
    # weights on the face corners (a, b, c): (nu-i-j, i, j)
    w = np.stack([nu - ii - jj, ii, jj], axis=1)   # [P,3]
    ids = F0[:, None, :].repeat(P, axis=1)          # [20,P,3]
    ws = np.broadcast_to(w[None], (20, P, 3))
    B = nu + 1
    code = np.where(ws > 0, ids * B + ws, 12 * B)   # zero weight -> sentinel
    code = np.sort(code, axis=2).astype(np.int64)
    K = 13 * B
    key = (code[..., 0] * K + code[..., 1]) * K + code[..., 2]
    key = key.reshape(-1)
    ukey, first, inv = np.unique(key, return_index=True, return_inverse=True)
    # canonical position from the canonical (sorted) code of each unique point
    c = code.reshape(-1, 3)[first]
    pos = np.zeros((ukey.size, 3))
    for s in range(3):
        cid = c[:, s] // B
        cw = c[:, s] % B
        ok = cid < 12
        pos[ok] += cw[ok, None] * V0[cid[ok]]
    pos /= np.linalg.norm(pos, axis=1, keepdims=True)
    inv = inv.reshape(20, P)
    # triangles of one face in lattice coordinates
    up_i, up_j = np.meshgrid(np.arange(nu), np.arange(nu), indexing="ij")
    mu = (up_i + up_j) <= nu - 1
    up_i, up_j = up_i[mu], up_j[mu]
    up = np.stack([lidx[up_i, up_j], lidx[up_i + 1, up_j], lidx[up_i, up_j + 1]], 1)
    dn_i, dn_j = np.meshgrid(np.arange(nu), np.arange(nu), indexing="ij")
    md = (dn_i + dn_j) <= nu - 2
    dn_i, dn_j = dn_i[md], dn_j[md]
    dn = np.stack([lidx[dn_i + 1, dn_j], lidx[dn_i + 1, dn_j + 1], lidx[dn_i, dn_j + 1]], 1)
    local = np.concatenate([up, dn], 0)            # [nu^2, 3]
    faces = inv[:, local].reshape(-1, 3)            # [20 nu^2, 3]
    return pos, faces.astype(np.int32)


def random_rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array(
        [[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
         [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
         [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def vertex_normals(verts, faces):
    """Area-weighted unit vertex normals (float64)."""
    a, b, c = (verts[faces[:, k]] for k in range(3))
    fn = np.cross(b - a, c - a)
    n = np.zeros_like(verts)
    for k in range(3):
        np.add.at(n, faces[:, k], fn)
    n /= np.maximum(np.linalg.norm(n, axis=1, keepdims=True), 1e-30)
    return n


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Camera:
    R: np.ndarray        # rows: camera x (right), y (down), z (forward) in world
    C: np.ndarray        # centre in world
    f: float             # focal length in pixels
    cx: float
    cy: float
    H: int
    W: int


def look_at(eye, target, f, H, W, cx=None, cy=None) -> Camera:
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    up = np.array([0.0, 1.0, 0.0])
    if abs(z @ up) > 0.99:
        up = np.array([0.0, 0.0, 1.0])
    y = -(up - (up @ z) * z)
    y /= np.linalg.norm(y)
    x = np.cross(y, z)
    return Camera(np.stack([x, y, z]), eye, float(f),
                  W / 2.0 if cx is None else float(cx),
                  H / 2.0 if cy is None else float(cy), int(H), int(W))


def focal_from_fov(fov_deg, W):
    return (W / 2.0) / math.tan(math.radians(fov_deg) / 2.0)


def fibonacci_sphere(n, radius, center=(0.0, 0.0, 0.0)):
    i = np.arange(n) + 0.5
    y = 1.0 - 2.0 * i / n
    r = np.sqrt(np.maximum(0.0, 1.0 - y * y))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    p = np.stack([r * np.cos(phi), y, r * np.sin(phi)], 1)
    return p * radius + np.asarray(center)


def project(verts_world, cam: Camera) -> np.ndarray:
    """World points -> screen vertices (x_px, y_px, z) as float32 [V,3]."""
    pc = (verts_world - cam.C) @ cam.R.T
    z = pc[:, 2]
    x = cam.f * pc[:, 0] / z + cam.cx
    y = cam.f * pc[:, 1] / z + cam.cy
    return np.stack([x, y, z], 1).astype(np.float32)


# --------------------------------------------------------------------------
# scene container
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Scene:
    name: str
    v: np.ndarray            # f32 [sum V_view, 3] screen vertices, all views
    tri: np.ndarray          # i32 [sum T, 3] view-local vertex indices
    attr: np.ndarray         # f32 [sum V_attr, C_a] vertex attributes
    views: np.ndarray        # i64 [n_views, 8] columns VIEW_COLS
    append_z: bool           # interpolate screen z as an extra channel
    mask_channel: bool       # coverage mask appended to the edge-gradient image
    v_target: np.ndarray | None = None   # perturbed screen vertices for an L2 target
    recompute: bool = False  # workload asks for barycentrics recomputed in backward
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_views(self):
        return int(self.views.shape[0])

    @property
    def n_px(self):
        return int((self.views[:, 6] * self.views[:, 7]).sum())

    @property
    def C_a(self):
        return int(self.attr.shape[1])

    @property
    def C_out(self):
        return self.C_a + int(self.append_z)

    @property
    def C_e(self):
        return self.C_out + int(self.mask_channel)

    def view(self, i):
        return dict(zip(VIEW_COLS, (int(x) for x in self.views[i])))


def _pack(name, per_view, attr_blocks, append_z, mask_channel, recompute=False,
          target_per_view=None):
    """per_view: list of (v_screen f32 [n_v,3], tri i32 [n_t,3], tri_block, attr_block, H, W)
    where views of one mesh share the same tri_block / attr_block index."""
    v_parts, rows = [], []
    tri_offs, attr_offs = {}, {}
    tri_parts, attr_parts = [], []
    t_total = a_total = v_total = px_total = 0
    tris_by_block = {}
    for (vs, tri, tb, ab, H, W) in per_view:
        if tb not in tri_offs:
            tri_offs[tb] = t_total
            tri_parts.append(tri)
            tris_by_block[tb] = tri
            t_total += tri.shape[0]
        if ab not in attr_offs:
            attr_offs[ab] = a_total
            attr_parts.append(attr_blocks[ab])
            a_total += attr_blocks[ab].shape[0]
        rows.append([v_total, tri_offs[tb], attr_offs[ab], px_total,
                     vs.shape[0], tri.shape[0], H, W])
        v_parts.append(vs)
        v_total += vs.shape[0]
        px_total += H * W
    vt = None
    if target_per_view is not None:
        vt = np.ascontiguousarray(np.concatenate(target_per_view, 0), dtype=np.float32)
    return Scene(name, np.ascontiguousarray(np.concatenate(v_parts, 0), dtype=np.float32),
                 np.ascontiguousarray(np.concatenate(tri_parts, 0), dtype=np.int32),
                 np.ascontiguousarray(np.concatenate(attr_parts, 0), dtype=np.float32),
                 np.asarray(rows, dtype=np.int64), append_z, mask_channel, vt, recompute)


def _world(blocks, block_of_view, cams):
    """World-space form of a scene for the vertex transform: world vertices
    (f32, the given blocks stacked), one pinhole camera per view (rows of R are
    the camera axes) and each view's first world row."""
    offs, acc = [], 0
    for b in blocks:
        offs.append(acc)
        acc += b.shape[0]
    return dict(v=np.ascontiguousarray(np.concatenate(blocks, 0), dtype=np.float32),
                R=np.stack([c.R for c in cams]), C=np.stack([c.C for c in cams]),
                f=np.array([c.f for c in cams]), cx=np.array([c.cx for c in cams]),
                cy=np.array([c.cy for c in cams]), w_off=np.array([offs[b] for b in block_of_view], np.int64))


def _displaced_pair(rng, nu, sigma, shift, second=True, nu2=None):
    """One or two radially displaced unit spheres; the copy is shifted along x."""
    vs, fs = icosphere(nu)
    r = 1.0 + sigma * rng.normal(size=vs.shape[0])
    V = vs * r[:, None]
    F = fs.copy()
    if second:
        if nu2 is not None and nu2 != nu:
            vs2, fs2 = icosphere(nu2)
        else:
            vs2, fs2 = vs, fs
        r2 = 1.0 + sigma * rng.normal(size=vs2.shape[0])
        V2 = vs2 * r2[:, None] + np.array([shift, 0.0, 0.0])
        F = np.concatenate([F, fs2 + V.shape[0]], 0)
        V = np.concatenate([V, V2], 0)
    return V, F.astype(np.int32)


def make_config(k: int, small: bool = False) -> Scene:
    """Workload ``k`` in 1..5 (see module docstring); seeded by ``k``."""
    rng = np.random.default_rng(k)
    if k == 1:
        # one icosphere (nu=4: 162 verts, 320 tris), 64x64, fov 45, distance 3
        vs, fs = icosphere(4)
        Rm = random_rotation(rng)
        V = vs @ Rm.T
        H = W = 64
        cam = look_at([0, 0, -3.0], [0, 0, 0], focal_from_fov(45, W), H, W)
        col = rng.uniform(0, 1, size=(V.shape[0], 3))
        vt = V + rng.normal(0, 0.01, size=V.shape)
        return _pack("icosphere-nu4-64px", [(project(V, cam), fs, 0, 0, H, W)],
                     [col.astype(np.float32)], False, False,
                     target_per_view=[project(vt, cam)])
    if k == 2:
        nu = 16 if small else 64
        H = W = 128 if small else 512
        V, F = _displaced_pair(rng, nu, 0.02, 0.3)
        Rm = random_rotation(rng)
        V = V @ Rm.T
        cam = look_at([0, 0, -3.0], [0, 0, 0], focal_from_fov(45, W), H, W)
        col = rng.uniform(0, 1, size=(V.shape[0], 3))
        nrm = vertex_normals(V, F)
        attr = np.concatenate([col, nrm], 1).astype(np.float32)
        vt = V + rng.normal(0, 0.01, size=V.shape)
        return _pack(f"displaced-pair-nu{nu}-{W}px", [(project(V, cam), F, 0, 0, H, W)],
                     [attr], True, True, target_per_view=[project(vt, cam)])
    if k == 3:
        nu = 20 if small else 55
        n_cam = 4 if small else 64
        W, H = (256, 167) if small else (1024, 667)
        f = 2000.0 * W / 1024.0
        vs, fs = icosphere(nu)
        th = np.arccos(np.clip(vs[:, 1], -1, 1))
        ph = np.arctan2(vs[:, 2], vs[:, 0])
        V = vs * np.array([0.09, 0.12, 0.11])
        V = V + vs * (0.004 * np.sin(3 * th) * np.cos(2 * ph))[:, None]
        rgb = rng.uniform(0, 1, size=(V.shape[0], 3))
        region = (vs[:, 1] > 0).astype(int) * 2 + (vs[:, 0] > 0).astype(int)
        seg = np.eye(4)[region]
        attr = np.concatenate([rgb, seg], 1).astype(np.float32)
        eyes = fibonacci_sphere(n_cam, 1.0)
        per, cams = [], []
        for e in eyes:
            cam = look_at(e, [0, 0, 0], f, H, W, cx=W / 2.0, cy=H / 2.0)
            per.append((project(V, cam), fs, 0, 0, H, W))
            cams.append(cam)
        sc = _pack(f"head-nu{nu}-{n_cam}x{W}x{H}", per, [attr], True, False)
        sc.meta["world"] = _world([V], [0] * n_cam, cams)
        return sc
    if k == 4:
        n_scenes = 8 if small else 256
        tmax = 2e4 if small else 2e5
        T_s = np.exp(rng.uniform(np.log(1e3), np.log(tmax), size=n_scenes))
        R_s = rng.integers(128, (384 if small else 1024) + 1, size=n_scenes)
        n_int = max(1, int(round(0.1 * n_scenes)))
        inter = np.zeros(n_scenes, bool)
        inter[rng.choice(n_scenes, n_int, replace=False)] = True
        per, attrs, tgt, blocks, cams = [], [], [], [], []
        for s in range(n_scenes):
            if inter[s]:
                nu = max(5, int(round(math.sqrt(T_s[s] / 40.0))))
                V, F = _displaced_pair(rng, nu, 0.02, 0.3)
            else:
                nu = max(7, int(round(math.sqrt(T_s[s] / 20.0))))
                V, F = _displaced_pair(rng, nu, 0.02, 0.0, second=False)
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            Wd = Hd = int(R_s[s])
            cam = look_at(3.0 * d, [0, 0, 0], focal_from_fov(45, Wd), Hd, Wd)
            attrs.append(rng.uniform(0, 1, size=(V.shape[0], 3)).astype(np.float32))
            vt = V + rng.normal(0, 0.01, size=V.shape)
            per.append((project(V, cam), F, s, s, Hd, Wd))
            tgt.append(project(vt, cam))
            blocks.append(V)
            cams.append(cam)
        sc = _pack(f"batched-{n_scenes}-scenes", per, attrs, False, False, target_per_view=tgt)
        sc.meta["intersecting"] = [int(i) for i in np.nonzero(inter)[0]]
        sc.meta["world"] = _world(blocks, list(range(n_scenes)), cams)
        return sc
    if k == 5:
        nu = 32 if small else 224
        n_cam = 2 if small else 16
        H = W = 512 if small else 2048
        V, F = _displaced_pair(rng, nu, 0.02, 0.3)
        attr = rng.uniform(0, 1, size=(V.shape[0], 8)).astype(np.float32)
        eyes = fibonacci_sphere(n_cam, 3.0, center=(0.15, 0.0, 0.0))
        per, cams = [], []
        for e in eyes:
            cam = look_at(e, [0.15, 0.0, 0.0], focal_from_fov(45, W), H, W)
            per.append((project(V, cam), F, 0, 0, H, W))
            cams.append(cam)
        sc = _pack(f"recompute-pair-nu{nu}-{n_cam}x{W}px", per, [attr], False, False,
                   recompute=True)
        sc.meta["world"] = _world([V], [0] * n_cam, cams)
        return sc
    raise ValueError("config index must be 1..5")


def image_grad(scene: Scene, seed: int, C: int | None = None) -> np.ndarray:
    """Seeded stand-in for dL/dI: f32 [n_px, C] (C defaults to the scene's C_e)."""
    C = scene.C_e if C is None else C
    rng = np.random.default_rng(1000 + seed)
    return rng.standard_normal(size=(scene.n_px, C), dtype=np.float32)


def texture_inputs(scene: Scene, seed: int, size: int = 1024, channels: int = 8, texels_per_pixel: float = 1.0):
    """Seeded stand-ins for a neural texture and per-vertex uv coordinates
    (the paper samples an 8-channel 1024 x 1024 neural texture at
    interpolated uv, rendering 800 x 800 images: about one texel per
    pixel).  uv f32 [rows of scene.attr, 2]: each attribute row takes its
    vertex's screen position in the first view that uses the row, times
    texels_per_pixel / size (a projected texture, smooth on the mesh;
    coordinates outside [0, 1] clamp to the edge); texture f32
    [size, size, channels], N(0, 1)."""
    rng = np.random.default_rng(2000 + seed)
    uv = np.zeros((scene.attr.shape[0], 2), np.float32)
    done = np.zeros(scene.attr.shape[0], bool)
    for i in range(scene.n_views):
        vw = scene.view(i)
        rows = np.arange(vw["a_off"], vw["a_off"] + vw["n_v"])
        todo = ~done[rows]
        if not todo.any():
            continue
        xy = scene.v[vw["v_off"]: vw["v_off"] + vw["n_v"], :2].astype(np.float64)
        uv[rows[todo]] = (xy[todo] * (texels_per_pixel / size)).astype(np.float32)
        done[rows] = True
    tex = rng.standard_normal((size, size, channels), dtype=np.float32)
    return uv, tex


def scattered_triangles(seed: int, n_tris: int, H: int, W: int, size: float) -> Scene:
    """One view of n_tris independent triangles (own vertices each) scattered
    uniformly over an H x W image: each triangle is a random triangle within
    a size x size pixel box, at a random depth in [1, 10], with RGB vertex
    colours.  Consecutive triangles land far apart, so every group of a few
    hundred of them touches thousands of distinct tiles -- the regime where
    the binning passes' per-workgroup tile tables fill up."""
    rng = np.random.default_rng(seed)
    centre = rng.uniform([0, 0], [W, H], size=(n_tris, 2))
    corner = rng.uniform(-size / 2, size / 2, size=(n_tris, 3, 2))
    xy = (centre[:, None, :] + corner).reshape(-1, 2)
    z = np.repeat(rng.uniform(1.0, 10.0, size=n_tris), 3) * (1.0 + 0.01 * rng.uniform(-1, 1, size=3 * n_tris))
    v = np.concatenate([xy, z[:, None]], 1).astype(np.float32)
    tri = np.arange(3 * n_tris, dtype=np.int32).reshape(n_tris, 3)
    col = rng.uniform(0, 1, size=(3 * n_tris, 3)).astype(np.float32)
    return _pack(f"scattered-{n_tris}-{W}x{H}", [(v, tri, 0, 0, H, W)], [col], False, False)
