"""Independent "truth" helpers for pinning the oracle (test infrastructure).

Nothing here calls the oracle or the GPU library:
  * ``inside_exact`` -- point-in-triangle with exact rational arithmetic.
  * ``render_supersampled`` -- area-coverage image (pixel integral with a box
    filter, Sec. 3 Eq. pixel_color) estimated with n x n stratified samples
    per pixel, binary64, continuous (unsnapped) geometry, z-buffer on the
    interpolated 1/z, perspective-correct attribute interpolation.
  * ``omega_torch`` -- the smooth term written directly as a binary64 torch
    expression of the vertex positions at a fixed triangle-id image, so that
    torch autograd gives its gradient.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def inside_exact(tri_xy, px, py):
    """Strict containment of pixel centre (px+1/2, py+1/2); None if on an edge."""
    P = (Fraction(2 * px + 1, 2), Fraction(2 * py + 1, 2))
    V = [(Fraction(float(x)), Fraction(float(y))) for x, y in tri_xy]

    def orient(a, b, c):
        return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])

    D = orient(V[0], V[1], V[2])
    e = [orient(V[1], V[2], P), orient(V[2], V[0], P), orient(V[0], V[1], P)]
    s = 1 if D > 0 else -1
    e = [s * x for x in e]
    if any(x == 0 for x in e):
        return None
    return all(x > 0 for x in e)


def render_supersampled(v, tri, attr, H, W, n=16):
    """v f64 [V,3] screen (x, y, z); attr f64 [V,C] -> image f64 [H*W, C]."""
    v = np.asarray(v, np.float64)
    attr = np.asarray(attr, np.float64)
    C = attr.shape[1]
    HS, WS = H * n, W * n
    qbuf = np.zeros((HS, WS))
    img = np.zeros((HS, WS, C))
    for t in np.asarray(tri):
        P = v[t]
        if np.any(P[:, 2] <= 0):
            continue
        x0, x1 = P[:, 0].min(), P[:, 0].max()
        y0, y1 = P[:, 1].min(), P[:, 1].max()
        i0 = max(0, int(np.floor(x0 * n - 0.5)))
        i1 = min(WS - 1, int(np.ceil(x1 * n - 0.5)))
        j0 = max(0, int(np.floor(y0 * n - 0.5)))
        j1 = min(HS - 1, int(np.ceil(y1 * n - 0.5)))
        if i1 < i0 or j1 < j0:
            continue
        X, Y = np.meshgrid((np.arange(i0, i1 + 1) + 0.5) / n, (np.arange(j0, j1 + 1) + 0.5) / n)
        (ax, ay), (bx, by), (cx, cy) = P[0, :2], P[1, :2], P[2, :2]
        D = (bx - ax) * (cy - ay) - (cx - ax) * (by - ay)
        if D == 0:
            continue
        b0 = ((cx - bx) * (Y - by) - (cy - by) * (X - bx)) / D
        b1 = ((ax - cx) * (Y - cy) - (ay - cy) * (X - cx)) / D
        b2 = 1.0 - b0 - b1
        ins = (b0 >= 0) & (b1 >= 0) & (b2 >= 0)
        q = b0 / P[0, 2] + b1 / P[1, 2] + b2 / P[2, 2]
        sub = qbuf[j0:j1 + 1, i0:i1 + 1]
        win = ins & (q > sub)
        if not win.any():
            continue
        sub[win] = q[win]
        w0, w1, w2 = b0 / P[0, 2] / q, b1 / P[1, 2] / q, b2 / P[2, 2] / q
        col = w0[..., None] * attr[t[0]] + w1[..., None] * attr[t[1]] + w2[..., None] * attr[t[2]]
        isub = img[j0:j1 + 1, i0:i1 + 1]
        isub[win] = col[win]
    return img.reshape(H, n, W, n, C).mean(axis=(1, 3)).reshape(H * W, C)


def omega_torch(v, tri, attr, H, W, tri_id, g, append_z=False):
    """L = sum g * interp at a fixed index image; returns (dL/dv, dL/dattr) by autograd."""
    import torch

    vt = torch.tensor(np.asarray(v, np.float64), requires_grad=True)
    at = torch.tensor(np.asarray(attr, np.float64), requires_grad=True)
    tid = np.asarray(tri_id)
    pix = np.nonzero(tid >= 0)[0]
    t = torch.tensor(np.asarray(tri)[tid[pix]].astype(np.int64))
    Px = torch.tensor((pix % W) + 0.5, dtype=torch.float64)
    Py = torch.tensor((pix // W) + 0.5, dtype=torch.float64)
    a, b, c = vt[t[:, 0]], vt[t[:, 1]], vt[t[:, 2]]

    def orient(p, q, rx, ry):
        return (q[:, 0] - p[:, 0]) * (ry - p[:, 1]) - (q[:, 1] - p[:, 1]) * (rx - p[:, 0])

    D = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1])
    beta = torch.stack([orient(b, c, Px, Py), orient(c, a, Px, Py), orient(a, b, Px, Py)], 1) / D[:, None]
    z = torch.stack([a[:, 2], b[:, 2], c[:, 2]], 1)
    w = beta / z
    bb = w / w.sum(1, keepdim=True)
    A = at[t]                                          # [n,3,C]
    out = (bb[:, :, None] * A).sum(1)
    if append_z:
        out = torch.cat([out, (bb * z).sum(1, keepdim=True)], 1)
    gt = torch.tensor(np.asarray(g, np.float64)[pix])
    L = (out * gt).sum()
    L.backward()
    return vt.grad.numpy(), at.grad.numpy()


def interp_jvp_torch(v, tri, attr, H, W, tri_id, dv, dattr=None, append_z=False):
    """Forward-mode tangent of the interpolated image at a fixed index image,
    by torch.func.jvp of the continuous binary64 formulas; [H*W, C]."""
    import torch
    from torch.func import jvp

    tid = np.asarray(tri_id)
    pix = np.nonzero(tid >= 0)[0]
    t = torch.tensor(np.asarray(tri)[tid[pix]].astype(np.int64))
    Px = torch.tensor((pix % W) + 0.5, dtype=torch.float64)
    Py = torch.tensor((pix // W) + 0.5, dtype=torch.float64)

    def orient(p, q, rx, ry):
        return (q[:, 0] - p[:, 0]) * (ry - p[:, 1]) - (q[:, 1] - p[:, 1]) * (rx - p[:, 0])

    def interp(vt, at):
        a, b, c = vt[t[:, 0]], vt[t[:, 1]], vt[t[:, 2]]
        D = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1])
        beta = torch.stack([orient(b, c, Px, Py), orient(c, a, Px, Py), orient(a, b, Px, Py)], 1) / D[:, None]
        z = torch.stack([a[:, 2], b[:, 2], c[:, 2]], 1)
        w = beta / z
        bb = w / w.sum(1, keepdim=True)
        out = (bb[:, :, None] * at[t]).sum(1)
        if append_z:
            out = torch.cat([out, (bb * z).sum(1, keepdim=True)], 1)
        return out

    vt = torch.tensor(np.asarray(v, np.float64))
    at = torch.tensor(np.asarray(attr, np.float64))
    dvt = torch.tensor(np.asarray(dv, np.float64))
    dat = torch.zeros_like(at) if dattr is None else torch.tensor(np.asarray(dattr, np.float64))
    _, d = jvp(interp, (vt, at), (dvt, dat))
    out = np.zeros((H * W, d.shape[1]))
    out[pix] = d.numpy()
    return out
