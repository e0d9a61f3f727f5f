"""torch.autograd wrappers over the C ABI (argument marshalling only).

The module split follows the paper's implementation (supplement,
"Implementation detail"): rasterization has no backward; interpolation has
one (the smooth term Omega); EdgeGrad is the identity in the forward pass
and computes dL/d(vertex positions) from the micro-edges in its backward
pass.  ``RenderStep`` fuses all three for one call per optimisation step:
its forward rasterizes and interpolates every view, its backward runs the
fused micro-edge + interpolation sweep once.

Screen vertices are per view (rows v_off .. v_off + n_v of ``v``).
``Transform`` (the vertex transform module) makes them from world vertices
and one pinhole camera per view, and its backward reduces the per-view
screen gradients to world space.
"""
from __future__ import annotations

import torch

from . import mer


class Renderer:
    """Plan, workspace and topology for a fixed view table."""

    def __init__(self, views_i64, tri, device="cuda", tile=(8, 8), small_px=0, bin_cap=0,
                 append_z=False, mask_channel=False, store_bary=True, big_tiles=0):
        self.ctx = mer.Context(views_i64, device=device, tile=tile, bin_cap=bin_cap, small_px=small_px,
                               big_tiles=big_tiles)
        self.tri = tri if isinstance(tri, torch.Tensor) else torch.from_numpy(tri).to(device)
        self.n_px = self.ctx.n_px
        self.append_z = bool(append_z)
        self.mask_channel = bool(mask_channel)
        self.store_bary = bool(store_bary)
        self.device = torch.device(device)

    def rasterize(self, v):
        """Index image, depth and (optionally) barycentrics; no gradient."""
        tid = torch.empty(self.n_px, dtype=torch.int32, device=self.device)
        depth = torch.empty(self.n_px, dtype=torch.float32, device=self.device)
        bary = torch.empty(self.n_px, 2, dtype=torch.float32, device=self.device) if self.store_bary else None
        self.ctx.rasterize(v.detach().contiguous(), self.tri, tid, depth, bary)
        return tid, depth, bary


    def backface(self, v, tid):
        """Back-face image [n_px, 1]: 1 where the visible triangle shows its
        back side.  A 0/1 image has no gradient of its own; pass it through
        EdgeGrad (``back_face_image``) so that a loss on it moves the edges."""
        out = torch.empty(self.n_px, 1, dtype=torch.float32, device=self.device)
        self.ctx.backface(v.detach().contiguous(), self.tri, tid, out)
        return out


class Transform(torch.autograd.Function):
    """World vertices -> screen vertices of every view (supplement,
    "Implementation detail", vertex transform module); backward: the
    transposed Jacobian of the projection, summed over the views."""

    @staticmethod
    def forward(ctx, v_world, cams: mer.Cameras, r: Renderer):
        vw = v_world.detach().contiguous()
        v = torch.zeros(r.ctx.need_v, 3, dtype=torch.float32, device=v_world.device)
        r.ctx.transform(cams, vw, v)
        ctx.save_for_backward(vw)
        ctx.cams = cams
        ctx.r = r
        return v

    @staticmethod
    def backward(ctx, g_v):
        (vw,) = ctx.saved_tensors
        g_world = torch.zeros_like(vw)
        ctx.r.ctx.transform_bwd(ctx.cams, vw, g_v.contiguous(), g_world)
        return g_world, None, None


class Interpolate(torch.autograd.Function):
    """out = sum_k b_k attr_k (+ interpolated z); backward: attr and Omega to v."""

    @staticmethod
    def forward(ctx, v, attr, tid, bary, r: Renderer):
        C = attr.shape[1] + int(r.append_z)
        out = torch.empty(r.n_px, C, dtype=torch.float32, device=v.device)
        r.ctx.interpolate(attr.detach().contiguous(), v.detach().contiguous(), r.tri, tid, out, bary=bary,
                          append_z=r.append_z)
        ctx.save_for_backward(v, attr, tid)
        ctx.r = r
        ctx.mark_non_differentiable(tid)
        return out

    @staticmethod
    def backward(ctx, g_out):
        v, attr, tid = ctx.saved_tensors
        r = ctx.r
        g_v = torch.zeros_like(v) if ctx.needs_input_grad[0] else None
        g_attr = torch.zeros_like(attr) if ctx.needs_input_grad[1] else None
        if g_v is not None or g_attr is not None:
            r.ctx.interpolate_bwd(attr.detach().contiguous(), v.detach().contiguous(), r.tri, tid,
                                  g_out.contiguous(), g_attr, g_v, append_z=r.append_z)
        return g_v, g_attr, None, None, None


class EdgeGrad(torch.autograd.Function):
    """Identity on the image; backward adds the micro-edge term to dL/dv and
    passes dL/dimage through unchanged (supplement, "EdgeGrad module")."""

    @staticmethod
    def forward(ctx, img, v, tid, r: Renderer, flags: int = 0):
        ctx.save_for_backward(img, v, tid)
        ctx.r = r
        ctx.flags = flags
        return img.view_as(img)

    @staticmethod
    def backward(ctx, g_img):
        img, v, tid = ctx.saved_tensors
        g_v = None
        if ctx.needs_input_grad[1]:
            g_v = torch.zeros_like(v)
            ctx.r.ctx.edge_grad(v.detach().contiguous(), ctx.r.tri, tid, img.detach().contiguous(),
                                g_img.contiguous(), g_v, flags=ctx.flags)
        return g_img, g_v, None, None, None


class Texture(torch.autograd.Function):
    """Deferred texturing: bilinear clamp-to-edge samples of tex [th, tw, C]
    at per-pixel uv (the first two columns of ``uv``, e.g. an interpolated
    uv attribute); 0 on background.  Backward: to the texture and to uv
    (whose gradient then flows through Interpolate to the uv attribute and,
    through the barycentrics, to the vertices)."""

    @staticmethod
    def forward(ctx, uv, tex, tid, r: Renderer):
        uvc = uv.detach()
        if uvc.stride(1) != 1:
            uvc = uvc.contiguous()
        texc = tex.detach().contiguous()
        out = torch.empty(r.n_px, tex.shape[2], dtype=torch.float32, device=uv.device)
        r.ctx.texture(tid, uvc, texc, out)
        ctx.save_for_backward(uvc, texc, tid)
        ctx.r = r
        ctx.mark_non_differentiable(tid)
        return out

    @staticmethod
    def backward(ctx, g_out):
        uv, tex, tid = ctx.saved_tensors
        g_tex = torch.zeros_like(tex) if ctx.needs_input_grad[1] else None
        g_uv2 = torch.empty(uv.shape[0], 2, dtype=torch.float32, device=uv.device) if ctx.needs_input_grad[0] else None
        if g_tex is not None or g_uv2 is not None:
            ctx.r.ctx.texture_bwd(tid, uv, tex, g_out.contiguous(), g_tex, g_uv2)
        g_uv = None
        if g_uv2 is not None:
            g_uv = torch.zeros(uv.shape, dtype=torch.float32, device=uv.device)
            g_uv[:, :2] = g_uv2
        return g_uv, g_tex, None, None


class RenderStep(torch.autograd.Function):
    """One call per step: image = [interpolated attributes (+ z), (mask)] with
    the EdgeGrad identity folded in; backward = one fused sweep."""

    @staticmethod
    def forward(ctx, v, attr, r: Renderer, flags: int = 0):
        vd, ad = v.detach().contiguous(), attr.detach().contiguous()
        dev = v.device
        tid = torch.empty(r.n_px, dtype=torch.int32, device=dev)
        depth = torch.empty(r.n_px, dtype=torch.float32, device=dev)
        bary = torch.empty(r.n_px, 2, dtype=torch.float32, device=dev) if r.store_bary else None
        C = attr.shape[1] + int(r.append_z)
        C_e = C + int(r.mask_channel)
        img = torch.empty(r.n_px, C_e, dtype=torch.float32, device=dev)
        # one pass: rasterize, resolve and interpolate
        out = img if C_e == C else torch.empty(r.n_px, C, dtype=torch.float32, device=dev)
        r.ctx.rasterize_interpolate(vd, r.tri, tid, ad, out, depth=depth, bary=bary, append_z=r.append_z)
        if C_e != C:
            img[:, :C].copy_(out)
            img[:, C].copy_(tid >= 0)
        ctx.save_for_backward(vd, ad, tid, img)
        ctx.r = r
        ctx.flags = flags
        ctx.mark_non_differentiable(tid, depth)
        return img, tid, depth

    @staticmethod
    def backward(ctx, g_img, _g_tid, _g_depth):
        v, attr, tid, img = ctx.saved_tensors
        r = ctx.r
        g_v = torch.zeros_like(v)
        g_attr = torch.zeros_like(attr)
        r.ctx.backward(v, r.tri, tid, attr, img, g_img.contiguous(), g_attr, g_v, append_z=r.append_z,
                       flags=ctx.flags)
        return (g_v if ctx.needs_input_grad[0] else None, g_attr if ctx.needs_input_grad[1] else None, None, None)


def render(v, attr, r: Renderer, flags: int = 0):
    """Fused forward (image, tri_id, depth); gradients flow to v and attr."""
    return RenderStep.apply(v, attr, r, flags)


def back_face_image(r: Renderer, v, tid, flags: int = 0):
    """The back-face image with the micro-edge gradient attached: the loss
    ||image||^2 (supplement, "Implementation detail", back-face loss) then
    moves the vertices so that fewer back sides show."""
    return EdgeGrad.apply(r.backface(v, tid), v, tid, r, flags)
