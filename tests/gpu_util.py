"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
the CPU oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import sys

import numpy as np

import oracle
from paper_2405_02508_amd import mer, scenes


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(x, dev="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def run_gpu(s: scenes.Scene, g_np, tile=(8, 8), per_view=False, store_bary=True, flags=0, bin_cap=0,
            fused=True, small_px=0, big_tiles=0):
    """Forward + backward on the GPU; returns numpy outputs."""
    import torch
    dev = torch.device("cuda")
    v, tri, attr = to_dev(s.v), to_dev(s.tri), to_dev(s.attr)
    n_px = s.n_px
    tid = torch.full((n_px,), -7, dtype=torch.int32, device=dev)
    depth = torch.full((n_px,), -7.0, dtype=torch.float32, device=dev)
    bary = torch.full((n_px, 2), -7.0, dtype=torch.float32, device=dev)
    interp = torch.full((n_px, s.C_out), -7.0, dtype=torch.float32, device=dev)
    g = to_dev(np.asarray(g_np, np.float32))
    g_v = torch.zeros_like(v)
    g_attr = torch.zeros_like(attr)
    status = []
    groups = [[i] for i in range(s.n_views)] if per_view else [list(range(s.n_views))]
    for grp in groups:
        ctx = mer.Context(s.views[grp], device=dev, tile=tile, bin_cap=bin_cap, small_px=small_px,
                          big_tiles=big_tiles)
        ctx.rasterize(v, tri, tid, depth, bary if store_bary else None)
        status.append(ctx.status())
    for grp in groups:
        ctx = mer.Context(s.views[grp], device=dev, tile=tile, bin_cap=bin_cap, small_px=small_px,
                          big_tiles=big_tiles)
        ctx.interpolate(attr, v, tri, tid, interp, bary=bary if store_bary else None, append_z=s.append_z)
    img = interp
    if s.mask_channel:
        img = torch.cat([interp, (tid >= 0).float()[:, None]], 1).contiguous()
    for grp in groups:
        ctx = mer.Context(s.views[grp], device=dev, tile=tile, bin_cap=bin_cap, small_px=small_px,
                          big_tiles=big_tiles)
        if fused:
            ctx.backward(v, tri, tid, attr, img, g, g_attr, g_v, append_z=s.append_z, flags=flags)
        else:
            ctx.edge_grad(v, tri, tid, img, g, g_v, flags=flags)
            g_out = g[:, :s.C_out].contiguous()
            ctx.interpolate_bwd(attr, v, tri, tid, g_out, g_attr, g_v, append_z=s.append_z)
    torch.cuda.synchronize()
    return dict(tri_id=tid.cpu().numpy(), depth=depth.cpu().numpy(), bary=bary.cpu().numpy(),
                interp=interp.cpu().numpy(), g_v=g_v.cpu().numpy(), g_attr=g_attr.cpu().numpy(), status=status)


def run_oracle(s: scenes.Scene, g_np, flags=0):
    f = oracle.forward(s)
    g_v, g_attr = oracle.backward(s, f, g_np, flags=flags)
    f.update(g_v=g_v, g_attr=g_attr)
    return f


def rel_l2(got, want):
    return float(np.linalg.norm(np.asarray(got, np.float64) - want) / max(np.linalg.norm(want), 1e-30))


def compare(got, ref, bary=True, tol=1e-5, grads=True):
    """Parity: bit-exact tri_id; per-pixel values within tol * max(1, |ref|);
    gradients within tol relative L2 per tensor."""
    assert np.array_equal(got["tri_id"], ref["tri_id"]), \
        f"tri_id differs at {int((got['tri_id'] != ref['tri_id']).sum())} pixels"
    cov = ref["tri_id"] >= 0
    np.testing.assert_array_less(np.abs(got["depth"] - ref["depth"]), tol * np.maximum(1, np.abs(ref["depth"])) + 1e-30)
    if bary:
        rb = ref["bary"][:, :2]
        assert np.all(np.abs(got["bary"] - rb) <= tol * np.maximum(1, np.abs(rb)))
        assert np.all(got["bary"][~cov] == 0)
    np.testing.assert_array_less(np.abs(got["interp"] - ref["interp"]),
                                 tol * np.maximum(1, np.abs(ref["interp"])) + 1e-30)
    errs = {}
    if grads:
        for k in ("g_v", "g_attr"):
            errs[k] = rel_l2(got[k], ref[k])
            assert errs[k] <= tol, f"{k} relative L2 error {errs[k]:.3e} > {tol}"
    return errs
