"""GPU parity of the forward-mode image tangent (mer_jvp) against the CPU
oracle, on the seeded scenes, plus its transpose identity with the GPU
backward.  The oracle computes in binary64; the kernel in binary32.

Tolerance: relative L2 error per tangent image <= 1e-5 (the gradient metric
of the backward), and every element within 1e-4 of the image's largest
magnitude.  Per element the kernel's value is a short sum of binary32
products (a few dozen roundings, about 1e-6 relative each), but a pixel's
interior term is a difference of nearly equal products on thin triangles,
so single elements are held to the image's scale rather than their own."""
import functools

import numpy as np
import pytest

import oracle
from paper_2405_02508_amd import mer, scenes
from tests.gpu_util import rel_l2, say, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOL_MAX = 1e-4


@functools.lru_cache(maxsize=None)
def small(k):
    return scenes.make_config(k, small=True)


@functools.lru_cache(maxsize=None)
def full(k):
    return scenes.make_config(k)


def tangents(s, seed):
    rng = np.random.default_rng(seed)
    dv = rng.standard_normal((s.v.shape[0], 3)).astype(np.float32)
    dv[:, 2] *= 0.01 * s.v[:, 2]                       # depth moves of about 1 %
    dattr = rng.standard_normal(s.attr.shape).astype(np.float32)
    return dv, dattr


def gpu_forward(ctx, s, v, tri, attr):
    """tri_id and the image (interpolated channels, then the mask if any)."""
    import torch
    dev = v.device
    n = s.n_px
    tid = torch.empty(n, dtype=torch.int32, device=dev)
    img = torch.zeros(n, s.C_e, dtype=torch.float32, device=dev)
    interp = torch.empty(n, s.C_out, dtype=torch.float32, device=dev)
    ctx.rasterize(v, tri, tid, None, None)
    ctx.interpolate(attr, v, tri, tid, interp, bary=None, append_z=s.append_z)
    img[:, :s.C_out].copy_(interp)
    if s.mask_channel:
        img[:, s.C_out].copy_(tid >= 0)
    return tid, img


def gpu_jvp(s, dv_np, dattr_np, flags=0, tile=(8, 8), use_dv=True, use_dattr=True, tune=None):
    import torch
    dev = torch.device("cuda")
    kw = dict(tile=tile) if tune is None else dict(tile=tune["tile"], small_px=tune["small_px"],
                                                    bin_cap=tune["bin_cap"], big_tiles=tune.get("big_tiles", 0))
    ctx = mer.Context(s.views, device=dev, **kw)
    v, tri, attr = to_dev(s.v), to_dev(s.tri), to_dev(s.attr)
    tid, img = gpu_forward(ctx, s, v, tri, attr)
    dimg = torch.full((s.n_px, s.C_e), -7.0, dtype=torch.float32, device=dev)
    dv = to_dev(dv_np) if use_dv else None
    da = to_dev(dattr_np) if use_dattr else None
    ctx.jvp(v, tri, tid, attr, img, dv, dimg, dattr=da, append_z=s.append_z, flags=flags)
    torch.cuda.synchronize()
    return dict(ctx=ctx, v=v, tri=tri, attr=attr, tid=tid, img=img, dimg=dimg)


def check(got, want, what):
    err = rel_l2(got, want)
    mx = float(np.abs(np.asarray(got, np.float64) - want).max()) if want.size else 0.0
    scale = float(np.abs(want).max()) if want.size else 0.0
    say(f"[jvp] {what}: rel L2 {err:.2e}, max |err| {mx:.2e} of max |ref| {scale:.2e}")
    assert err <= TOL, f"{what}: relative L2 error {err:.3e} > {TOL}"
    assert mx <= TOL_MAX * max(scale, 1e-30), f"{what}: max error {mx:.3e} > {TOL_MAX} x {scale:.3e}"


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("flags", [0, mer.NO_INTERSECT])
def test_jvp_matches_oracle(k, flags):
    s = small(k)
    say(f"[jvp] config {k} (small) {s.name}: {s.n_views} views, {s.n_px} px, flags {flags}")
    dv, da = tangents(s, 70 + k)
    got = gpu_jvp(s, dv, da, flags=flags)
    f = oracle.forward(s)
    assert np.array_equal(got["tid"].cpu().numpy(), f["tri_id"])
    ref = oracle.jvp(s, f, dv, da, flags=flags)
    check(got["dimg"].cpu().numpy(), ref, f"config {k} flags {flags}")


@pytest.mark.parametrize("k", [2, 4])
@pytest.mark.parametrize("part", ["edge", "interp", "dattr-only"])
def test_jvp_parts_match_oracle(k, part):
    s = small(k)
    say(f"[jvp] config {k} (small) part {part}")
    dv, da = tangents(s, 80 + k)
    f = oracle.forward(s)
    if part == "edge":
        got = gpu_jvp(s, dv, da, flags=mer.SKIP_INTERP)
        ref = oracle.jvp(s, f, dv, None, interp=False)
    elif part == "interp":
        got = gpu_jvp(s, dv, da, flags=mer.SKIP_EDGE)
        ref = oracle.jvp(s, f, dv, da, edge=False)
    else:
        got = gpu_jvp(s, dv, da, use_dv=False)
        ref = oracle.jvp(s, f, np.zeros_like(dv), da, edge=False)
    check(got["dimg"].cpu().numpy(), ref, f"config {k} {part}")


@pytest.mark.parametrize("k", [1, 2, 4, 5])
def test_jvp_is_the_transpose_of_the_gpu_backward(k):
    """sum g . J(dv, dattr) = dL/dv . dv + dL/dattr . dattr, both sides from
    the GPU (binary32 sums over the whole image)."""
    import torch
    s = small(k)
    dv, da = tangents(s, 90 + k)
    got = gpu_jvp(s, dv, da)
    g = torch.from_numpy(np.random.default_rng(k).standard_normal((s.n_px, s.C_e), dtype=np.float32)).cuda()
    g_v = torch.zeros_like(got["v"])
    g_attr = torch.zeros_like(got["attr"])
    got["ctx"].backward(got["v"], got["tri"], got["tid"], got["attr"], got["img"], g, g_attr, g_v,
                        append_z=s.append_z)
    torch.cuda.synchronize()
    lhs = float((g.double() * got["dimg"].double()).sum())
    rhs = float((g_v.double() * to_dev(dv).double()).sum() + (g_attr.double() * to_dev(da).double()).sum())
    say(f"[jvp] config {k}: <g, J t> = {lhs:.6e}, <J^T g, t> = {rhs:.6e}")
    assert abs(lhs - rhs) <= 1e-4 * max(abs(rhs), 1e-30)


def test_jvp_zero_tangent_is_zero_and_background_is_written():
    s = small(1)
    dv, da = tangents(s, 1)
    got = gpu_jvp(s, np.zeros_like(dv), np.zeros_like(da))
    assert float(got["dimg"].abs().max()) == 0.0   # every pixel written, all zero


@pytest.mark.parametrize("k", [3, 4, 5])
def test_jvp_fullsize_views(k):
    """Full workload size in the batched plan bench.py uses (autotuned);
    the oracle recomputes whole views of it."""
    from paper_2405_02508_amd import autotune
    s = full(k)
    say(f"[jvp] full config {k} {s.name}: {s.n_views} views, {s.n_px} px")
    dv, da = tangents(s, 100 + k)
    tune = autotune.tune(s.views, to_dev(s.v), to_dev(s.tri))
    got = gpu_jvp(s, dv, da, tune=tune)
    dimg = got["dimg"].cpu().numpy()
    tid = got["tid"].cpu().numpy()
    views = {3: [0, 63], 4: [0, 255] + list(s.meta.get("intersecting", [])[:2]), 5: [0]}[k]
    f = oracle.forward(s, views=views)
    ref = oracle.jvp(s, f, dv, da, views=views)
    for i in views:
        vw = s.view(i)
        sl = slice(vw["px_off"], vw["px_off"] + vw["H"] * vw["W"])
        assert np.array_equal(tid[sl], f["tri_id"][sl])
        check(dimg[sl], ref[sl], f"full config {k} view {i}")
