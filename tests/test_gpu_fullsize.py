"""GPU parity at the full workload sizes, in the batched launch configuration
that bench.py times (every view in one plan, autotuned tiles and bin pool).

Every view of every workload is compared with the oracle (the oracle runs
its views on a pool of threads; its per-view sums are added in view order):
the index image bit-exactly, depth, barycentrics and interpolated attributes
element by element, and the vertex and attribute gradients over the whole
tensors -- so the attribute gradient of the workloads whose views share one
mesh (the head mesh's 64 views, the 2M-triangle pair's 16) is checked after
its reduction over all views.  Two call paths:

  * ``calls``: mer_rasterize, mer_interpolate, mer_backward_fused with a
    seeded N(0, 1) dL/d(image);
  * ``step``: the benchmark's own step (bench.Step: mer_rasterize_interpolate
    then mer_backward_l2 forming dL/dI = 2 (I - T) in the kernel) against a
    seeded target image T.

Besides the relative L2 bar, each gradient's largest element error is
reported relative to max(|ref|, 1e-3 * max|ref|)."""
import functools
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2405_02508_amd import scenes
from tests.gpu_util import rel_l2, say, to_dev

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
THREADS = min(16, os.cpu_count() or 1)


@functools.lru_cache(maxsize=1)
def full(k):
    s = scenes.make_config(k)
    return s, oracle.forward(s, threads=THREADS)


def max_elem_err(got, ref):
    ref = np.asarray(ref, np.float64)
    floor = 1e-3 * max(float(np.abs(ref).max()), 1e-30)
    return float((np.abs(np.asarray(got, np.float64) - ref) / np.maximum(np.abs(ref), floor)).max())


def check_forward(s, got, ref):
    bad = got["tri_id"] != ref["tri_id"]
    assert not bad.any(), f"tri_id differs at {int(bad.sum())} pixels"
    d = np.abs(got["depth"] - ref["depth"])
    assert np.all(d <= 1e-5 * np.maximum(1, np.abs(ref["depth"]))), "depth"
    if got.get("bary") is not None:
        rb = ref["bary"][:, :2]
        assert np.all(np.abs(got["bary"] - rb) <= 1e-5 * np.maximum(1, np.abs(rb))), "bary"
    it = ref["interp"]
    assert np.all(np.abs(got["interp"] - it) <= 1e-5 * np.maximum(1, np.abs(it))), "interp"


def check_grads(s, got, rgv, rga, label):
    out = {}
    for name, a, b in (("g_v", got["g_v"], rgv), ("g_attr", got["g_attr"], rga)):
        e = rel_l2(a, b)
        assert e <= 1e-5, f"{label}: {name} rel L2 {e}"
        out[name] = (e, max_elem_err(a, b))
    # per view, screen-vertex gradients (each view owns its rows)
    worst = 0.0
    for i in range(s.n_views):
        vw = s.view(i)
        vs = slice(vw["v_off"], vw["v_off"] + vw["n_v"])
        if np.linalg.norm(rgv[vs]) > 0:
            worst = max(worst, rel_l2(got["g_v"][vs], rgv[vs]))
    assert worst <= 1e-5, f"{label}: worst per-view g_v rel L2 {worst}"
    say(f"[full] {label}: rel L2 / max-element g_v {out['g_v'][0]:.2e} / {out['g_v'][1]:.2e}, "
        f"g_attr {out['g_attr'][0]:.2e} / {out['g_attr'][1]:.2e}, worst view g_v {worst:.2e}")
    return out


def tuned(s):
    from paper_2405_02508_amd import autotune
    tune = autotune.tune(s.views, to_dev(s.v), to_dev(s.tri))  # every candidate's status is checked
    say(f"[full] tuning {tune['tile']} small_px {tune['small_px']} big_tiles {tune.get('big_tiles')} "
        f"cap {tune['bin_cap']}")
    return tune


CASES = [(k, path) for k in (1, 2, 3, 4, 5) for path in ("calls", "step")]


@pytest.mark.parametrize("k,path", CASES)
def test_fullsize(k, path):
    (run_calls if path == "calls" else run_step)(k)


def run_calls(k):
    import torch

    from paper_2405_02508_amd import mer
    s, ref = full(k)
    say(f"[full] calls: config {k} {s.name}: {s.n_views} views, {s.n_px} px")
    tune = tuned(s)
    dev = torch.device("cuda")
    ctx = mer.Context(s.views, device=dev, tile=tune["tile"], small_px=tune["small_px"], bin_cap=tune["bin_cap"],
                      big_tiles=tune.get("big_tiles", 0))
    v, tri, attr = to_dev(s.v), to_dev(s.tri), to_dev(s.attr)
    n = s.n_px
    tid = torch.empty(n, dtype=torch.int32, device=dev)
    depth = torch.empty(n, dtype=torch.float32, device=dev)
    bary = None if s.recompute else torch.empty(n, 2, dtype=torch.float32, device=dev)
    img = torch.empty(n, s.C_e, dtype=torch.float32, device=dev)
    interp = img if s.C_e == s.C_out else torch.empty(n, s.C_out, dtype=torch.float32, device=dev)
    ctx.rasterize(v, tri, tid, depth, bary)
    st = ctx.status()  # raises on a nonzero integrity count
    assert st["overflow_tiles"] == 0
    ctx.interpolate(attr, v, tri, tid, interp, bary=bary, append_z=s.append_z)
    if interp is not img:
        img[:, : s.C_out].copy_(interp)
        img[:, s.C_out].copy_(tid >= 0)
    g = np.random.default_rng(50 + k).standard_normal((n, s.C_e), dtype=np.float32)
    g_v = torch.zeros_like(v)
    g_attr = torch.zeros_like(attr)
    ctx.backward(v, tri, tid, attr, img, to_dev(g), g_attr, g_v, append_z=s.append_z)
    torch.cuda.synchronize()
    got = dict(tri_id=tid.cpu().numpy(), depth=depth.cpu().numpy(),
               bary=None if bary is None else bary.cpu().numpy(), interp=interp.cpu().numpy(),
               g_v=g_v.cpu().numpy(), g_attr=g_attr.cpu().numpy())
    del ctx, img, interp, tid, depth, bary
    torch.cuda.empty_cache()
    check_forward(s, got, ref)
    rgv, rga = oracle.backward(s, ref, g, threads=THREADS)
    check_grads(s, got, rgv, rga, f"calls config {k}")


def run_step(k):
    """The benchmark's timed step, call for call, against the oracle."""
    import torch
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench
    s, ref = full(k)
    say(f"[full] step: config {k} {s.name}")
    tune = tuned(s)
    dev = torch.device("cuda")
    st = bench.Step(s, [list(range(s.n_views))], tuple(tune["tile"]), not s.recompute, dev, tune["small_px"],
                    tune["bin_cap"], tune.get("big_tiles", 0))
    target = np.random.default_rng(70 + k).uniform(0, 1, size=(s.n_px, s.C_e)).astype(np.float32)
    st.target.copy_(to_dev(target))
    st.run()
    torch.cuda.synchronize()
    assert st.ctxs[0].status()["overflow_tiles"] == 0
    got = dict(tri_id=st.tid.cpu().numpy(), depth=st.depth.cpu().numpy(),
               bary=None if st.bary is None else st.bary.cpu().numpy(), interp=st.interp.cpu().numpy(),
               g_v=st.g_v.cpu().numpy(), g_attr=st.g_attr.cpu().numpy())
    del st
    torch.cuda.empty_cache()
    check_forward(s, got, ref)
    g = 2.0 * (ref["image"] - target.astype(np.float64))  # L = sum (I - T)^2 on the oracle's own image
    rgv, rga = oracle.backward(s, ref, g, threads=THREADS)
    check_grads(s, got, rgv, rga, f"step config {k}")
