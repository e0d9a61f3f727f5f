"""GPU: mer_backward_l2_noalloc -- the L2 backward without a workspace, its
scratch in the library's fixed per-GPU array -- against mer_backward_l2 with
a workspace, through the C ABI, on the same inputs: two calls of the
no-workspace entry point in a row, the second on a smaller plan, each
compared with the workspace call (vertex and attribute gradients within
1e-5 relative L2, the loss within 1e-5 relative)."""
import ctypes

import numpy as np
import pytest

from paper_2405_02508_amd import mer, scenes
from tests.gpu_util import rel_l2, say, to_dev

pytestmark = pytest.mark.gpu


def prepare(s):
    """Plan, forward outputs and a seeded target for scene s."""
    import torch
    ctx = mer.Context(s.views, device="cuda")
    v, tri, attr = to_dev(s.v), to_dev(s.tri), to_dev(s.attr)
    tid = torch.empty(s.n_px, dtype=torch.int32, device="cuda")
    img = torch.empty(s.n_px, s.C_e, dtype=torch.float32, device="cuda")
    out = img if s.C_e == s.C_out else torch.empty(s.n_px, s.C_out, dtype=torch.float32, device="cuda")
    ctx.rasterize_interpolate(v, tri, tid, attr, out, append_z=s.append_z)
    if out is not img:
        img[:, :s.C_out].copy_(out)
        img[:, s.C_out].copy_(tid >= 0)
    target = to_dev(np.random.default_rng(s.n_px).uniform(0, 1, (s.n_px, s.C_e)).astype(np.float32))
    return dict(ctx=ctx, v=v, tri=tri, attr=attr, tid=tid, img=img, target=target, append_z=s.append_z)


def backward(d, noalloc, with_loss):
    import torch
    g_v = torch.zeros_like(d["v"])
    g_attr = torch.zeros_like(d["attr"])
    loss = torch.zeros(1, dtype=torch.float32, device="cuda") if with_loss else None
    fn = d["ctx"].backward_l2_noalloc if noalloc else d["ctx"].backward_l2
    fn(d["v"], d["tri"], d["tid"], d["attr"], d["img"], d["target"], g_attr, g_v, weight=0.75, loss=loss,
       append_z=d["append_z"])
    return g_v, g_attr, loss


@pytest.mark.parametrize("with_loss", [True, False])
def test_noalloc_matches_the_workspace_call(with_loss):
    import torch
    big, small = scenes.make_config(4, small=True), scenes.make_config(2, small=True)
    assert big.n_px > small.n_px
    say(f"[noalloc] {big.name} ({big.n_px} px) then {small.name} ({small.n_px} px), loss {with_loss}")
    db, ds = prepare(big), prepare(small)
    ref = [backward(db, False, with_loss), backward(ds, False, with_loss)]
    got = [backward(db, True, with_loss), backward(ds, True, with_loss)]  # two calls in a row, big then small
    torch.cuda.synchronize()
    for (rv, ra, rl), (gv, ga, gl) in zip(ref, got):
        assert rel_l2(gv.cpu().numpy(), rv.cpu().numpy().astype(np.float64)) <= 1e-5
        assert rel_l2(ga.cpu().numpy(), ra.cpu().numpy().astype(np.float64)) <= 1e-5
        if with_loss:
            assert abs(gl.item() - rl.item()) <= 1e-5 * abs(rl.item())


def test_noalloc_rejects_a_plan_beyond_its_scratch():
    # one 32767 x 32767 view: 4.2 M backward tiles, 16 MB of loss partials
    P = mer.plan_init(np.array([[0, 0, 0, 0, 3, 1, 32767, 32767]], np.int64))
    L = mer.lib()
    fake = ctypes.c_void_p(256)  # never dereferenced: the size check comes first
    rc = L.mer_backward_l2_noalloc(ctypes.byref(P), fake, fake, fake, fake, fake, 3, 0, fake, fake,
                                   ctypes.c_float(1.0), 3, 0, fake, fake, fake, None)
    assert rc == -6 and b"scratch" in L.mer_strerror(rc)
