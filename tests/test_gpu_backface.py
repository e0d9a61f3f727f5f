"""GPU back-face image and its micro-edge gradient against the oracle
(supplement, "Implementation detail": the image that is 1 where the wrong
side of a triangle is visible, passed through EdgeGrad with the loss
10 ||I||^2)."""
import functools

import numpy as np
import pytest

import oracle
from paper_2405_02508_amd import mer, scenes
from tests.gpu_util import rel_l2, say, to_dev

pytestmark = pytest.mark.gpu

WEIGHT = 10.0


def _reversed(s, frac):
    """The same scene with the winding of a seeded fraction of its triangles reversed."""
    flip = np.random.default_rng(11).random(s.tri.shape[0]) < frac
    t = np.where(flip[:, None], s.tri[:, [0, 2, 1]], s.tri).astype(np.int32)
    per = []
    for i in range(s.n_views):
        vw = s.view(i)
        per.append((s.v[vw["v_off"]: vw["v_off"] + vw["n_v"]], t[vw["t_off"]: vw["t_off"] + vw["n_t"]],
                    i, i, vw["H"], vw["W"]))
    attrs = [s.attr[s.view(i)["a_off"]: s.view(i)["a_off"] + s.view(i)["n_v"]] for i in range(s.n_views)]
    return scenes._pack(s.name + "-reversed", per, attrs, s.append_z, s.mask_channel)


@functools.lru_cache(maxsize=None)
def scene(k, reverse=0.0):
    s = scenes.make_config(k, small=True)
    return _reversed(s, reverse) if reverse else s


def oracle_backface(s):
    tid = np.full(s.n_px, -1, np.int32)
    img = np.zeros(s.n_px)
    g_v = np.zeros((s.v.shape[0], 3))
    for i in range(s.n_views):
        vw, vs, ts, _ = oracle._view_slices(s, i)
        H, W, o = vw["H"], vw["W"], vw["px_off"]
        t = oracle.rasterize(vs, ts, H, W)
        b = oracle.backface(vs, ts, H, W, t)
        sl = slice(o, o + H * W)
        tid[sl], img[sl] = t, b
        gv = oracle.edge_grad(vs, ts, H, W, t, b[:, None], 2.0 * WEIGHT * b[:, None])
        g_v[vw["v_off"]: vw["v_off"] + vw["n_v"]] += gv
    return tid, img, g_v


def gpu_backface(s, tile=(8, 8)):
    import torch
    v, tri = to_dev(s.v), to_dev(s.tri)
    ctx = mer.Context(s.views, tile=tile)
    tid = torch.empty(s.n_px, dtype=torch.int32, device="cuda")
    ctx.rasterize(v, tri, tid)
    img = torch.full((s.n_px, 1), -3.0, dtype=torch.float32, device="cuda")
    ctx.backface(v, tri, tid, img)
    g_v = torch.zeros_like(v)
    ctx.edge_grad(v, tri, tid, img, (2.0 * WEIGHT) * img, g_v)
    torch.cuda.synchronize()
    return tid.cpu().numpy(), img[:, 0].cpu().numpy(), g_v.cpu().numpy()


@pytest.mark.parametrize("k,reverse", [(1, 0.0), (1, 1.0), (2, 0.5), (3, 1.0), (4, 0.0), (4, 0.5), (5, 0.5)])
def test_backface_image_and_gradient_match_the_oracle(k, reverse):
    s = scene(k, reverse)
    say(f"[backface] config {k} reversed={reverse}")
    t_ref, b_ref, gv_ref = oracle_backface(s)
    t, b, gv = gpu_backface(s)
    assert np.array_equal(t, t_ref)
    assert np.array_equal(b, b_ref.astype(np.float32))  # a 0/1 decision on exact integers: bit-exact
    if reverse == 1.0:
        assert np.array_equal(b, (t >= 0).astype(np.float32))
    if np.abs(gv_ref).max() > 0:
        assert rel_l2(gv, gv_ref) <= 1e-5
    else:
        assert np.abs(gv).max() == 0
    say(f"[backface] config {k} reversed={reverse}: {int(b.sum())} back-face px, ok")


def test_backface_loss_through_autograd():
    """back_face_image + the loss 10 ||I||^2 through torch autograd gives the
    oracle's micro-edge gradient."""
    import torch

    from paper_2405_02508_amd.autograd import Renderer, back_face_image
    s = scene(4, 0.5)
    say("[backface] autograd")
    _, _, gv_ref = oracle_backface(s)
    r = Renderer(s.views, s.tri)
    v = to_dev(s.v).requires_grad_(True)
    tid, _, _ = r.rasterize(v)
    img = back_face_image(r, v, tid)
    loss = WEIGHT * (img * img).sum()
    loss.backward()
    assert rel_l2(v.grad.cpu().numpy(), gv_ref) <= 1e-5
