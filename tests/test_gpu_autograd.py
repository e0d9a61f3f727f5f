"""GPU: autograd wrappers and HIP-graph replay against the oracle and the
eager calls."""
import functools

import numpy as np
import pytest

from paper_2405_02508_amd import scenes
from tests.gpu_util import rel_l2, run_oracle, say, to_dev

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def case(k):
    s = scenes.make_config(k, small=True)
    g = scenes.image_grad(s, 3)
    return s, g, run_oracle(s, g)


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("store_bary", [True, False])
def test_render_step_matches_oracle(k, store_bary):
    import torch

    from paper_2405_02508_amd.autograd import Renderer, render
    s, g, ref = case(k)
    say(f"[autograd] RenderStep config {k} store_bary={store_bary}")
    r = Renderer(s.views, s.tri, append_z=s.append_z, mask_channel=s.mask_channel, store_bary=store_bary)
    v = to_dev(s.v).requires_grad_(True)
    a = to_dev(s.attr).requires_grad_(True)
    img, tid, depth = render(v, a, r)
    assert np.array_equal(tid.cpu().numpy(), ref["tri_id"])
    (img * to_dev(g)).sum().backward()
    assert rel_l2(v.grad.cpu().numpy(), ref["g_v"]) <= 1e-5
    assert rel_l2(a.grad.cpu().numpy(), ref["g_attr"]) <= 1e-5


def test_modules_compose_to_the_fused_step():
    """Interpolate -> (mask) -> EdgeGrad with torch autograd equals RenderStep."""
    import torch

    from paper_2405_02508_amd.autograd import EdgeGrad, Interpolate, Renderer, render
    s, g, ref = case(2)
    say("[autograd] module composition config 2")
    r = Renderer(s.views, s.tri, append_z=s.append_z, mask_channel=s.mask_channel)
    v = to_dev(s.v).requires_grad_(True)
    a = to_dev(s.attr).requires_grad_(True)
    tid, depth, bary = r.rasterize(v)
    it = Interpolate.apply(v, a, tid, bary, r)
    img = torch.cat([it, (tid >= 0).float()[:, None]], 1)
    out = EdgeGrad.apply(img, v, tid, r)
    (out * to_dev(g)).sum().backward()
    gv1, ga1 = v.grad.clone(), a.grad.clone()
    v.grad = None
    a.grad = None
    img2, _, _ = render(v, a, r)
    (img2 * to_dev(g)).sum().backward()
    assert rel_l2(gv1.cpu().numpy(), v.grad.cpu().numpy().astype(np.float64)) <= 1e-5
    assert rel_l2(ga1.cpu().numpy(), a.grad.cpu().numpy().astype(np.float64)) <= 1e-5
    assert rel_l2(gv1.cpu().numpy(), ref["g_v"]) <= 1e-5


def torch_projection(v_world, R, C, f, cx, cy):
    """World points [V,3] -> per-view screen vertices [n_cam * V, 3] with
    torch ops (differentiable): camera frame rows R [n,3,3], centres C
    [n,3], focal f [n], principal point (cx, cy) [n]."""
    import torch
    pc = v_world[None, :, :] @ R.transpose(1, 2).contiguous() - (R @ C[:, :, None])[:, :, 0][:, None, :]
    z = pc[..., 2]
    x = f[:, None] * pc[..., 0] / z + cx[:, None]
    y = f[:, None] * pc[..., 1] / z + cy[:, None]
    return torch.stack([x, y, z], -1).reshape(-1, 3)


def test_world_space_gradient_through_projection():
    """Per-view screen gradients reduce to world space through a torch
    projection in front of RenderStep (config-3-like multi-view rig)."""
    import torch

    from paper_2405_02508_amd.autograd import Renderer, render
    project = torch_projection
    say("[autograd] world-space projection, 4 views")
    vs, fs = scenes.icosphere(12)
    Vw = vs * np.array([0.09, 0.12, 0.11])
    cams = [scenes.look_at(e, [0, 0, 0], 400.0, 120, 160) for e in scenes.fibonacci_sphere(4, 1.0)]
    R = torch.tensor(np.stack([c.R for c in cams]), dtype=torch.float32, device="cuda")
    C = torch.tensor(np.stack([c.C for c in cams]), dtype=torch.float32, device="cuda")
    f = torch.tensor([c.f for c in cams], dtype=torch.float32, device="cuda")
    cx = torch.tensor([c.cx for c in cams], dtype=torch.float32, device="cuda")
    cy = torch.tensor([c.cy for c in cams], dtype=torch.float32, device="cuda")
    nv = Vw.shape[0]
    views = np.array([[i * nv, 0, 0, i * 120 * 160, nv, fs.shape[0], 120, 160] for i in range(4)], np.int64)
    r = Renderer(views, fs.astype(np.int32))
    vw = torch.tensor(Vw, dtype=torch.float32, device="cuda", requires_grad=True)
    attr = torch.rand(nv, 3, device="cuda", generator=torch.Generator(device="cuda").manual_seed(1))
    vscr = project(vw, R, C, f, cx, cy)
    vscr.retain_grad()
    img, tid, _ = render(vscr, attr, r)
    w = torch.rand(img.shape, device="cuda", generator=torch.Generator(device="cuda").manual_seed(2))
    (img * w).sum().backward()
    assert torch.isfinite(vw.grad).all() and vw.grad.abs().sum() > 0
    # same reduction by hand: sum over views of J_view^T g_screen_view in float64
    vw64 = vw.detach().double().requires_grad_(True)
    s64 = project(vw64, R.double(), C.double(), f.double(), cx.double(), cy.double())
    (s64 * vscr.grad.double()).sum().backward()
    np.testing.assert_allclose(vw.grad.cpu().numpy(), vw64.grad.cpu().numpy(), rtol=1e-4,
                               atol=1e-5 * vw64.grad.abs().max().item())


def test_graph_replay_matches_eager():
    """A captured step replays with the eager results every time, with eager
    work and synchronisation between replays."""
    import torch

    import bench
    s, g, ref = case(4)
    say("[graph] capture config 4 small, 3 replays")
    st = bench.Step(s, [list(range(s.n_views))], (8, 8), True, torch.device("cuda"))
    st.run()
    torch.cuda.synchronize()
    tid0, gv0, ga0 = st.tid.clone(), st.g_v.clone(), st.g_attr.clone()
    graph = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        st.run()
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=cs):
            st.run()
    torch.cuda.current_stream().wait_stream(cs)
    torch.cuda.synchronize()
    for i in range(3):
        st.tid.fill_(-5)
        st.g_v.fill_(123.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(st.tid, tid0), f"replay {i}: tri_id"
        assert rel_l2(st.g_v.cpu().numpy(), gv0.cpu().numpy().astype(np.float64)) <= 1e-5, f"replay {i}: g_v"
        assert rel_l2(st.g_attr.cpu().numpy(), ga0.cpu().numpy().astype(np.float64)) <= 1e-5
        _ = (torch.randn(1000, device="cuda") * 2).sum().item()   # eager work between replays


def test_textured_image_through_edge_grad():
    """The paper's deferred pipeline with torch autograd: Interpolate (uv)
    -> Texture -> EdgeGrad -> L = sum g * image; gradients to the texture,
    the uv attribute and the vertices against the same chain in the oracle
    (texture adjoint, interpolation adjoint with Omega, and the micro-edge
    term on the textured image).  A smooth texture, and pixels within 1e-3
    texel of a texel-centre line get dL/d(image) = 0, as in the sampler's
    chain test."""
    import torch

    import oracle
    from paper_2405_02508_amd.autograd import EdgeGrad, Interpolate, Renderer, Texture
    s = scenes.make_config(2, small=True)
    say("[autograd] textured image through EdgeGrad, config 2")
    uv_attr, _ = scenes.texture_inputs(s, 21, size=32, channels=4, texels_per_pixel=0.25)
    rng = np.random.default_rng(21)
    yy, xx = np.mgrid[0:32, 0:32]
    tex = np.stack([np.sin(2 * np.pi * (rng.integers(1, 5) * xx + rng.integers(-4, 5) * yy) / 32 + rng.uniform(0, 6))
                    for _ in range(4)], -1).astype(np.float32)
    r = Renderer(s.views, s.tri, append_z=s.append_z, mask_channel=False)
    v = to_dev(s.v).requires_grad_(True)
    ua = to_dev(uv_attr).requires_grad_(True)
    td = to_dev(tex).requires_grad_(True)
    tid, depth, bary = r.rasterize(v)
    uv_img = Interpolate.apply(v, ua, tid, bary, r)          # [px, 2 (+ z)]
    img = EdgeGrad.apply(Texture.apply(uv_img, td, tid, r), v, tid, r)
    # oracle chain (one view)
    vw = s.view(0)
    H, W = vw["H"], vw["W"]
    t_o = oracle.rasterize(s.v, s.tri, H, W)
    assert np.array_equal(tid.cpu().numpy(), t_o)
    uv_o = oracle.interpolate(uv_attr, s.v, s.tri, H, W, t_o, s.append_z)
    st = uv_o[:, :2] * 32 - 0.5
    edge = (np.abs(st - np.round(st)) < 1e-3).any(1)
    g = rng.standard_normal((s.n_px, 4))
    g[edge] = 0
    (img * to_dev(g.astype(np.float32))).sum().backward()
    img_o = oracle.texture(tex, uv_o, t_o)
    gt_o, gu_o = oracle.texture_bwd(tex, uv_o, g, t_o)
    g_uv_full = np.zeros((s.n_px, uv_o.shape[1]))
    g_uv_full[:, :2] = gu_o
    ga_o, gv_o = oracle.interpolate_bwd(uv_attr, s.v, s.tri, H, W, t_o, g_uv_full, s.append_z)
    oracle.edge_grad(s.v, s.tri, H, W, t_o, img_o, g, g_v=gv_o)
    for got, want, name in ((td.grad, gt_o, "g_tex"), (ua.grad, ga_o, "g_uv_attr"), (v.grad, gv_o, "g_v")):
        err = rel_l2(got.cpu().numpy(), want)
        say(f"[autograd] {name}: rel L2 {err:.2e}")
        assert err <= 1e-5, (name, err)
