"""Benchmark: forward + backward Mpixels/s of the micro-edge path on one GPU.

A step is one pass of the whole path over one batch of views, with the
inputs resident in HBM: rasterize (set-up, binning, tiled z-buffer, resolve),
interpolate, clearing the gradient buffers, and the fused micro-edge +
interpolation backward of the L2 image loss L = sum (I - T)^2, whose
gradient 2 (I - T) is formed inside the backward kernel.
Batched = all views of the workload in one captured HIP graph; per-view =
the same calls issued view by view without a graph.

It also times, on the same pixels and outside the step's timed region, the
forward-mode image tangent (field ``jvp``) and deferred texturing with an
8-channel 1024^2 texture, forward and adjoint (field ``texture``);
``--no-extras`` skips them.

The roofline object is for the backward sweep: algorithmic bytes over its
measured launch time against HBM peak, the HBM bytes from stored rocprofv3
counters (``traffic``), and the time its VALU instructions take at the
chip's issue rate over the launch time (``valu_issue``); the stored figures
are reported only while the kernel's sources hash to what they were taken on.

Prints ONE JSON line.  ``--gpus`` above 1 is refused: the benchmark
measures one GPU (views shard across GPUs with one gradient all-reduce, which
is not part of it).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")

WORKLOADS = {
    4: "batched: 256 displaced-icosphere scenes (1k-200k tris, 10% intersecting pairs), 128-1024 px square",
    2: "one 512x512 view of two interpenetrating displaced icospheres (nu=64, 163,840 tris)",
    3: "head-like mesh (60,500 tris), 64 views at 1024x667",
    5: "2M-tri intersecting pair, 16 views at 2048x2048, barycentrics recomputed",
    1: "icosphere nu=4 (320 tris), one 64x64 view",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Step:
    """Device buffers and the call sequence of one step for a set of views."""

    def __init__(self, scene, groups, tile, store_bary, dev, small_px=0, bin_cap=0, big_tiles=0):
        import torch

        from paper_2405_02508_amd import mer
        s = scene
        self.s = s
        self.dev = dev
        self.v = torch.from_numpy(s.v).to(dev)
        self.tri = torch.from_numpy(s.tri).to(dev)
        self.attr = torch.from_numpy(s.attr).to(dev)
        n = s.n_px
        self.tid = torch.empty(n, dtype=torch.int32, device=dev)
        self.depth = torch.empty(n, dtype=torch.float32, device=dev)
        self.bary = torch.empty(n, 2, dtype=torch.float32, device=dev) if store_bary else None
        self.img = torch.empty(n, s.C_e, dtype=torch.float32, device=dev)
        self.interp = self.img if s.C_e == s.C_out else torch.empty(n, s.C_out, dtype=torch.float32, device=dev)
        self.g_v = torch.zeros_like(self.v)
        self.g_attr = torch.zeros_like(self.attr)
        self.ctxs = [mer.Context(s.views[grp], device=dev, tile=tile, small_px=small_px, big_tiles=big_tiles,
                                 bin_cap=bin_cap if len(groups) == 1 else 0) for grp in groups]
        # L2 target image rendered once from perturbed vertices (outside the timed region)
        self.target = torch.zeros(n, s.C_e, dtype=torch.float32, device=dev)
        if s.v_target is not None:
            vt = torch.from_numpy(s.v_target).to(dev)
            for c in self.ctxs:
                c.rasterize(vt, self.tri, self.tid, None, self.bary)
                c.interpolate(self.attr, vt, self.tri, self.tid, self.interp, bary=self.bary, append_z=s.append_z)
            self._assemble()
            self.target.copy_(self.img)
        else:
            self.target.copy_(torch.rand(n, s.C_e, generator=torch.Generator(device=dev).manual_seed(7), device=dev))

    def _assemble(self):
        if self.img is not self.interp:
            self.img[:, : self.s.C_out].copy_(self.interp)
            self.img[:, self.s.C_out].copy_((self.tid >= 0).float())

    def forward(self):
        """Rasterize, resolve and interpolate in one pass per plan."""
        s = self.s
        for c in self.ctxs:
            c.rasterize_interpolate(self.v, self.tri, self.tid, self.attr, self.interp, depth=self.depth,
                                    bary=self.bary, append_z=s.append_z)
        self._assemble()

    def backward(self):
        """Gradient of L = sum (I - T)^2 to vertices and attributes in one sweep
        (dL/dI is formed inside the backward kernel; the value of L is not
        needed for the step and is not computed)."""
        self.g_v.zero_()
        self.g_attr.zero_()
        for c in self.ctxs:
            c.backward_l2(self.v, self.tri, self.tid, self.attr, self.img, self.target, self.g_attr, self.g_v,
                          weight=1.0, append_z=self.s.append_z)

    def run(self):
        self.forward()
        self.backward()


def time_region(fn, steps, stream):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def kernel_times(st, iters, stream):
    """Average duration of each library call on its stream, HIP events."""
    import torch
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    names = ("rasterize_interpolate", "backward")
    acc = {k: 0.0 for k in names}
    for _ in range(iters):
        marks = [ev() for _ in range(6)]
        marks[0].record(stream)
        for c in st.ctxs:
            c.rasterize_interpolate(st.v, st.tri, st.tid, st.attr, st.interp, depth=st.depth, bary=st.bary,
                                    append_z=st.s.append_z)
        marks[1].record(stream)
        marks[2].record(stream)
        st._assemble()
        st.g_v.zero_()
        st.g_attr.zero_()
        marks[3].record(stream)
        for c in st.ctxs:
            c.backward_l2(st.v, st.tri, st.tid, st.attr, st.img, st.target, st.g_attr, st.g_v, weight=1.0,
                          append_z=st.s.append_z)
        marks[4].record(stream)
        torch.cuda.synchronize()
        acc["rasterize_interpolate"] += marks[0].elapsed_time(marks[1])
        acc["backward"] += marks[3].elapsed_time(marks[4])
    return {k: acc[k] / iters for k in names}


def jvp_time(st, iters, stream):
    """Forward-mode image tangent of the step's image (mer_jvp, one call per
    plan) for a seeded tangent of every screen vertex and attribute: average
    call time on its stream, HIP events."""
    import torch
    s = st.s
    gen = torch.Generator(device=st.dev).manual_seed(11)
    dv = torch.randn(st.v.shape, generator=gen, device=st.dev)
    dv[:, 2] *= 0.01 * st.v[:, 2]
    dattr = torch.randn(st.attr.shape, generator=gen, device=st.dev)
    dimg = torch.empty(s.n_px, s.C_e, dtype=torch.float32, device=st.dev)
    st.forward()

    def call():
        for c in st.ctxs:
            c.jvp(st.v, st.tri, st.tid, st.attr, st.img, dv, dimg, dattr=dattr, append_z=s.append_z)

    call()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(iters):
        call()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / iters


def texture_time(st, iters, stream, size=1024, channels=8):
    """Deferred texturing on the step's pixels: uv interpolated from seeded
    per-vertex uv, an 8-channel 1024^2 texture (the paper's neural texture)
    sampled, then its adjoint to the texture and uv.  Average call times on
    the stream, HIP events."""
    import torch

    from paper_2405_02508_amd import scenes
    s = st.s
    uv_attr, tex = scenes.texture_inputs(s, 1, size=size, channels=channels)
    ua = torch.from_numpy(uv_attr).to(st.dev)
    texd = torch.from_numpy(tex).to(st.dev)
    uvp = torch.empty(s.n_px, 2, dtype=torch.float32, device=st.dev)
    out = torch.empty(s.n_px, channels, dtype=torch.float32, device=st.dev)
    g = torch.randn(s.n_px, channels, generator=torch.Generator(device=st.dev).manual_seed(5), device=st.dev)
    g_tex = torch.zeros_like(texd)
    g_uv = torch.empty(s.n_px, 2, dtype=torch.float32, device=st.dev)
    st.forward()
    for c in st.ctxs:
        c.interpolate(ua, st.v, st.tri, st.tid, uvp, bary=None, append_z=False)

    def fwd():
        for c in st.ctxs:
            c.texture(st.tid, uvp, texd, out)

    def bwd():
        for c in st.ctxs:
            c.texture_bwd(st.tid, uvp, texd, g, g_tex, g_uv)

    res = {}
    for name, fn in (("forward", fwd), ("backward", bwd)):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(iters):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / iters
    return res


def algorithmic_bytes(s, kernel, channels=8, tex_bytes=1024 * 1024 * 8 * 4):
    """Bytes the method must move per launch (model stated in the design notes)."""
    n_px = s.n_px
    V = s.views
    view_tris = int(V[:, 5].sum())
    view_verts = int(V[:, 4].sum())
    if kernel == "backward":
        # read tri_id, image, dL/dimage per pixel; per view-triangle its index row,
        # per view-vertex its position and gradient row (read + write)
        return n_px * (4 + 8 * s.C_e) + view_tris * 12 + view_verts * 12 * 3 + s.attr.size * 4 * 3
    if kernel == "rasterize":
        # per view-triangle index row, per view-vertex position; write tri_id, depth (+bary)
        return view_tris * 12 + view_verts * 12 + n_px * (8 + (8 if not s.recompute else 0))
    if kernel == "jvp":
        # read tri_id and image, write the tangent image per pixel; per
        # view-triangle its index row, per view-vertex position and tangent;
        # attributes and their tangent
        return n_px * (4 + 8 * s.C_e) + view_tris * 12 + view_verts * 24 + s.attr.size * 4 * 2
    if kernel == "texture":
        # read tri_id and uv, write the samples; the texture once
        return n_px * (4 + 8 + 4 * channels) + tex_bytes
    if kernel == "texture_bwd":
        # read tri_id, uv and dL/d(out), write dL/duv; texture read once,
        # its gradient read and written once
        return n_px * (4 + 8 + 4 * channels + 8) + 3 * tex_bytes
    if kernel == "interpolate":
        return n_px * (4 + (8 if not s.recompute else 0) + 4 * s.C_out) + s.attr.size * 4 + view_tris * 12
    raise KeyError(kernel)


# HIP sources that define the backward sweep kernel (its file and the device
# helpers it includes)
BACKWARD_SOURCES = ("mer_backward.hip", "mer_device.h")


def source_hash(names=BACKWARD_SOURCES):
    """Hash of a kernel's HIP sources, to tell whether stored counter data
    still describes the kernel being run."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2405_02508_amd", "csrc")
    for name in names:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def stored_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from rocprofv3 FETCH_SIZE / WRITE_SIZE
    runs (KiB per dispatch, scaled by the same counters of a plain copy of
    known size), or None when absent or taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("src_hash") != source_hash():
        return None
    e = t.get("workloads", {}).get(str(workload), {}).get(kernel)
    if not e:
        return None
    return int(1024 * (e["fetch_kib"] * t["fetch_scale"] + e["write_kib"] * t["write_scale"]))


VALU_ISSUE_PER_S = 256 * 2.4e9  # wave64 VALU instructions per second: one per CU per cycle


def stored_valu_issue(workload, kernel, launch_ms):
    """Time the kernel's VALU instructions take at the chip's issue rate,
    and that time over the measured launch, from a stored SQ_INSTS_VALU
    count (rocprofv3 --pmc); None when absent or taken on other sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("src_hash") != source_hash():
        return None
    n = t.get("workloads", {}).get(str(workload), {}).get(kernel, {}).get("valu_instr")
    if not n:
        return None
    ms = n / VALU_ISSUE_PER_S * 1e3
    return {"valu_instr": n, "issue_ms": round(ms, 4), "frac": round(ms / launch_ms, 4)}


def cpu_baseline(scene, budget_s=15.0):
    """The CPU oracle as it stands (single thread) on a bounded sample of the
    workload: whole views, forward + backward, until the time budget is used."""
    import oracle
    oracle.lib()
    n_views, px = 0, 0
    t0 = time.perf_counter()
    for i in range(scene.n_views):
        px += oracle.step_view(scene, i)
        n_views += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": round(px / dt / 1e6, 4), "unit": "Mpx/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_views} of {scene.n_views} views ({px} px), forward+backward, one thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=4, choices=sorted(WORKLOADS))
    ap.add_argument("--tile", default="auto", help="WxH, or 'auto' for the autotuner's choice")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the timings of the forward-mode image tangent and the texture sampler")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (3 times), to scale HBM "
                         "byte counters, and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        ms = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            dst.copy_(src)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        print(json.dumps({"copy_bytes": 4 * n, "ms": [round(x, 4) for x in ms],
                          "GBps": round(8 * n / min(ms) / 1e6, 1)}), flush=True)
        return

    from paper_2405_02508_amd import mer, scenes
    mer.lib()  # fail loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    s = scenes.make_config(args.workload)
    log(f"[bench] workload {args.workload} {s.name}: {s.n_views} views, {s.n_px} px, "
        f"{int(s.views[:, 5].sum())} view-tris, scene built in {time.perf_counter() - t0:.1f}s")
    stream = torch.cuda.current_stream()
    if args.tile == "auto":
        from paper_2405_02508_amd import autotune
        t0 = time.perf_counter()
        tu = autotune.tune(s.views, torch.from_numpy(s.v).to(dev), torch.from_numpy(s.tri).to(dev), log=log)
        tuning = {"tile": list(tu["tile"]), "small_px": tu["small_px"], "big_tiles": tu["big_tiles"], "bin_cap": tu["bin_cap"],
                  "source": "autotuner (cached)" if tu.get("cached") else "autotuner"}
        log(f"[bench] autotune {time.perf_counter() - t0:.1f}s -> {tuning}")
    else:
        tuning = {"tile": [int(x) for x in args.tile.split("x")], "small_px": 0, "big_tiles": 0, "bin_cap": 0,
                  "source": "flag"}
    tile = tuple(tuning["tile"])

    # ---- batched: every view in one plan, captured in a HIP graph
    st = Step(s, [list(range(s.n_views))], tile, not s.recompute, dev, tuning["small_px"], tuning["bin_cap"],
              tuning["big_tiles"])
    for _ in range(args.warmup):
        st.run()
    torch.cuda.synchronize()
    graph = None
    if not args.no_graph:
        graph = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream()
        cs.wait_stream(stream)
        with torch.cuda.stream(cs):
            st.run()
            torch.cuda.synchronize()
            with torch.cuda.graph(graph, stream=cs):
                st.run()
        stream.wait_stream(cs)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        run_batched = graph.replay
    else:
        run_batched = st.run
    ms = time_region(run_batched, args.steps, stream)
    log(f"[bench] batched {'graph' if graph else 'eager'}: {ms:.3f} ms/step")
    kt = kernel_times(st, max(3, min(args.steps, 10)), stream)
    log(f"[bench] per-call ms: {kt}")
    extras = {}
    if not args.no_extras:
        jvp_ms = jvp_time(st, max(3, min(args.steps, 10)), stream)
        log(f"[bench] forward-mode image tangent: {jvp_ms:.3f} ms per call")
        tex_ms = texture_time(st, max(3, min(args.steps, 10)), stream)
        log(f"[bench] texture sampler 1024^2 x 8: {tex_ms}")
        jb, tb, tbb = algorithmic_bytes(s, "jvp"), algorithmic_bytes(s, "texture"), algorithmic_bytes(s, "texture_bwd")
        # forward-mode image tangent of the same image (Sec. 5, forward
        # gradients), and deferred texturing of the same pixels with an
        # 8-channel 1024^2 texture: each its own call, outside the step
        extras = {
            "jvp": {"kernel": "k_jvp", "ms_per_call": round(jvp_ms, 4), "value": round(s.n_px / jvp_ms / 1e3, 2),
                    "unit": "Mpx/s",
                    "roofline": {"bound": "hbm", "achieved": round(jb / (jvp_ms * 1e-3) / 1e9, 1), "peak": PEAK_HBM_GBS,
                                 "unit": "GB/s", "frac": round(jb / (jvp_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                                 "algorithmic_bytes": jb}},
            "texture": {"kernels": ["k_texture", "k_texture_bwd"], "texture": [1024, 1024, 8],
                        "ms_forward": round(tex_ms["forward"], 4), "ms_backward": round(tex_ms["backward"], 4),
                        "roofline_forward": {"bound": "hbm", "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                             "achieved": round(tb / (tex_ms["forward"] * 1e-3) / 1e9, 1),
                                             "algorithmic_bytes": tb},
                        "roofline_backward": {"bound": "alu", "peak": None, "unit": "GB/s",
                                              "achieved": round(tbb / (tex_ms["backward"] * 1e-3) / 1e9, 1),
                                              "algorithmic_bytes": tbb}},
        }
    status = st.ctxs[0].status()
    log(f"[bench] status {status}")

    # ---- per-view: one plan and one launch sequence per view, no graph
    pv = None
    used_graph = graph is not None
    if not args.no_per_view and s.n_views > 1:
        graph = None
        st_pv = Step(s, [[i] for i in range(s.n_views)], tile, not s.recompute, dev, tuning["small_px"],
                     big_tiles=tuning["big_tiles"])
        for _ in range(max(1, args.warmup)):
            st_pv.run()
        ms_pv = time_region(st_pv.run, max(2, args.steps // 4), stream)
        pv = {"ms_per_step": round(ms_pv, 4), "value": round(s.n_px / ms_pv / 1e3, 2)}
        log(f"[bench] per-view eager: {ms_pv:.3f} ms/step")
        del st_pv

    # roofline of the dominant single kernel: k_backward, the one kernel of the
    # backward call (plus a ~5 us view-table prep); the rasterize call is a
    # pipeline of eight kernels, none as long as the backward sweep
    dom = "backward"
    ab = algorithmic_bytes(s, dom)
    achieved = ab / (kt[dom] * 1e-3) / 1e9
    out = {
        "metric": "fwd+bwd Mpixels/s (raster+micro-edge grad), batched vs per-view, err<=1e-5",
        "value": round(s.n_px / ms / 1e3, 2),
        "unit": "Mpx/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"config {args.workload}: {WORKLOADS[args.workload]}", "scene": s.name,
                   "views": s.n_views, "pixels": s.n_px, "view_triangles": int(s.views[:, 5].sum()),
                   "tuning": tuning, "graph": used_graph, "barycentrics": "recomputed" if s.recompute else "stored"},
        "per_view": pv,
        "per_call_ms": {k: round(v, 4) for k, v in kt.items()},
        "roofline": {"kernel": "k_backward", "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": stored_traffic(args.workload, "k_backward"),
                     "valu_issue": stored_valu_issue(args.workload, "k_backward", kt[dom]),
                     "algorithmic_bytes": ab, "avg_launch_ms": round(kt[dom], 4), "src_hash": source_hash()},
        "cpu_baseline": None,
        **extras,
    }
    if not args.no_cpu:
        del st
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
