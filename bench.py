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


def autograd_time(s, tuning, dev, steps, warmup, stream, lr=1e-9):
    """The autograd form of the step on world-space geometry (the vertex
    transform module in front): Transform -> RenderStep (one call: raster,
    resolve, interpolation, EdgeGrad identity) -> L2 loss against a seeded
    target in torch -> loss.backward() (one fused sweep, then the transform's
    backward reducing the per-view screen gradients to world space) -> an
    SGD update of the world vertices and attributes.  Eager, HIP events on
    the stream; returns ms per step."""
    import torch

    from paper_2405_02508_amd import mer
    from paper_2405_02508_amd.autograd import Renderer, Transform, render
    w = s.meta["world"]
    r = Renderer(s.views, torch.from_numpy(s.tri).to(dev), device=dev, tile=tuple(tuning["tile"]),
                 small_px=tuning["small_px"], bin_cap=tuning["bin_cap"], big_tiles=tuning["big_tiles"],
                 append_z=s.append_z, mask_channel=s.mask_channel, store_bary=not s.recompute)
    cams = mer.Cameras(s.views, w["R"], w["C"], w["f"], w["cx"], w["cy"], w["w_off"], device=dev)
    vw = torch.from_numpy(w["v"]).to(dev).requires_grad_(True)
    attr = torch.from_numpy(s.attr).to(dev).requires_grad_(True)
    target = torch.rand(s.n_px, s.C_e, generator=torch.Generator(device=dev).manual_seed(9), device=dev)

    def step():
        v = Transform.apply(vw, cams, r)
        img, _, _ = render(v, attr, r)
        loss = ((img - target) ** 2).sum()
        loss.backward()
        with torch.no_grad():
            vw.sub_(lr * vw.grad)
            attr.sub_(lr * attr.grad)
            vw.grad.zero_()
            attr.grad.zero_()

    for _ in range(max(1, warmup)):
        step()
    return time_region(step, steps, stream)


def peak_rates(dev, stream, footprint_floats, copy_bytes=1 << 30):
    """Measured reference rates on this GPU (libmer_peak.so): a plain
    streaming copy of copy_bytes (GB/s counting read + write), and float
    atomic adds into a buffer of the workload's gradient footprint and into
    a 256 MiB buffer (atomics/s).  Best of 5 launches each, HIP events."""
    import torch

    from paper_2405_02508_amd import peak

    def best(fn, reps=5):
        fn()
        t = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            t.append(e0.elapsed_time(e1))
        return min(t)

    n = copy_bytes // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    ms_copy = best(lambda: peak.copy(src, dst))
    del src, dst
    lanes, per_lane = 256 * 8192, 32
    out = {"copy_GBps": round(2 * copy_bytes / ms_copy / 1e6, 1)}
    for name, fp in (("footprint", int(footprint_floats)), ("256MiB", 1 << 26)):
        buf = torch.zeros(fp, dtype=torch.float32, device=dev)
        ms = best(lambda: peak.atomic_add(buf, fp, lanes, per_lane))
        out[f"atomic_Gops_{name}"] = round(lanes * per_lane / ms / 1e6, 2)
        del buf
    out["footprint_floats"] = int(footprint_floats)
    torch.cuda.empty_cache()
    return out


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
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters.json")
VALU_PEAK_GIPS = 256 * 4 * 2.4e9 / 4 / 1e9  # wave64 VALU instructions: 4 SIMDs per CU, 4 cycles each


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


def stored_counters(workload, kernel):
    """Per-dispatch rocprofv3 counter figures of `kernel` on `workload`
    (profiles/counters.json), or None when absent or taken on other sources
    of the backward kernel."""
    try:
        with open(COUNTERS_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("src_hash") != source_hash():
        return None
    return t.get("workloads", {}).get(str(workload), {}).get(kernel)


def backward_roofline(s, workload, launch_ms, covered, pk):
    """Roofline object of the backward sweep (one launch = every pixel of
    every view): HBM bytes, VALU issue and float atomics, each as achieved
    over its peak; `bound` names the largest fraction and the top-level
    achieved/peak/frac are that one's."""
    sec = launch_ms * 1e-3
    ab = algorithmic_bytes(s, "backward")
    hbm = {"achieved": round(ab / sec / 1e9, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(ab / sec / 1e9 / PEAK_HBM_GBS, 4), "algorithmic_bytes": ab,
           "measured_copy_GBps": pk["copy_GBps"], "frac_of_copy": round(ab / sec / 1e9 / pk["copy_GBps"], 4)}
    # (3 position + C_a attribute) gradient values for each of the 3 vertices
    # of every covered pixel: the contributions the scatter must sum.  As
    # float atomics they would need contrib / peak seconds; the kernel sums
    # them in LDS first and issues `issued` atomics (stored counter), which
    # is what it asks of the atomic units.
    contrib = covered * 3 * (3 + s.C_a)
    apk = pk["atomic_Gops_footprint"]
    atom = {"contributions": contrib, "contributions_per_s": round(contrib / sec / 1e9, 2),
            "unreduced_frac": round(contrib / sec / 1e9 / apk, 4), "peak": apk, "unit": "Gatomic/s",
            "issued": None, "achieved": None, "frac": None, "pre_reduction": None}
    cs = stored_counters(workload, "k_backward")
    valu = None
    traffic = None
    lds = None
    if cs:
        if cs.get("valu_instr"):
            gi = cs["valu_instr"] / sec / 1e9
            valu = {"valu_instr": cs["valu_instr"], "achieved": round(gi, 1), "peak": VALU_PEAK_GIPS,
                    "unit": "G wave-instr/s", "frac": round(gi / VALU_PEAK_GIPS, 4),
                    "per_wave": round(cs["valu_instr"] / cs["waves"], 1) if cs.get("waves") else None}
        # the L2's atomic request counter (TCC_ATOMIC) counts requests, not
        # lanes: the reference kernel's requests per lane-atomic convert the
        # measured peak into requests per second
        ref = stored_counters("reference", "k_atomic_add")
        if cs.get("atomics") and ref and ref.get("atomics") and ref.get("lane_atomics"):
            rpk = apk * ref["atomics"] / ref["lane_atomics"]
            atom["issued"] = cs["atomics"]
            atom["achieved"] = round(cs["atomics"] / sec / 1e9, 3)
            atom["peak"] = round(rpk, 3)
            atom["unit"] = "G L2 atomic requests/s"
            atom["frac"] = round(cs["atomics"] / sec / 1e9 / rpk, 4)
            atom["pre_reduction"] = round(contrib / cs["atomics"], 2)
        traffic = cs.get("hbm_bytes")
        if cs.get("lds_bank_conflict_cycles") is not None:
            lds = {"bank_conflict_cycles": cs["lds_bank_conflict_cycles"], "lds_instr": cs.get("lds_instr")}
    parts = {"hbm": hbm, "alu": valu, "atomic": atom if atom["frac"] is not None else None}
    bound = max((k for k in parts if parts[k]), key=lambda k: parts[k]["frac"])
    top = parts[bound]
    return {"kernel": "k_backward", "bound": bound, "achieved": top["achieved"], "peak": top["peak"],
            "unit": top["unit"], "frac": top["frac"], "traffic": traffic, "hbm": hbm, "valu": valu,
            "atomic": atom, "lds": lds, "avg_launch_ms": round(launch_ms, 4), "src_hash": source_hash()}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_threads():
    """Threads for the all-cores oracle run: the CPUs this process may use,
    at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(scene, budget_s=12.0):
    """The CPU oracle as it stands on a bounded sample of the workload: whole
    views, forward + backward (rasterize, resolve, interpolate, L2 gradient,
    edge term, interpolation adjoint).  First one thread until the time
    budget is used, then the same views on every host core (views on a
    thread pool; the C calls release the interpreter lock).  The all-cores
    figure is the reported value."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    oracle.lib()
    n_views, px = 0, 0
    t0 = time.perf_counter()
    for i in range(scene.n_views):
        px += oracle.step_view(scene, i)
        n_views += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt1 = time.perf_counter() - t0
    threads = host_threads()
    # at least a few views per thread, so the pool is busy
    n_all = min(scene.n_views, max(n_views, 4 * threads))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        px_all = sum(ex.map(lambda i: oracle.step_view(scene, i), range(n_all)))
    dtn = time.perf_counter() - t0
    return {"value": round(px_all / dtn / 1e6, 4), "unit": "Mpx/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_all} of {scene.n_views} views ({px_all} px), forward+backward, "
                      f"{threads} threads (views on a thread pool), {dtn:.1f} s",
            "cpu_model": cpu_model(),
            "single_thread": {"value": round(px / dt1 / 1e6, 4), "cores": 1,
                              "sample": f"first {n_views} views ({px} px), {dt1:.1f} s"}}


def step_stats(fn, n, stream):
    """Per-step times (HIP events around each step) over n steps: median,
    10th and 90th percentile in ms."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    return {"n": n, "median": round(float(np.median(ms)), 4), "p10": round(float(np.percentile(ms, 10)), 4),
            "p90": round(float(np.percentile(ms, 90)), 4)}


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
    ap.add_argument("--no-autograd", action="store_true", help="skip the autograd-form step timing")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the timings of the forward-mode image tangent and the texture sampler")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run the reference copy kernel (k_copy16) over BYTES bytes (3 times), to check "
                         "the HBM byte counters against a known transfer, and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        from paper_2405_02508_amd import peak
        n = args.calibrate_copy // 16 * 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        ms = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            peak.copy(src, dst)
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
    stats = step_stats(run_batched, max(50, args.steps), stream)
    log(f"[bench] per-step ms over {stats['n']} steps: median {stats['median']} p10 {stats['p10']} p90 {stats['p90']}")
    kt = kernel_times(st, max(3, min(args.steps, 10)), stream)
    log(f"[bench] per-call ms: {kt}")
    covered = int((st.tid >= 0).sum().item())
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

    # ---- the autograd form on world-space geometry (vertex transform in front)
    ag = None
    if not args.no_autograd and "world" in s.meta:
        del st
        torch.cuda.empty_cache()
        st = None
        ms_ag = autograd_time(s, tuning, dev, max(3, args.steps // 2), args.warmup, stream)
        ag = {"ms_per_step": round(ms_ag, 4), "value": round(s.n_px / ms_ag / 1e3, 2), "unit": "Mpx/s",
              "calls": "Transform -> RenderStep -> torch L2 loss -> backward (fused sweep, transform backward) "
                       "-> SGD update", "graph": False}
        log(f"[bench] autograd step (eager): {ms_ag:.3f} ms/step")
        torch.cuda.empty_cache()

    # ---- reference rates for the rooflines, measured on this GPU
    grad_floats = s.v.shape[0] * 3 + s.attr.size
    pk = peak_rates(dev, stream, grad_floats)
    log(f"[bench] reference rates: {pk}")

    # roofline of the dominant single kernel: k_backward, the one kernel of the
    # backward call (plus a ~5 us view-table prep); the rasterize call is a
    # pipeline of eight kernels, none as long as the backward sweep
    dom = "backward"
    roof = backward_roofline(s, args.workload, kt[dom], covered, pk)
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
        "step_ms": stats,
        "per_view": pv,
        "autograd_step": ag,
        "per_call_ms": {k: round(v, 4) for k, v in kt.items()},
        "roofline": roof,
        "reference_rates": pk,
        "cpu_baseline": None,
        **extras,
    }
    if not args.no_cpu:
        st = None
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
