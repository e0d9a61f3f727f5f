"""The C-ABI library loads and exports what include/mer.h declares; the
host-only plan call validates its inputs.  No GPU needed."""
import ctypes
import functools
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2405_02508_amd import mer

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mer.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(mer.LIB_PATH):
        from paper_2405_02508_amd import build
        build.build()
    return mer.lib()


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mer_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_binding_symbols():
    assert set(declared()) == set(mer.SYMBOLS)


def test_library_exports_every_declared_symbol(L):
    out = subprocess.run(["nm", "-D", "--defined-only", mer.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (mer_\w+)", out))
    for name in declared():
        assert name in exported, name
        assert hasattr(L, name)


def test_struct_layout_matches_header(tmp_path):
    c = tmp_path / "lay.c"
    c.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "mer.h"\nint main(void){'
                 'printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(mer_view), sizeof(mer_tuning),'
                 'sizeof(mer_plan), offsetof(mer_view,n_v), offsetof(mer_plan,ws_bytes), offsetof(mer_plan,n_part),'
                 'sizeof(mer_camera), offsetof(mer_camera,f), offsetof(mer_camera,w_off));return 0;}')
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(c), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = [ctypes.sizeof(mer.View), ctypes.sizeof(mer.Tuning), ctypes.sizeof(mer.Plan),
            mer.View.n_v.offset, mer.Plan.ws_bytes.offset, mer.Plan.n_part.offset,
            ctypes.sizeof(mer.Camera), mer.Camera.f.offset, mer.Camera.w_off.offset]
    assert got == want
    assert want[6] == 72


def test_version_and_strerror(L):
    assert L.mer_version() >= 1
    assert L.mer_strerror(0) == b"ok"
    assert b"invalid" in L.mer_strerror(-1)


def _views(rows):
    return np.array(rows, np.int64)


def test_plan_totals_and_layout(L):
    V = _views([[0, 0, 0, 0, 10, 20, 17, 33], [10, 0, 0, 17 * 33, 10, 20, 8, 8]])
    P = mer.plan_init(V, (8, 8))
    assert P.total_tris == 40 and P.total_px == 17 * 33 + 64
    assert P.total_tiles == 3 * 5 + 1
    offs = [P.off_viewtab, P.off_rec, P.off_bbox, P.off_count, P.off_offs, P.off_part, P.off_bins, P.off_status,
            P.off_key]
    assert offs == sorted(offs) and all(o % 256 == 0 for o in offs) and P.ws_bytes > offs[-1]
    assert P.bin_cap > 0 and P.small_px == 16
    assert P.ws_bytes - P.off_key >= 8 * P.total_px
    P2 = mer.plan_init(V, (16, 16), bin_cap=5)
    assert P2.bin_cap == 5 and P2.total_tiles == 2 * 3 + 1
    # bin offsets are 32-bit and saturate at INT_MAX, so the pool stays below it
    assert mer.plan_init(V, (8, 8), bin_cap=1 << 40).bin_cap == 2**31 - 2


def _regions(P):
    """(name, offset, bytes the kernels index) for every workspace region:
    the view tables, the set-up records and boxes, the tile counters, offsets
    and scan partials, the bin pool, the status words, the 64-bit key image,
    the 16x16-tile view table, the vertex bases, the per-wave loss partials,
    and the per-workgroup large-triangle lists with their lengths, offsets,
    scan partials and flat copy."""
    nv, T, ng = P.n_views, P.total_tiles, P.n_bingroups
    return [
        ("viewtab", P.off_viewtab, 2 * (nv + 1) * 8),
        ("rec", P.off_rec, P.total_tris * 64),
        ("bbox", P.off_bbox, P.total_tris * 8),
        ("count", P.off_count, T * 4),
        ("offs", P.off_offs, (T + 1) * 4),
        ("part", P.off_part, -(-T // 1024) * 8),
        ("bins", P.off_bins, P.bin_cap * 4),
        ("status", P.off_status, 8 * 8),
        ("key", P.off_key, (P.total_px - P.px_begin) * 8),
        ("bviewtab", P.off_bviewtab, 2 * (nv + 1) * 8),
        ("vbase", P.off_vbase, (nv + 1) * 8),
        ("bloss", P.off_bloss, 4 * P.total_btiles * 4),
        ("big", P.off_big, ng * 256 * 4),
        ("bign", P.off_bign, (2 * ng + 1) * 4),
        ("bigpart", P.off_bigpart, -(-ng // 1024) * 8),
        ("bigflat", P.off_bigflat, P.total_tris * 4),
    ]


@functools.lru_cache(maxsize=None)
def _full_views(k):
    from paper_2405_02508_amd import scenes
    return scenes.make_config(k).views


def _tiles(V, tw, th):
    return int(sum(-(-int(w) // tw) * -(-int(h) // th) for h, w in zip(V[:, 6], V[:, 7])))


@pytest.mark.parametrize("k", [2, 3, 4, 5])
@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (32, 8), (16, 8)])
def test_plan_regions_hold_what_the_kernels_index(L, k, tile):
    """Every workspace region is 256-byte aligned, lies inside ws_bytes and
    is at least as large as the kernels index it, with no two regions
    overlapping, for the full-size view tables; the counts the launches size
    their grids from agree with the view table (the forward-mode sweep covers
    its 8x8 tiles with four workgroups per 16x16 tile)."""
    V = _full_views(k)
    P = mer.plan_init(V, tile)
    assert P.total_tiles == _tiles(V, *tile)
    assert P.total_btiles == _tiles(V, 16, 16)
    assert _tiles(V, 8, 8) <= 4 * P.total_btiles
    assert P.n_part == -(-P.total_tiles // 1024)
    assert P.n_bingroups == -(-P.total_tris // 256)
    assert P.total_px - P.px_begin == int((V[:, 6] * V[:, 7]).sum())
    regs = sorted(_regions(P), key=lambda r: r[1])
    for (name, off, size), nxt in zip(regs, regs[1:] + [("end", P.ws_bytes, 0)]):
        assert off % 256 == 0, name
        assert off + size <= nxt[1], f"{name} [{off}, {off + size}) runs into {nxt[0]} at {nxt[1]}"


@pytest.mark.parametrize("bad", [
    [[0, 0, 0, 0, 3, 1, 0, 8]],          # H = 0
    [[0, 0, 0, 0, 3, 1, 8, 40000]],      # W too large
    [[0, 0, 0, 0, -1, 1, 8, 8]],         # negative n_v
    [[0, 0, 0, 64, 3, 1, 8, 8], [0, 0, 0, 0, 3, 1, 8, 8]],   # views out of order
    [[0, 0, 0, 0, 3, 1, 8, 8], [0, 0, 0, 60, 3, 1, 8, 8]],   # overlapping pixels
])
def test_plan_rejects_bad_views(L, bad):
    with pytest.raises(mer.MerError, match="-1"):
        mer.plan_init(_views(bad))


def test_plan_rejects_too_many_tiles(L):
    # 128 views of 32767^2 pixels: 128 * 4096^2 = 2^31 tiles of 8x8 (the tile
    # counters and bin offsets are 32-bit); 127 such views are accepted
    n = 32767 * 32767
    rows = [[0, 0, 0, i * n, 3, 1, 32767, 32767] for i in range(128)]
    with pytest.raises(mer.MerError, match="-1"):
        mer.plan_init(_views(rows))
    assert mer.plan_init(_views(rows[:127]), (16, 16)).total_tiles == 127 * 2048 * 2048


def test_plan_rejects_bad_tile(L):
    with pytest.raises(mer.MerError, match="-4"):
        mer.plan_init(_views([[0, 0, 0, 0, 3, 1, 8, 8]]), (4, 4))


def test_calls_reject_null_arguments_before_any_launch(L):
    """Argument checks run on the host and return an error code; nothing is
    enqueued, so these run without a GPU."""
    V = _views([[0, 0, 0, 0, 3, 1, 8, 8]])
    P = mer.plan_init(V)
    p = ctypes.byref(P)
    fake = ctypes.c_void_p(16)  # never dereferenced: every call below fails its checks first
    assert L.mer_rasterize(p, None, fake, fake, fake, None, None, fake, None) == -1
    assert L.mer_rasterize(p, fake, fake, fake, fake, None, None, None, None) == -2
    assert L.mer_interpolate(p, fake, fake, 0, fake, fake, fake, fake, 0, fake, None) == -1
    assert L.mer_interpolate(p, fake, fake, 64, fake, fake, fake, fake, 1, fake, None) == -1
    assert L.mer_transform(p, fake, None, fake, fake, fake, None) == -1
    assert L.mer_transform(p, fake, fake, fake, fake, None, None) == -2
    assert L.mer_transform_bwd(p, fake, fake, fake, fake, None, fake, None) == -1
    assert L.mer_transform_bwd(p, fake, fake, fake, fake, fake, None, None) == -2
    assert L.mer_backface(p, fake, fake, fake, fake, None, None) == -1
    assert L.mer_backface(p, None, fake, fake, fake, fake, None) == -1
    assert L.mer_edge_grad(p, fake, fake, fake, fake, fake, fake, 0, 0, fake, fake, None) == -1
    assert L.mer_edge_grad(p, fake, fake, fake, fake, fake, fake, 3, 0, fake, None, None) == -2
    assert L.mer_interpolate_bwd(p, fake, fake, 3, fake, fake, fake, 0, fake, 2, fake, fake, fake, None) == -1
    assert L.mer_backward_fused(p, fake, fake, fake, fake, fake, 3, 0, fake, fake, 2, 0, fake, fake, fake,
                                None) == -1
    assert L.mer_backward_fused(p, fake, fake, fake, fake, fake, 3, 0, fake, fake, 3, 0, fake, fake, None,
                                None) == -2
    f = ctypes.c_float
    assert L.mer_backward_l2(p, fake, fake, fake, fake, fake, 3, 0, fake, None, f(1.0), 3, 0, fake, fake, None,
                             fake, None) == -1
    assert L.mer_backward_l2(p, fake, fake, fake, fake, fake, 3, 0, fake, fake, f(float("nan")), 3, 0, fake, fake,
                             None, fake, None) == -1
    assert L.mer_backward_l2(p, fake, fake, fake, fake, fake, 3, 0, fake, fake, f(1.0), 3, 0, fake, fake, None,
                             None, None) == -2
    # mer_jvp(plan, views, v, tri, tri_id, attr, dattr, C_a, append_z, img, C_e, dv, flags, dimg, ws, stream)
    assert L.mer_jvp(p, fake, fake, fake, fake, fake, None, 3, 0, fake, 3, fake, 0, None, fake, None) == -1
    assert L.mer_jvp(p, fake, fake, fake, fake, fake, None, 3, 0, fake, 0, fake, 0, fake, fake, None) == -1
    assert L.mer_jvp(p, fake, fake, fake, fake, fake, None, 3, 0, None, 3, fake, 0, fake, fake, None) == -1
    assert L.mer_jvp(p, fake, fake, fake, fake, None, None, 3, 0, fake, 3, fake, 0, fake, fake, None) == -1
    assert L.mer_jvp(p, fake, fake, fake, fake, fake, None, 3, 1, fake, 3, fake, 0, fake, fake, None) == -1
    assert L.mer_jvp(p, fake, fake, fake, fake, fake, None, 3, 0, fake, 3, fake, 0, fake, None, None) == -2
    # mer_texture(plan, views, tri_id, uv, ld_uv, tex, th, tw, C, out, stream)
    assert L.mer_texture(p, fake, None, fake, 1, fake, 4, 4, 3, fake, None) == -1
    assert L.mer_texture(p, fake, None, fake, 2, fake, 0, 4, 3, fake, None) == -1
    assert L.mer_texture(p, fake, None, fake, 2, fake, 4, 4, 65, fake, None) == -1
    assert L.mer_texture(p, fake, None, None, 2, fake, 4, 4, 3, fake, None) == -1
    assert L.mer_texture_bwd(p, fake, None, fake, 2, fake, 4, 4, 3, None, fake, fake, fake, None) == -1
    assert L.mer_texture_bwd(p, fake, None, fake, 2, fake, 4, 4, 3, fake, fake, fake, None, None) == -2
    assert L.mer_status(p, None, None, (ctypes.c_int64 * 6)()) == -2
    assert L.mer_plan_init(None, 1, None, p) == -1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No fallback: without the built library every call path raises."""
    monkeypatch.setattr(mer, "LIB_PATH", str(tmp_path / "absent" / "libmer.so"))
    monkeypatch.setattr(mer, "_lib", None)
    with pytest.raises(mer.MerError, match="missing"):
        mer.lib()
    with pytest.raises(mer.MerError, match="missing"):
        mer.plan_init(_views([[0, 0, 0, 0, 3, 1, 8, 8]]))


def test_peak_library_exports_what_its_header_declares():
    from paper_2405_02508_amd import peak
    if not os.path.exists(peak.LIB_PATH):
        from paper_2405_02508_amd import build
        build.build()
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "mer_peak.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(mer_peak_[a-z0-9_]+)\s*\(", src)))
    assert set(names) == set(peak.SYMBOLS)
    out = subprocess.run(["nm", "-D", "--defined-only", peak.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (mer_peak_\w+)", out))
    L = peak.lib()
    for name in names:
        assert name in exported and hasattr(L, name)
    # argument checks return before anything is enqueued (no GPU needed)
    assert L.mer_peak_copy(None, None, 16, None) == -1
    assert L.mer_peak_atomic_add(None, 16, 256, 1, None) == -1
    assert L.mer_peak_atomic_add(ctypes.c_void_p(256), 16, 100, 1, None) == -1


def test_noalloc_backward_checks_its_scratch_before_touching_the_device(L):
    """mer_backward_l2_noalloc: argument errors and a plan beyond its fixed
    scratch are refused before any device call."""
    P = mer.plan_init(np.array([[0, 0, 0, 0, 3, 1, 32767, 32767]], np.int64))  # 4.2 M backward tiles
    fake = ctypes.c_void_p(256)
    args = lambda loss: (ctypes.byref(P), fake, fake, fake, fake, fake, 3, 0, fake, fake,  # noqa: E731
                         ctypes.c_float(1.0), 3, 0, fake, fake, loss, None)
    assert L.mer_backward_l2_noalloc(*args(fake)) == -6
    assert b"scratch" in L.mer_strerror(-6)
    bad = list(args(fake))
    bad[9] = None  # no target
    assert L.mer_backward_l2_noalloc(*bad) == -1
