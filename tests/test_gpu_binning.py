"""GPU: the binning passes' tile lists, read back from the workspace.

The fill pass keeps a hash table of tiles per workgroup; when a workgroup's
triangles touch more tiles than the table holds, entries go through the
tiles' global counters instead, and the table's two passes must agree on
every entry (see tests/test_bin_table.py for the protocol on the CPU).
These tests drive that regime -- scattered triangles, each workgroup of the
binning passes touching thousands of tiles -- and check the lists the
rasterizer then reads: every tile counter back at 0, every list entry a
distinct triangle of the view, every triangle that the CPU oracle shows
visible at some pixel of a tile present in that tile's list, and the index
image bit-exact against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2405_02508_amd import scenes
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def tile_lists(ctx):
    """(offs int64 [tiles + 1], bins int32 [entries], count int32 [tiles]) of
    the last rasterize, read from the workspace."""
    P = ctx.plan
    ws = ctx.ws.cpu().numpy()
    nt = int(P.total_tiles)

    def view(off, n, dt):
        return np.frombuffer(ws[int(off): int(off) + n * np.dtype(dt).itemsize].tobytes(), dt)

    offs = view(P.off_offs, nt + 1, np.int32).astype(np.int64)
    count = view(P.off_count, nt, np.int32)
    bins = view(P.off_bins, int(offs[-1]), np.int32)
    return offs, bins, count


@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (32, 8), (16, 8)])
@pytest.mark.parametrize("big_tiles", [-1, 16])
def test_tile_lists_overfull_tables(tile, big_tiles):
    import torch
    from paper_2405_02508_amd import mer
    s = scenes.scattered_triangles(7, 65536, 2048, 2048, 40.0)
    vw = s.view(0)
    H, W, n_t = vw["H"], vw["W"], vw["n_t"]
    say(f"[binning] {s.name} tile {tile} big_tiles {big_tiles}")
    ctx = mer.Context(s.views, device="cuda", tile=tile, small_px=-1, big_tiles=big_tiles)
    v, tri = to_dev(s.v), to_dev(s.tri)
    tid = torch.empty(s.n_px, dtype=torch.int32, device="cuda")
    ctx.rasterize(v, tri, tid)
    st = ctx.status()  # raises on a nonzero integrity count
    assert st["overflow_tiles"] == 0 and st["bad_entries"] == 0 and st["unbalanced_tiles"] == 0
    offs, bins, count = tile_lists(ctx)
    assert np.all(count == 0)
    assert bins.size == st["entries"]
    assert np.all((bins >= 0) & (bins < n_t))
    tw, th = tile
    tiles_x = (W + tw - 1) // tw
    n_tiles = tiles_x * ((H + th - 1) // th)
    assert offs.size == n_tiles + 1
    # distinct entries per tile
    tile_of = np.repeat(np.arange(n_tiles, dtype=np.int64), np.diff(offs))
    keys = tile_of * n_t + bins
    assert np.unique(keys).size == keys.size
    # every visible triangle is listed in the tile of each pixel showing it
    ref = oracle.rasterize(s.v, s.tri, H, W)
    got = tid.cpu().numpy()
    assert np.array_equal(got, ref), f"tri_id differs at {int((got != ref).sum())} pixels"
    yy, xx = np.divmod(np.arange(H * W, dtype=np.int64), W)
    vis = ref >= 0
    need = np.unique((yy[vis] // th * tiles_x + xx[vis] // tw) * n_t + ref[vis])
    assert np.all(np.isin(need, keys, assume_unique=True))
    say(f"[binning] ok: {bins.size} entries, {int(vis.sum())} covered px")
