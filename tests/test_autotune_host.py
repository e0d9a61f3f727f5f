"""Host-side pieces of the autotuner: the shape class that keys its cache,
and a cache hit, which returns before any device work."""
import json

import numpy as np

from paper_2405_02508_amd import autotune


def _views(n, H, W, tris):
    return np.array([[0, 0, 0, i * H * W, 3, tris, H, W] for i in range(n)], np.int64)


def test_shape_class_rounds_pixels_and_triangles_to_powers_of_two():
    a = autotune.shape_class(_views(64, 1024, 667, 60500))
    assert a == "v2-v64-px2^25-t2^22"
    # same view count, counts within the same power-of-two bucket: same class
    assert autotune.shape_class(_views(64, 1024, 660, 61000)) == a
    assert autotune.shape_class(_views(63, 1024, 667, 60500)) != a
    assert autotune.shape_class(_views(64, 2048, 1334, 60500)) != a


def test_cache_hit_returns_the_stored_choice(tmp_path):
    V = _views(16, 2048, 2048, 2007040)
    path = tmp_path / "tune.json"
    entry = {"tile": [8, 8], "small_px": -1, "big_tiles": -1, "bin_cap": 183216823, "entries": 146570182, "ms": 13.0}
    path.write_text(json.dumps({autotune.shape_class(V): entry}))
    got = autotune.tune(V, None, None, cache_path=str(path))
    assert got["cached"] and got["tile"] == (8, 8) and got["bin_cap"] == 183216823 and got["big_tiles"] == -1


def test_unreadable_cache_is_treated_as_empty(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert autotune._load(str(path)) == {}
    assert autotune._load(str(tmp_path / "absent.json")) == {}
