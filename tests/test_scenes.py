"""Seeded input generator: mesh closed forms and determinism."""
import numpy as np
import pytest

from paper_2405_02508_amd import scenes


@pytest.mark.parametrize("nu", [1, 2, 4, 7, 16])
def test_icosphere_counts_and_watertight(nu):
    v, f = scenes.icosphere(nu)
    assert v.shape[0] == 10 * nu * nu + 2 and f.shape[0] == 20 * nu * nu
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]]).astype(np.int64)
    key = e[:, 0] * v.shape[0] + e[:, 1]
    rkey = e[:, 1] * v.shape[0] + e[:, 0]
    assert np.unique(key).size == key.size and np.isin(rkey, key).all()
    a, b, c = (v[f[:, k]] for k in range(3))
    assert np.all((np.cross(b - a, c - a) * (a + b + c)).sum(1) > 0)
    np.testing.assert_allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_configs_are_deterministic(k):
    a = scenes.make_config(k, small=True)
    b = scenes.make_config(k, small=True)
    for name in ("v", "tri", "attr", "views"):
        assert np.array_equal(getattr(a, name), getattr(b, name))
    assert a.views[:, 3].tolist() == np.concatenate([[0], np.cumsum(a.views[:-1, 6] * a.views[:-1, 7])]).tolist()
    assert a.tri.min() >= 0
    for i in range(a.n_views):
        vw = a.view(i)
        t = a.tri[vw["t_off"]: vw["t_off"] + vw["n_t"]]
        assert t.max() < vw["n_v"]
