"""The oracle's C library under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): every C entry point, on the small form of every workload,
must run without a sanitizer report.  An out-of-bounds index or an integer
overflow in the oracle would otherwise corrupt the values every parity test
trusts without failing anything by itself."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SCRIPT = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[2])
import oracle
oracle._LIB = sys.argv[1]
oracle._lib = None
from paper_2405_02508_amd import scenes
for k in (1, 2, 3, 4, 5):
    s = scenes.make_config(k, small=True)
    rng = np.random.default_rng(k)
    f = oracle.forward(s)
    g = rng.standard_normal((s.n_px, s.C_e)).astype(np.float32)
    oracle.backward(s, f, g)
    oracle.backward(s, f, g, flags=oracle.NO_INTERSECT)
    dv = (0.01 * rng.standard_normal(s.v.shape)).astype(np.float32)
    da = rng.standard_normal(s.attr.shape).astype(np.float32)
    oracle.jvp(s, f, dv, da)
    vw = s.view(0)
    v = s.v[vw["v_off"]: vw["v_off"] + vw["n_v"]]
    tri = s.tri[vw["t_off"]: vw["t_off"] + vw["n_t"]]
    H, W = int(s.views[0, 6]), int(s.views[0, 7])
    tid = oracle.rasterize(v, tri, H, W)
    oracle.backface(v, tri, H, W, tid)
    if k == 1:  # brute force over every (triangle, centre) pair: smallest workload only
        oracle.cover_count(v, tri, H, W)
        assert np.array_equal(oracle.rasterize(v, tri, H, W, brute=True), tid)
    uv, tex = scenes.texture_inputs(s, k, size=64, channels=4)
    uvp = rng.uniform(-0.2, 1.2, (H * W, 2))
    uvp[::97] = np.nan
    out = oracle.texture(tex, uvp, tid)
    oracle.texture_bwd(tex, uvp, np.ones_like(out), tid)
    print("workload", k, "clean", flush=True)
"""


def _runtime(name):
    try:
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True, timeout=60)
    except (OSError, subprocess.TimeoutExpired):
        return None
    p = p.stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_runs_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = tmp_path / "liboracle_sanitized.so"
    src = os.path.join(ROOT, "oracle", "mer_oracle.c")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-o", str(lib), src, "-lm"], check=True, timeout=300)
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", SCRIPT, str(lib), ROOT], capture_output=True, text=True, env=env,
                       timeout=900, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.count("clean") == 5
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
