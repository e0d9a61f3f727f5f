"""The HIP library's host code (plan layout, argument checks) built with
clang's AddressSanitizer and UndefinedBehaviorSanitizer on the host side
only: plan construction for every workload, tile shape and bin pool, the
rejected view tables, and every entry point's argument checks must run
without a report (a signed overflow in the layout arithmetic would be one).
No kernel is launched."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2405_02508_amd", "csrc")

SCRIPT = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[2])
from paper_2405_02508_amd import mer, scenes
mer.LIB_PATH = sys.argv[1]
mer._lib = None
L = mer.lib()
from tests import test_abi
for k in (1, 2, 3, 4, 5):
    for V in (scenes.make_config(k, small=True).views, test_abi._full_views(k)):
        for tile in ((8, 8), (16, 16), (32, 8), (16, 8)):
            for cap in (0, 5, 1 << 40):
                P = mer.plan_init(V, tile, bin_cap=cap)
                test_abi._regions(P)
bad = [[[0, 0, 0, 0, 3, 1, 0, 8]], [[0, 0, 0, 0, 3, 1, 8, 40000]], [[0, 0, 0, 0, -1, 1, 8, 8]],
       [[0, 0, 0, 64, 3, 1, 8, 8], [0, 0, 0, 0, 3, 1, 8, 8]], [[0, 0, 0, 0, 3, 1, 8, 8], [0, 0, 0, 60, 3, 1, 8, 8]]]
for b in bad:
    test_abi.test_plan_rejects_bad_views(L, b)
test_abi.test_plan_rejects_too_many_tiles(L)
test_abi.test_plan_rejects_bad_tile(L)
test_abi.test_calls_reject_null_arguments_before_any_launch(L)
for c in range(-8, 3):
    L.mer_strerror(c)
print("host clean", flush=True)
"""


def _clang_runtime():
    hits = sorted(glob.glob("/opt/rocm*/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_host_code_runs_clean_under_sanitizers(tmp_path):
    rt = _clang_runtime()
    if not rt or not shutil.which("hipcc"):
        pytest.skip("hipcc or clang's sanitizer runtime not installed")
    lib = tmp_path / "libmer_host_sanitized.so"
    srcs = [os.path.join(CSRC, s) for s in ("mer_api.hip", "mer_raster.hip", "mer_backward.hip", "mer_transform.hip",
                                            "mer_jvp.hip", "mer_texture.hip")]
    # the sanitizers go to the host pass only (-Xarch_host before each flag)
    subprocess.run(["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-shared-libsan",
                    "-Xarch_host", "-fno-omit-frame-pointer", "-o", str(lib), *srcs],
                   check=True, timeout=600, capture_output=True)
    env = dict(os.environ, LD_PRELOAD=rt, LD_LIBRARY_PATH=os.path.dirname(rt),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", SCRIPT, str(lib), ROOT], capture_output=True, text=True, env=env,
                       timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "host clean" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
