"""Build libmer.so in-tree with hipcc for gfx950 (cross-compiles without a GPU)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["mer_api.hip", "mer_raster.hip", "mer_backward.hip", "mer_transform.hip", "mer_jvp.hip", "mer_texture.hip"]
OUT = os.path.join(HERE, "libmer.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # the depth key and plane slopes are specified operation by operation
    "-ffp-contract=off",
    # hardware float atomics on coarse-grained memory
    "-munsafe-fp-atomics",
    # no packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


# reference kernels for the rooflines (copy, float atomics): their own library
PEAK_SOURCES = ["mer_peak.hip"]
PEAK_OUT = os.path.join(HERE, "libmer_peak.so")


def _hipcc(sources, out, verbose):
    tmp = out + ".tmp"
    cmd = ["hipcc", *FLAGS, "-o", tmp, *[os.path.join(CSRC, s) for s in sources]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    _hipcc(PEAK_SOURCES, PEAK_OUT, verbose)
    return _hipcc(SOURCES, OUT, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
