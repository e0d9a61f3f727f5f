"""Stored rocprofv3 counter figures for the benchmark's rooflines.

``python -m paper_2405_02508_amd.counters --workload 4 CSV...`` reads
rocprofv3 ``--pmc`` output (``*_counter_collection.csv``), averages every
counter per kernel over its dispatches, derives the figures the benchmark
reports, prints them as a markdown table, and merges them into
``profiles/counters.json`` under the workload, keyed by the backward
kernel's source hash (bench.py ignores figures taken on other sources).

Derived figures, per dispatch:
  * ``hbm_read_bytes``: L2-to-fabric read bytes, 32 B x TCC_EA0_RDREQ_32B +
    64 B x TCC_EA0_RDREQ_64B + 128 B x TCC_EA0_RDREQ_128B (the MALL in front
    of HBM may serve some of them);
  * ``hbm_write_bytes``: WRITE_SIZE (KiB) x 1024;
  * ``atomics``: float atomics issued to L2 (TCC_ATOMIC);
  * ``valu_instr``, ``waves``, ``lds_instr``, ``lds_bank_conflict_cycles``:
    SQ_INSTS_VALU, SQ_WAVES, SQ_INSTS_LDS, SQ_LDS_BANK_CONFLICT.
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DEFAULT_OUT = os.path.join(ROOT, "profiles", "counters.json")


def kernel_key(name: str) -> str:
    """'void mer::k_backward<true, false, true>(...)' -> 'k_backward<true, false, true>'."""
    n = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").strip()
    return n.split("::")[-1] if "::" in n else n


def read(paths):
    """{kernel: {counter: mean per dispatch}, with 'dispatches'}."""
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                acc[kernel_key(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = {}
    for k, d in acc.items():
        out[k] = {c: sum(v) / len(v) for c, v in d.items()}
        out[k]["dispatches"] = max(len(v) for v in d.values())
    return out


def derive(c):
    """The figures bench.py reads, from one kernel's averaged counters."""
    g = lambda *names: next((c[n] for n in names if n in c), None)  # noqa: E731
    out = {}
    n32, n64, n128 = g("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_32B"), g("TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_64B"), \
        g("TCC_EA0_RDREQ_128B_sum", "TCC_EA0_RDREQ_128B")
    if None not in (n32, n64, n128):
        out["hbm_read_bytes"] = int(32 * n32 + 64 * n64 + 128 * n128)
    ws = g("WRITE_SIZE")
    if ws is not None:
        out["hbm_write_bytes"] = int(ws * 1024)
    if "hbm_read_bytes" in out and "hbm_write_bytes" in out:
        out["hbm_bytes"] = out["hbm_read_bytes"] + out["hbm_write_bytes"]
    for key, names in (("atomics", ("TCC_ATOMIC_sum", "TCC_ATOMIC")), ("valu_instr", ("SQ_INSTS_VALU",)),
                       ("salu_instr", ("SQ_INSTS_SALU",)), ("waves", ("SQ_WAVES",)), ("lds_instr", ("SQ_INSTS_LDS",)),
                       ("lds_bank_conflict_cycles", ("SQ_LDS_BANK_CONFLICT",)),
                       ("lds_active_cycles", ("SQ_LDS_IDX_ACTIVE",)), ("wave_cycles", ("SQ_WAVE_CYCLES",)),
                       ("busy_cycles", ("SQ_BUSY_CYCLES",)), ("wait_any", ("SQ_WAIT_ANY",))):
        v = g(*names)
        if v is not None:
            out[key] = int(round(v))
    out["dispatches"] = c["dispatches"]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--note", default="")
    ap.add_argument("--lane-atomics", type=int, default=0,
                    help="lane-level float atomics per dispatch of the reference kernel k_atomic_add "
                         "(bench.py issues 256 x 8192 lanes x 32)")
    ap.add_argument("--only", default="", help="keep only kernels whose name starts with this")
    ap.add_argument("csv", nargs="+")
    a = ap.parse_args(argv)
    sys.path.insert(0, ROOT)
    import bench
    per = {k: derive(c) for k, c in read(a.csv).items() if k.startswith(a.only)}
    try:
        with open(a.out) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    if data.get("src_hash") != bench.source_hash():
        data = {"src_hash": bench.source_hash(), "workloads": {}}
    wl = data["workloads"].setdefault(str(a.workload), {})
    # one entry per kernel template: its instantiation with the most dispatches
    best = {}
    for k, d in per.items():
        base = k.split("<")[0]
        if base not in best or d["dispatches"] > per[best[base]]["dispatches"]:
            best[base] = k
    for base, k in best.items():
        wl.setdefault(base, {}).update(per[k])
        wl[base]["kernel"] = k
        if base == "k_atomic_add" and a.lane_atomics:
            wl[base]["lane_atomics"] = a.lane_atomics
    if a.note:
        data["note"] = a.note
    with open(a.out, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    keys = sorted({x for d in per.values() for x in d})
    print("| kernel | " + " | ".join(keys) + " |")
    print("|---|" + "---|" * len(keys))
    for k, d in sorted(per.items()):
        print(f"| `{k}` | " + " | ".join(str(d.get(x, "")) for x in keys) + " |")


if __name__ == "__main__":
    main()
