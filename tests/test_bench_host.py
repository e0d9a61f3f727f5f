"""Host-side pieces of the benchmark: argument checks and the stored
counter figures (no GPU)."""
import json
import subprocess
import sys

import bench


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


class _Scene:
    """Stand-in with the attributes the byte model reads."""
    def __init__(self):
        import numpy as np
        self.n_px = 1000
        self.C_e, self.C_a, self.C_out, self.recompute = 3, 3, 3, False
        self.views = np.array([[0, 0, 0, 0, 50, 80, 25, 40]], np.int64)
        self.attr = np.zeros((50, 3), np.float32)
        self.v = np.zeros((50, 3), np.float32)


PK = {"copy_GBps": 5000.0, "atomic_Gops_footprint": 100.0}


def test_stored_figures_follow_the_source_hash(tmp_path, monkeypatch):
    t = {"src_hash": bench.source_hash(),
         "workloads": {"4": {"k_backward": {"valu_instr": 614400000, "waves": 1000, "atomics": 500000,
                                            "hbm_bytes": 12345, "lds_bank_conflict_cycles": 7, "lds_instr": 9}},
                       "reference": {"k_atomic_add": {"atomics": 1000, "lane_atomics": 64000}}}}
    f = tmp_path / "counters.json"
    f.write_text(json.dumps(t))
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(f))
    r = bench.backward_roofline(_Scene(), 4, 2.0, covered=800, pk=PK)
    # 614.4 M wave-instructions in 2 ms at 614.4 G/s peak: half the issue rate
    assert abs(r["valu"]["frac"] - 0.5) < 1e-9 and r["valu"]["per_wave"] == 614400.0
    assert r["traffic"] == 12345 and r["lds"]["bank_conflict_cycles"] == 7
    assert r["atomic"]["contributions"] == 800 * 3 * 6 and r["atomic"]["pre_reduction"] == round(14400 / 500000, 2)
    # 0.25 G requests/s against 100 G lane-atomics/s x (1000 / 64000) requests per lane-atomic
    assert abs(r["atomic"]["frac"] - 0.25 / (100.0 / 64)) < 1e-3
    # the bound is the largest fraction
    assert r["bound"] == "alu" and r["frac"] == r["valu"]["frac"]
    assert bench.stored_counters(3, "k_backward") is None
    t["src_hash"] = "other"
    f.write_text(json.dumps(t))
    r = bench.backward_roofline(_Scene(), 4, 2.0, covered=800, pk=PK)
    assert r["valu"] is None and r["traffic"] is None and r["atomic"]["issued"] is None
    assert r["bound"] == "hbm" and r["atomic"]["unreduced_frac"] > 0


def test_cpu_baseline_reports_both_thread_counts():
    from paper_2405_02508_amd import scenes
    s = scenes.make_config(1)
    out = bench.cpu_baseline(s, budget_s=0.01)
    assert out["kind"] == "oracle" and out["cores"] >= 1 and out["value"] > 0
    assert out["single_thread"]["cores"] == 1 and out["single_thread"]["value"] > 0
