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


def test_stored_figures_follow_the_source_hash(tmp_path, monkeypatch):
    t = {"src_hash": bench.source_hash(), "fetch_scale": 2.0, "write_scale": 1.0,
         "workloads": {"4": {"k_backward": {"fetch_kib": 10.0, "write_kib": 3.0, "valu_instr": 614400000}}}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(t))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.stored_traffic(4, "k_backward") == 1024 * (2 * 10 + 3)
    v = bench.stored_valu_issue(4, "k_backward", 2.0)
    assert abs(v["issue_ms"] - 1.0) < 1e-9 and abs(v["frac"] - 0.5) < 1e-9
    assert bench.stored_traffic(3, "k_backward") is None and bench.stored_valu_issue(3, "k_backward", 1.0) is None
    t["src_hash"] = "other"
    f.write_text(json.dumps(t))
    assert bench.stored_traffic(4, "k_backward") is None and bench.stored_valu_issue(4, "k_backward", 1.0) is None

