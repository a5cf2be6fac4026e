"""bench.py's host-side contract: one GPU only, and HBM traffic reported only
for the kernel sources the byte counters were taken on."""
import json
import subprocess
import sys

import bench


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(bench.ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_follows_the_source_digest(tmp_path, monkeypatch):
    rec = {"kernels": {"y/c128": {"bytes_per_launch": 123, "source_sha256_16": bench.source_digest(
        bench.KERNEL_SOURCES["y"])}}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", f)
    assert bench.measured_traffic("y", "c128") == 123
    assert bench.measured_traffic("y", "c64") is None          # not measured
    rec["kernels"]["y/c128"]["source_sha256_16"] = "0" * 16     # sources changed since
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic("y", "c128") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", tmp_path / "missing.json")
    assert bench.measured_traffic("y", "c128") is None


def test_committed_profile_names_every_sweep():
    rec = json.loads(bench.TRAFFIC_FILE.read_text())["kernels"]
    for k in ("nu_x", "y", "z"):
        for dt in ("c128", "c64"):
            r = rec[f"{k}/{dt}"]
            # the counters see what the algorithm moves: one read and one write of psi
            assert abs(r["bytes_per_launch"] / r["alg_bytes_per_launch"] - 1.0) < 0.01
