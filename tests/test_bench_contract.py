"""The parts of bench.py's contract that need no GPU: a request for more than one GPU ends with
a message before anything touches a device, and the committed HBM-traffic figure is reported
only while the kernel source is the one the counters were taken on."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_reported_only_for_the_measured_kernel_source(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_1901_08140_amd", "csrc", "swarm_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"kernel_source_sha256": sha, "hbm_bytes_per_launch": 4.5e8}
    (prof / "swarm_dummy_f32_argon_sweep_traffic.json").write_text(json.dumps(rec))
    csrc = tmp_path / "paper_1901_08140_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "swarm_kernels.hip").write_bytes(open(src, "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.committed_traffic() == 4.5e8
    (csrc / "swarm_kernels.hip").write_bytes(open(src, "rb").read() + b"\n// edited\n")
    assert bench.committed_traffic() is None
    (prof / "swarm_dummy_f32_argon_sweep_traffic.json").write_text("not json")
    assert bench.committed_traffic() is None
