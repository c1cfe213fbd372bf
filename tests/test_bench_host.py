"""Host-side checks of bench.py: the one-GPU guard and the committed HBM-traffic record it
reads (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_record_parses_and_follows_the_kernel_source(tmp_path, monkeypatch):
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.loads(f.read().split("```json", 1)[1].split("```", 1)[0])
    assert rec["kernel"] == "k_cfr_mfma16"
    assert rec["hbm_bytes_per_launch"] == rec["read_bytes"] + rec["write_bytes"]
    # the figure is used only while the kernel source hashes to the recorded value
    src = tmp_path / "kernels.hip"
    src.write_bytes(b"// another source\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    assert bench.measured_traffic("k_cfr_mfma16") is None
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(tmp_path / "missing.hip"))
    assert bench.measured_traffic("k_cfr_mfma16") is None
    assert bench.measured_traffic("k_other") is None
