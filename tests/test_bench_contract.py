"""bench.py's host-side contract (CPU): one GPU only, and the roofline's measured
traffic taken from the committed profile only while it matches the kernel source."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_measured_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    src = tmp_path / "kernels.hip"
    src.write_bytes(b"// kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    md = tmp_path / "profile.md"
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    monkeypatch.setattr(bench, "PROFILE_MD", str(md))
    md.write_text(f"# profile\n\n- traffic_primal_phase_bytes: 123456\n- kernel_source_sha256: {sha}\n")
    assert bench.measured_traffic() == 123456.0
    src.write_bytes(b"// kernel source, changed\n")   # counters taken on other code: void
    assert bench.measured_traffic() is None
    md.unlink()
    assert bench.measured_traffic() is None
