"""The host-threaded layout builders of qp_create (P = [Q | -A'] and the column
panels) equal their definitions; compiled with hipcc against the built library,
run on the CPU with no GPU call."""
import os
import subprocess

import paper_2311_07710_amd as qpa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_threaded_layout_builders(tmp_path):
    qpa.load()  # the library must be built
    lib = os.path.join(ROOT, "paper_2311_07710_amd", "lib")
    exe = tmp_path / "host_layouts"
    subprocess.run(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-pthread", "-x", "hip",
                    "--offload-arch=gfx950", os.path.join(ROOT, "tests", "host_layouts.cpp"),
                    "-o", str(exe), "-I", os.path.join(ROOT, "include"), "-L", lib,
                    "-lqp_mi355x", "-Wl,-rpath," + lib],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all ok" in out.stdout
