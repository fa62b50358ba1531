"""Build the gfx950 shared library ``lib/libqp_mi355x.so`` with hipcc.

Every source is compiled for gfx950 only.  Packed FP32 instructions are
disabled (``-packed-fp32-ops``).  The solver sources are compiled with
``-ffp-contract=off`` so each FP64 operation in the source is one IEEE
operation (no fused multiply-add), which keeps row sums and epilogues
comparable operation-for-operation with a sequential reference.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libqp_mi355x.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# per-source extra flags
SOURCES = {
    "qp_kernels.hip": ["-ffp-contract=off"],
    "qp_batch.hip": ["-ffp-contract=off"],
    "qp_scale.hip": ["-ffp-contract=off"],
    "qp_api.cpp": ["-ffp-contract=off", "-pthread", "-x", "hip"],
}
OPTIONAL = {
    "mlp_kernels.hip": [],
    "mlp_api.cpp": ["-x", "hip"],
}


def _compile(src: str, extra: list, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(line for line in (r.stderr or "").splitlines()
                     if "packed-fp32-ops" not in line and line.strip())
    if warn and verbose:
        print(warn, flush=True)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    jobs = dict(SOURCES)
    for src, extra in OPTIONAL.items():
        if os.path.exists(os.path.join(CSRC, src)):
            jobs[src] = extra
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        objs = list(ex.map(lambda kv: _compile(kv[0], kv[1], verbose), jobs.items()))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
