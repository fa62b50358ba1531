"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed).

* The CPU oracle (oracle/rapdhg_oracle.c) with a driver that calls every entry point on
  small seeded problems with edge cases (tests/oracle_sanitize.c), built with gcc.
* The host side of qp_create -- input validation of invalid host problems, and the
  threaded P = [Q | -A'] and column-panel layout builders (tests/host_layouts.cpp) --
  built with hipcc, the sanitizers applied to the host code only.
Any sanitizer report aborts the program; leak detection is on."""
import os
import subprocess

import paper_2311_07710_amd as qpa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe, want):
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=900, env=ENV)
    assert out.returncode == 0, out.stdout[-3000:] + out.stderr[-3000:]
    assert want in out.stdout
    assert "ERROR: AddressSanitizer" not in out.stderr
    assert "runtime error" not in out.stderr


def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-fopenmp",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-o", str(exe),
                    os.path.join(ROOT, "oracle", "rapdhg_oracle.c"),
                    os.path.join(ROOT, "tests", "oracle_sanitize.c"), "-lm"],
                   check=True, capture_output=True)
    _run(exe, "oracle sanitize run ok")


def test_host_validation_and_layouts_under_asan_ubsan(tmp_path):
    qpa.load()  # the library must be built
    lib = os.path.join(ROOT, "paper_2311_07710_amd", "lib")
    exe = tmp_path / "host_layouts_san"
    san = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
                 "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", flag]
    subprocess.run(["/opt/rocm/bin/hipcc", "-O1", "-g", "-std=c++17", "-pthread", "-x", "hip",
                    "--offload-arch=gfx950", *san,
                    os.path.join(ROOT, "tests", "host_layouts.cpp"), "-o", str(exe),
                    "-I", os.path.join(ROOT, "include"), "-L", lib, "-lqp_mi355x",
                    "-Wl,-rpath," + lib],
                   check=True, capture_output=True)
    _run(exe, "all ok")


def test_oracle_test_suite_under_asan_ubsan(tmp_path):
    """The oracle's own CPU tests (pins, preprocessing, infeasibility, threads, classes)
    against a build of the oracle with AddressSanitizer and UndefinedBehaviorSanitizer,
    loaded into Python with the sanitizer runtimes preloaded (leak detection off: the
    interpreter itself is not instrumented)."""
    import sys
    so = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-D_POSIX_C_SOURCE=199309L",
                    "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-o", str(so),
                    os.path.join(ROOT, "oracle", "rapdhg_oracle.c"), "-lm"],
                   check=True, capture_output=True)
    rt = [subprocess.run(["gcc", f"-print-file-name={n}"], capture_output=True, text=True,
                         check=True).stdout.strip() for n in ("libasan.so", "libubsan.so")]
    env = dict(ENV, ORACLE_LIB=str(so), LD_PRELOAD=" ".join(rt),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    files = ["tests/test_oracle_pins.py", "tests/test_oracle_precondition.py",
             "tests/test_oracle_infeas.py", "tests/test_oracle_threads.py",
             "tests/test_classes.py"]
    out = subprocess.run([sys.executable, "-c", "from oracle import oracle; print(oracle.LIB_PATH)"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert out.stdout.strip() == str(so), out.stderr[-2000:]
    out = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          "-m", "not gpu", *files], cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=1200)
    assert out.returncode == 0, out.stdout[-3000:] + out.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in out.stderr and "runtime error" not in out.stderr
