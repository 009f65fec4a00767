"""CPU check of the per-site reverse derivatives of the HIP path.

The device functions of physics.hpp / adjoint.hpp are host-callable; a small
C++ program (tests/cpp/adjoint_check.cpp) compares every hand-written
vector-Jacobian product with central differences of the forward function in
float64 (stress + molecular field w.r.t. the gradient data, zeta and q0; mu;
co-rotation; collision)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpp", "adjoint_check.cpp")
INC = os.path.join(ROOT, "paper_2011_00287_amd", "csrc")


def test_local_adjoints_match_central_differences():
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "adjoint_check")
        r = subprocess.run([hipcc, "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-I" + INC, SRC,
                            "-o", exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        print(r.stdout)
        assert r.returncode == 0, r.stdout
        assert "ALL OK" in r.stdout


def test_local_adjoints_under_host_sanitizers():
    """The same host program built with AddressSanitizer and UndefinedBehaviorSanitizer
    on its host code (out-of-bounds or uninitialised-index reads in the per-site
    functions, signed overflow, misaligned access); any report fails the run."""
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "adjoint_check_san")
        r = subprocess.run([hipcc, "-O1", "-g", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                            "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                            "-Xarch_host", "-fno-sanitize-recover=undefined", "-I" + INC, SRC, "-o", exe],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
        assert "ALL OK" in r.stdout
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
