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
