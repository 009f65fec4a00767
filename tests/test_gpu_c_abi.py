"""The library driven from plain C (tests/cpp/abi_c.c), without Python or
torch: a uniform body force gives total momentum N f (t + 1/2) exactly
(float64); a chiral droplet conserves mass and sum(phi) in float64 and
float32; invalid arguments return LB_EINVAL."""
import subprocess
import tempfile

import pytest

from c_abi_build import compile_c_consumer

pytestmark = pytest.mark.gpu


def test_c_consumer_runs():
    with tempfile.TemporaryDirectory() as d:
        exe = compile_c_consumer(d)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "C ABI OK" in r.stdout
