"""The allocation-free centre (lb_centre_noalloc) against lb_centre, through the C ABI.

Two calls in a row on one GPU, the second on a smaller box, in float64 and
float32, each compared with lb_centre of a context holding the same phi: the
two run the same kernels and fixed-order float64 sums, so the linear centre
and sum phi agree to 1e-13 relative and the circular mean (atan2 on the
device instead of the host) to 1e-12 absolute.  A box above the maximum is
rejected before any work.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_2011_00287_amd import inputs
from paper_2011_00287_amd._lib import LB_EINVAL, LB_FP32, LB_FP64, LB_OK, lib
from paper_2011_00287_amd.sim import Sim

pytestmark = pytest.mark.gpu

# (nx, ny, nz, droplet radius): the second box is smaller than the first; the
# first has more than 4096 blocks of partials, so its sums take the chunked path
BOXES = [(128, 96, 100, 20.0), (40, 36, 30, 7.0)]


def _noalloc(phi_dev, shape, prec, out, stream):
    nz, ny, nx = shape
    return lib().lb_centre_noalloc(nx, ny, nz, prec, ctypes.c_void_p(phi_dev.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_centre_noalloc_matches_lb_centre(prec):
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    p = dict(inputs.BASE_PARAMS, q0=0.5, zeta=0.0)
    dt = torch.float64 if prec == "fp64" else torch.float32
    code = LB_FP64 if prec == "fp64" else LB_FP32
    out = torch.full((7,), float("nan"), dtype=torch.float64, device="cuda")
    for k, (nx, ny, nz, R) in enumerate(BOXES):
        phi, q5 = inputs.droplet_fields(nx, ny, nz, R, p["q0"], seed=k)
        phi = np.roll(phi, (3 * k + 2, -5, 7), axis=(0, 1, 2))  # off-centre, across the periodic faces
        with Sim(p, phi, q5, precision=prec, stream=stream) as s:
            lin, circ, tot = s.centre()
        phi_dev = torch.tensor(phi, dtype=dt, device="cuda")
        print(f"lb_centre_noalloc {prec} call {k + 1}: box {nx}x{ny}x{nz}", flush=True)
        assert _noalloc(phi_dev, phi.shape, code, out, stream) == LB_OK, lib().lb_last_error()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        print(got, lin, circ, tot, flush=True)
        assert np.all(np.abs(got[:3] - lin) <= 1e-13 * np.abs(lin)), (got[:3], lin)
        assert abs(got[6] - tot) <= 1e-13 * abs(tot), (got[6], tot)
        d = np.remainder(got[3:6] - circ + np.array([nx, ny, nz]) / 2, [nx, ny, nz]) - np.array([nx, ny, nz]) / 2
        assert np.all(np.abs(d) <= 1e-12), (got[3:6], circ)


def test_centre_noalloc_rejects_a_box_above_the_maximum():
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    phi = torch.zeros(8, dtype=torch.float64, device="cuda")
    out = torch.zeros(7, dtype=torch.float64, device="cuda")
    # 2^25 + 1024 sites: refused before any launch, so the small arrays are never read
    st = lib().lb_centre_noalloc(1024, 1024, 33, LB_FP64, ctypes.c_void_p(phi.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
    assert st == LB_EINVAL
    assert b"maximum" in lib().lb_last_error()
    assert lib().lb_centre_noalloc(4, 4, 4, LB_FP64, None, ctypes.c_void_p(out.data_ptr()), None) == LB_EINVAL
