"""The whole coupled step in one launch (k_step_fused), through the C ABI.

The one-launch kernel is selected with LB_PATH_ONE_LAUNCH (the default is the
two-launch path, which is faster on MI355X).  It runs in float64 too, which
holds it to the 1e-12 parity of the FP64 oracle:

* random states on ragged boxes (tiles and slabs cut by the box, boxes
  smaller than one tile that wrap periodically inside it, sides of 3), with a
  body force, several slab depths, D3Q19 and the paper's D3Q15 scheme:
  <= 1e-12 per field (l2 and max norms) against the oracle after 3 steps;
* the 16^3 droplet over 100 steps: <= 1e-12 per field;
* recording steps (the replay of a checkpointed adjoint): the output state
  and the recorded u, F and rho - rho0 equal those of the two-launch path
  to 1e-13;
* float32 and float16 storage: the one-launch step equals the two-launch
  step to float32 rounding (2e-5, the tolerance of the tiled-vs-site tests),
  and to the float16 resolution of the stored populations (2e-3).
"""
import math

import numpy as np
import pytest
import torch

from oracle import d3q15
from paper_2011_00287_amd import inputs
from paper_2011_00287_amd.sim import Sim

from helpers import field_errors, oracle_observe, oracle_run, rel_err, t64

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
ONE = {"path": "one"}
TWO = {"path": "two"}
SHAPES = [(4, 4, 4), (5, 3, 4), (7, 6, 5), (12, 6, 7), (33, 9, 5), (34, 18, 11), (40, 20, 19), (3, 35, 6),
          (64, 16, 5)]


def _p(**kw):
    return dict(inputs.BASE_PARAMS, **kw)


def _check(errs, tol=TOL64):
    for name, (l2, mx) in errs.items():
        assert l2 <= tol and mx <= tol, (name, l2, mx)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("tz", [0, 1, 3])
def test_fp64_one_launch_vs_oracle(shape, tz):
    nx, ny, nz = shape
    p = _p(q0=2 * math.pi / 7, zeta=0.01, body_force=(1e-5, -2e-5, 3e-5))
    g, phi, q5 = inputs.random_fields(nx, ny, nz, seed=nx * 100 + ny * 10 + nz, g_amp=2e-3, q_amp=0.2)
    print(f"one-launch fp64 d3q19 {shape} tz {tz}", flush=True)
    with Sim(p, phi, q5, precision="fp64", tuning=dict(ONE, tz_step=tz)) as s:
        s.set_fields(g=g)
        s.step(3)
        go, qo, po = oracle_run(p, g, q5, phi, 3)
        rho_o, u_o = oracle_observe(p, go, qo, po)
        errs = field_errors(s.moments(), (rho_o, u_o, po, qo), p["rho0"])
        errs["g"] = rel_err(s.populations(), go)
    _check(errs)


@pytest.mark.parametrize("shape", [(5, 3, 4), (12, 6, 7), (34, 18, 11), (40, 20, 19)])
def test_fp64_one_launch_d3q15_vs_oracle(shape):
    nx, ny, nz = shape
    p = _p(q0=2 * math.pi / 7, zeta=0.01, body_force=(1e-5, -2e-5, 3e-5))
    g, phi, q5 = inputs.random_fields(nx, ny, nz, seed=nx * 100 + ny * 10 + nz, g_amp=2e-3, q_amp=0.2)
    g = np.ascontiguousarray(g[:15])
    print(f"one-launch fp64 d3q15 {shape}", flush=True)
    with Sim(p, phi, q5, precision="fp64", lattice="d3q15", tuning=ONE) as s:
        s.set_fields(g=g)
        s.step(3)
        go, qo, po = d3q15.run(t64(g), t64(q5), t64(phi), p, 3)
        rho_o, u_o = d3q15.observe(go, qo, po, p)
        errs = field_errors(s.moments(), (rho_o.numpy(), u_o.numpy(), po.numpy(), qo.numpy()), p["rho0"])
        errs["g"] = rel_err(s.populations(), go.numpy())
    _check(errs)


def test_fp64_one_launch_droplet16_100_steps():
    p = inputs.params_for("droplet16")
    phi, q5 = inputs.workload_fields("droplet16")
    g = np.zeros((19,) + phi.shape)
    with Sim(p, phi, q5, precision="fp64", tuning=ONE) as s:
        s.step(100)
        go, qo, po = oracle_run(p, g, q5, phi, 100)
        rho_o, u_o = oracle_observe(p, go, qo, po)
        errs = field_errors(s.moments(), (rho_o, u_o, po, qo), p["rho0"])
        errs["g"] = rel_err(s.populations(), go)
    _check(errs)


@pytest.mark.parametrize("lattice", ["d3q19", "d3q15"])
def test_fp64_recording_step_one_launch_equals_two_launches(lattice):
    p = _p(q0=2 * math.pi / 9, zeta=0.01)
    g, phi, q5 = inputs.random_fields(34, 18, 11, seed=5, g_amp=2e-3, q_amp=0.2)
    if lattice == "d3q15":
        g = np.ascontiguousarray(g[:15])
    outs = []
    for tuning in (ONE, TWO):
        with Sim(p, phi, q5, precision="fp64", lattice=lattice, tuning=tuning) as s:
            s.set_fields(g=g)
            s.step(2)
            st = s.get_state()
            out = torch.zeros_like(st)  # zero-filled: the alignment gaps between parts compare equal
            rec = s.record_buffer().zero_()
            s.step_record(st, out, rec)
            lean = s.lean_record_buffer().zero_()
            s.set_state(st)
            s.step_record_lean(lean)
            g_next = s.populations()  # the context advanced by the lean recording step
            torch.cuda.synchronize()
            outs.append((out.cpu().numpy(), rec.cpu().numpy(), lean.cpu().numpy(), g_next))
    (o1, r1, l1, g1), (o2, r2, l2_, g2) = outs
    n8 = (o1.size // 8) * 8  # state: populations, Q, phi in float64, then the int64 step counter
    assert rel_err(o1[:n8].view(np.float64)[:-1], o2[:n8].view(np.float64)[:-1])[1] <= 1e-13
    assert np.array_equal(o1[-8:], o2[-8:])
    assert rel_err(r1, r2)[1] <= 1e-13
    assert rel_err(l1.view(np.float64), l2_.view(np.float64))[1] <= 1e-13
    assert rel_err(g1, g2)[1] <= 1e-13


@pytest.mark.parametrize("shape", [(34, 18, 11), (12, 6, 7), (64, 16, 5)])
@pytest.mark.parametrize("prec", ["fp32", "fp16s"])
@pytest.mark.parametrize("lattice", ["d3q19", "d3q15"])
def test_reduced_precision_one_launch_equals_two_launches(shape, prec, lattice):
    p = _p(q0=2 * math.pi / 9, zeta=0.01)
    g, phi, q5 = inputs.random_fields(*shape, seed=77, g_amp=2e-3, q_amp=0.2)
    if lattice == "d3q15":
        g = np.ascontiguousarray(g[:15])
    res = []
    for tuning in (ONE, None):
        with Sim(p, phi, q5, precision=prec, lattice=lattice, tuning=tuning) as s:
            names = list(s.profile(1))
            s.set_fields(g=g, phi=phi, q5=q5)  # back to the initial state after the profiled step
            s.step(4)
            res.append((names, s.moments(), s.populations()))
    (n1, m1, g1), (n2, m2, g2) = res
    assert n1 == ["k_step_fused"] and n2[0] == "k_lb_fused"
    # float16 storage: a different float32 rounding of g* can move a stored value by one
    # float16 step (2^-11 relative), so the bound is that resolution, not float32's
    tol = 2e-5 if prec == "fp32" else 2e-3
    for a, b in zip(m1, m2):
        l2, mx = rel_err(a, b)
        assert l2 < tol and mx < tol
    l2, mx = rel_err(g1, g2)
    assert l2 < tol and mx < tol
