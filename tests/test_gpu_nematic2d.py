"""GPU parity of the 2D bulk active nematic (D2Q9 + 2x2 Q tensor) against the
FP64 oracle of that model, through the C ABI (include/lb_nematic2d.h), and the
activity regimes of Fig. 4 (qualitative).

FP64: 1e-12 relative per field for g, u and Q, as for the 3D step.  rho is
reported near rho0 = 1 while rho - rho0 = sum g is ~1e-5 here, so it is checked
against rho0 + sum g to a few units of the last place of 1 (rho - rho0 itself is
carried by g).  FP32: an accuracy statement against FP64."""
import math

import numpy as np
import pytest
import torch

from oracle import nematic2d as n2
from paper_2011_00287_amd import inputs
from paper_2011_00287_amd._lib import LB_EINVAL, LbError
from paper_2011_00287_amd.sim2d import Nematic2D

from helpers import rel_err, t64

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _p(**kw):
    return dict(inputs.NEMATIC2D_PARAMS, **kw)


def _random(nx, ny, seed):
    rng = np.random.default_rng(seed)
    g = 2e-3 * rng.standard_normal((9, ny, nx))
    q2 = rng.uniform(-0.3, 0.3, (2, ny, nx))
    return g, q2


def _compare(sim, p, g, q2, tol=TOL64):
    _, u_o = n2.observe(t64(g), t64(q2), p)
    rho, u, q = sim.moments()
    errs = {"u": rel_err(u, u_o.numpy()), "Q": rel_err(q, q2), "g": rel_err(sim.populations(), g)}
    bad = {k: v for k, v in errs.items() if not (v[0] <= tol and v[1] <= tol)}
    assert not bad, errs
    assert float(np.abs(rho - (p["rho0"] + g.sum(0))).max()) <= 4.5e-16


@pytest.mark.parametrize("shape", [(4, 4), (5, 3), (7, 6), (33, 9), (40, 19), (70, 35)])
def test_fp64_random_state_parity(shape):
    nx, ny = shape
    p = _p(zeta=0.01, body_force=(1e-5, -2e-5))
    g, q2 = _random(nx, ny, nx * 10 + ny)
    with Nematic2D(p, q2, precision="fp64") as s:
        s.set_fields(g=g)
        _compare(s, p, g, q2)
        s.step(3)
        go, qo = n2.run(t64(g), t64(q2), p, 3)
        _compare(s, p, go.numpy(), qo.numpy())


def test_fp64_nematic64_200_steps():
    p = inputs.nematic2d_params("nematic64")
    q2 = inputs.nematic2d_workload_fields("nematic64")
    g = np.zeros((9,) + q2.shape[1:])
    with Nematic2D(p, q2, precision="fp64") as s:
        s.step(200)
        go, qo = n2.run(t64(g), t64(q2), p, 200)
        _compare(s, p, go.numpy(), qo.numpy())


@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("fp32", 1e-5)])
def test_nematic512_full_box_vs_oracle(prec, tol):
    """The 512^2 workload of the benchmark (zeta = 0.02), in its launch configuration:
    10 steps from a random state with flow, every site against the FP64 oracle
    (FP64: 1e-12 relative per field; FP32: float32 rounding of 10 steps)."""
    p = inputs.nematic2d_params("nematic512")
    q2 = inputs.nematic2d_workload_fields("nematic512")
    rng = np.random.default_rng(512)
    g = 1e-3 * rng.standard_normal((9,) + q2.shape[1:])
    with Nematic2D(p, q2, precision=prec) as s:
        s.set_fields(g=g)
        s.step(10)
        go, qo = n2.run(t64(g), t64(q2), p, 10)
        if prec == "fp64":
            _compare(s, p, go.numpy(), qo.numpy())
        else:
            _, u_o = n2.observe(go, qo, p)
            _, u, q = s.moments()
            for name, a, b in (("g", s.populations(), go.numpy()), ("u", u, u_o.numpy()), ("Q", q, qo.numpy())):
                l2, mx = rel_err(a, b)
                assert l2 <= tol and mx <= tol, (name, l2, mx)


def test_init_with_velocity_and_totals():
    p = _p(zeta=0.01)
    ny, nx = 12, 10
    _, y = np.meshgrid(np.arange(nx), np.arange(ny))
    u0 = np.zeros((2, ny, nx))
    u0[0] = 1e-3 * np.sin(2 * np.pi * y / ny)
    q2 = inputs.nematic_fields(nx, ny, 0.4, 0.3, seed=2)
    geq = n2.equilibrium_dev(torch.full((ny, nx), p["rho0"], dtype=torch.float64), t64(u0), p).numpy()
    with Nematic2D(p, q2, u0=u0) as s:
        l2, mx = rel_err(s.populations(), geq)
        assert l2 < 1e-15 and mx < 1e-15
        s.step(5)
        t = s.totals()
        g, q = s.populations(), s.q()
    o = n2.totals(t64(g), t64(q), p)
    assert abs(t["mass"] - o["mass"]) <= 1e-13 * o["mass"]
    assert abs(t["free_energy"] - o["free_energy"]) <= 1e-12 * abs(o["free_energy"])
    assert abs(t["kinetic_energy"] - o["kinetic_energy"]) <= 1e-11 * o["kinetic_energy"]
    for a in range(2):
        assert abs(t["momentum"][a] - o["momentum"][a]) <= 1e-12 * max(1e-12, abs(o["momentum"][a])) + 1e-15
    assert t["step"] == 5


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-6)])
def test_conservation(prec, tol):
    p = inputs.nematic2d_params("nematic64", zeta=0.02)
    q2 = inputs.nematic2d_workload_fields("nematic64")
    with Nematic2D(p, q2, precision=prec) as s:
        t0 = s.totals()
        s.step(500)
        t1 = s.totals()
    assert abs(t1["mass"] - t0["mass"]) <= tol * t0["mass"]
    for a in range(2):
        assert abs(t1["momentum"][a] - t0["momentum"][a]) <= tol * t0["mass"]


def test_fp32_accuracy_nematic64():
    p = inputs.nematic2d_params("nematic64")
    q2 = inputs.nematic2d_workload_fields("nematic64")
    with Nematic2D(p, q2, precision="fp64") as a, Nematic2D(p, q2, precision="fp32") as b:
        a.step(200)
        b.step(200)
        ra, rb = a.moments(), b.moments()
    assert rel_err(rb[2], ra[2])[0] < 1e-5
    assert rel_err(rb[1], ra[1])[0] < 1e-3


def test_rejected():
    with pytest.raises(LbError) as e:
        Nematic2D(_p(), np.zeros((2, 4, 4)), precision="fp16s")
    assert e.value.status == LB_EINVAL
    with Nematic2D(_p(), np.zeros((2, 5, 5))) as s:
        with pytest.raises(LbError) as e:
            s.step(-1)
        assert e.value.status == LB_EINVAL
        assert list(s.profile(2)) == ["k2_lb", "k2_order"]


def _run_regime(workload, steps=10000):
    w = inputs.NEMATIC2D_WORKLOADS[workload]
    p = inputs.nematic2d_params(workload)
    q2 = inputs.nematic2d_workload_fields(workload)
    E, nd = [], []
    with Nematic2D(p, q2, precision="fp32") as s:
        for _ in range(10):
            s.step(steps // 10)
            E.append(s.totals()["kinetic_energy"] / s.n_sites)
            nd.append(int((n2.defect_charges(torch.tensor(s.q())).abs() > 0.25).sum()))
    return E, nd


def test_regime_quiescent():
    """Below the finite-box threshold (64^2, zeta = 0.0005): the flow stirred by the
    initial noise decays and the nematic stays free of defects (Fig. 4a)."""
    E, nd = _run_regime("quiescent64")
    assert E[-1] < E[1] and E[-1] < 1e-10, E
    assert max(nd) == 0


def test_regime_spontaneous_flow():
    """zeta = 0.002 on 128^2: a self-sustained stationary flow without defects (Fig. 4b)."""
    E, nd = _run_regime("flow128")
    assert 1e-6 < E[-1] < 1e-4, E
    assert abs(E[-1] / E[-2] - 1) < 0.05, E
    assert max(nd) == 0


def test_regime_chaotic():
    """zeta = 0.02 on 128^2: active turbulence with +-1/2 defects (Fig. 4c)."""
    E, nd = _run_regime("chaos128")
    assert E[-1] > 1e-4, E
    assert min(nd[3:]) >= 10, nd

