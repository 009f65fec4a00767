"""GPU checks of the adjoint of the paper's finite-difference integrator (Sec. 3:
Heun predictor-corrector, first-order upwind advection, fourth-order stencils;
M = 0.05), through the C ABI, against the autograd of the pc4 oracle step:

* one reverse step == the oracle's vector-Jacobian product (FP64, element by
  element, 1e-10 relative), with u, F recomputed and from a step record, on
  boxes of one tile and of ragged tiles on both in-plane axes;
* the same with the paper's D3Q15 LB scheme underneath (the paper's full
  scheme), and in FP32 (1e-5 relative);
* a rollout's gradient w.r.t. zeta, q0 and the initial Q field == the oracle's
  autograd gradient of the same rollout, with checkpoints and with lean records;
* the 32^3 droplet over 400 steps (checkpoints every 20), D3Q19 and D3Q15,
  FP64: the gradient against central differences.

The inputs are random states with flow, so no velocity (or face velocity) is
exactly zero: there the upwind switch has a kink, whose w-derivative the
reverse takes as the sum of both one-sided parts, as the oracle's clamp form
does under autograd.
"""
import math

import numpy as np
import pytest
import torch

from oracle import core, d3q15, pc4
from paper_2011_00287_amd import inputs
from paper_2011_00287_amd.autograd import displacement_loss
from paper_2011_00287_amd.sim import Sim

from helpers import rel_err

pytestmark = pytest.mark.gpu
DT = torch.float64


def _p(**kw):
    return dict(inputs.BASE_PARAMS, **dict(dict(M=0.05), **kw))


def _step15_pc4(g, q5, phi, p):
    """The paper's LB scheme (D3Q15) followed by the paper's order-parameter integrator."""
    Q = core.q_full(q5)
    _, _, S, F = d3q15.thermo(phi, Q, p)
    rho, u = d3q15.moments(g, F, p)
    g1 = d3q15.stream(d3q15.collide(g, u, rho, S, F, p))
    Q1, phi1 = pc4.update_pc(Q, phi, u, p)
    return g1, core.q5_of(Q1), phi1


def _oracle_vjp(step, p, g, q5, phi, ab):
    gt = torch.tensor(g, requires_grad=True)
    qt = torch.tensor(q5, requires_grad=True)
    pt = torch.tensor(phi, requires_grad=True)
    zt = torch.tensor(p["zeta"], dtype=DT, requires_grad=True)
    q0t = torch.tensor(p["q0"], dtype=DT, requires_grad=True)
    go, qo, pho = step(gt, qt, pt, dict(p, zeta=zt, q0=q0t))
    s = (go * torch.tensor(ab[0])).sum() + (qo * torch.tensor(ab[1])).sum() + (pho * torch.tensor(ab[2])).sum()
    s.backward()
    return gt.grad.numpy(), qt.grad.numpy(), pt.grad.numpy(), float(zt.grad), float(q0t.grad)


def _inputs(shape, nq, seed):
    nx, ny, nz = shape
    _, phi, q5 = inputs.random_fields(nx, ny, nz, seed=seed, q_amp=0.2)
    rng = np.random.default_rng(seed + 100)
    g = rng.uniform(-2e-3, 2e-3, (nq, nz, ny, nx))
    ab = (rng.normal(size=g.shape), rng.normal(size=q5.shape), rng.normal(size=phi.shape))
    return g, phi, q5, ab


def _gpu_vjp(p, g, phi, q5, ab, precision, lattice, record, tuning=None):
    with Sim(p, phi, q5, precision=precision, lattice=lattice, fd_scheme="pc4", tuning=tuning) as sim:
        sim.set_fields(g=g)
        state = sim.get_state()
        adj = sim.adjoint_buffer()
        for part, a in zip(sim.adjoint_parts(adj), ab):
            part.copy_(torch.tensor(a, dtype=part.dtype))
        out = sim.adjoint_buffer()
        rec = None
        if record:
            rec = sim.record_buffer()
            nxt = torch.empty_like(state)
            sim.step_record(state, nxt, rec)
            # the recording step is an ordinary pc4 step
            sim.set_state(state)
            sim.step(1)
            ref = sim.moments() + (sim.populations(),)
            sim.set_state(nxt)
            for a, b in zip(ref, sim.moments() + (sim.populations(),)):
                assert np.array_equal(a, b)
        zb, qb = sim.adjoint_step(state, adj, out, rec=rec)
        parts = tuple(t.double().cpu().numpy() for t in sim.adjoint_parts(out))
    return parts + (zb, qb)


def _check(got, ref, tol, ptol):
    for name, a, b in zip(("g", "q", "phi"), got[:3], ref[:3]):
        l2, mx = rel_err(a, b)
        assert l2 < tol and mx < tol, (name, l2, mx)
    for a, b in zip(got[3:], ref[3:]):
        assert abs(a - b) <= ptol * abs(b), (a, b)


@pytest.mark.parametrize("record", [False, True])
@pytest.mark.parametrize("shape", [(6, 5, 7), (34, 9, 5)])
def test_pc4_single_step_vjp_matches_oracle(shape, record):
    """(34, 9, 5): tiles of 16 x 8 (FP64) leave a two-column x tile and a one-row y tile."""
    p = _p(q0=2 * math.pi / 7, zeta=0.01)
    g, phi, q5, ab = _inputs(shape, 19, seed=51 + shape[0])
    ref = _oracle_vjp(pc4.step, p, g, q5, phi, ab)
    _check(_gpu_vjp(p, g, phi, q5, ab, "fp64", "d3q19", record), ref, 1e-10, 1e-10)


@pytest.mark.parametrize("record", [False, True])
def test_d3q15_pc4_single_step_vjp_matches_oracle(record):
    """The paper's full scheme: D3Q15 LB with the pc4 order-parameter integrator."""
    p = _p(q0=2 * math.pi / 7, zeta=0.01)
    g, phi, q5, ab = _inputs((9, 7, 6), 15, seed=63)
    ref = _oracle_vjp(_step15_pc4, p, g, q5, phi, ab)
    _check(_gpu_vjp(p, g, phi, q5, ab, "fp64", "d3q15", record), ref, 1e-10, 1e-10)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_d3q15_pc4_multi_tile_vjp_matches_oracle(prec, tol):
    """The paper's full scheme on a box of several ragged tiles along x and y
    (the stress reverse, compiled without the Euler update's seeds, with its
    tile-face terms, and the one-kernel Heun products), in FP64 and FP32."""
    p = _p(q0=2 * math.pi / 7, zeta=0.01)
    g, phi, q5, ab = _inputs((35, 19, 6), 15, seed=67)
    ref = _oracle_vjp(_step15_pc4, p, g, q5, phi, ab)
    _check(_gpu_vjp(p, g, phi, q5, ab, prec, "d3q15", True), ref, tol, 10 * tol)


# Boxes whose tiles exercise the one-kernel product of the reverse (tiles of
# 32 x 16 in float, 16 x 16 in double): several tiles along both in-plane
# axes, ragged last tiles two and more sites wide (the terms owed across a
# tile face reach two sites: in a tile two or three sites wide a column or
# row receives from both faces), a lone tile along one axis wrapping inside
# itself.
FUSED_SHAPES = [(70, 20, 9), (36, 18, 7), (34, 10, 6), (18, 12, 5), (40, 6, 7), (20, 40, 5), (35, 19, 6)]


@pytest.mark.parametrize("shape", FUSED_SHAPES)
def test_pc4_fused_product_vjp_matches_oracle(shape):
    p = _p(q0=2 * math.pi / 7, zeta=0.01)
    g, phi, q5, ab = _inputs(shape, 19, seed=91 + shape[0] + shape[1])
    ref = _oracle_vjp(pc4.step, p, g, q5, phi, ab)
    _check(_gpu_vjp(p, g, phi, q5, ab, "fp64", "d3q19", True), ref, 1e-10, 1e-10)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", FUSED_SHAPES + [(33, 9, 5), (34, 17, 6)])
def test_pc4_fused_product_equals_site_parallel_product(shape, prec):
    """pc_adj = 0 (one z-marching kernel per Heun product where the tiling
    allows it) against pc_adj = 1 (the site-parallel kernels); (33, 9, 5) and
    (34, 17, 6) leave a one-column or one-row edge tile, where both settings
    run the site-parallel kernels."""
    p = _p(q0=2 * math.pi / 7, zeta=0.01)
    g, phi, q5, ab = _inputs(shape, 19, seed=17 + shape[0])
    a = _gpu_vjp(p, g, phi, q5, ab, prec, "d3q19", True, tuning={"pc_adj": 0})
    b = _gpu_vjp(p, g, phi, q5, ab, prec, "d3q19", True, tuning={"pc_adj": 1})
    tol = 1e-13 if prec == "fp64" else 2e-5
    _check(a, b, tol, tol)


@pytest.mark.parametrize("adj_tile", [0, 1])
def test_pc4_single_step_vjp_fp32(adj_tile):
    """adj_tile 0: the default 32 x 16 stress-adjoint tile; 1: 32 x 8."""
    p = _p(q0=2 * math.pi / 7, zeta=0.01)
    g, phi, q5, ab = _inputs((35, 10, 6), 19, seed=78)
    ref = _oracle_vjp(pc4.step, p, g, q5, phi, ab)
    _check(_gpu_vjp(p, g, phi, q5, ab, "fp32", "d3q19", True, tuning={"adj_tile": adj_tile}), ref, 1e-5, 1e-4)


def _oracle_rollout_grad(p, phi, q5, steps):
    qt = torch.tensor(q5, requires_grad=True)
    zt = torch.tensor(p["zeta"], dtype=DT, requires_grad=True)
    q0t = torch.tensor(p["q0"], dtype=DT, requires_grad=True)
    po = dict(p, zeta=zt, q0=q0t)
    phit = torch.tensor(phi)
    zc0 = core.centre_linear(phit)[2].detach()
    g = torch.zeros((19,) + phi.shape, dtype=DT)
    g, q, ph = pc4.run(g, qt, phit, po, steps)
    L = core.displacement_loss(ph, zc0)
    L.backward()
    return float(L.detach()), float(zt.grad), float(q0t.grad), qt.grad.numpy()


@pytest.mark.parametrize("checkpoint", [3, 0])
def test_pc4_rollout_gradient_matches_oracle_autograd(checkpoint):
    p = _p(q0=2 * math.pi / 8, zeta=0.02)
    phi, q5 = inputs.droplet_fields(8, 8, 10, 2.5, p["q0"], seed=3)
    steps = 7
    L_o, dz_o, dq0_o, dq5_o = _oracle_rollout_grad(p, phi, q5, steps)
    zeta = torch.tensor(p["zeta"], dtype=DT, requires_grad=True)
    q0 = torch.tensor(p["q0"], dtype=DT, requires_grad=True)
    q5t = torch.tensor(q5, requires_grad=True)
    L = displacement_loss(zeta, q0, q5t, params=p, phi=phi, steps=steps, checkpoint=checkpoint,
                          precision="fp64", fd_scheme="pc4")
    L.backward()
    # L = (z_c(T) - z_c(0))^2 with z_c ~ 5 and a displacement ~ 1e-3: float64
    # rounding of the centre (1e-15 relative) is amplified ~ 1e4 in L
    assert abs(float(L.detach()) - L_o) <= 1e-10 * abs(L_o)
    assert abs(float(zeta.grad) - dz_o) <= 1e-9 * abs(dz_o)
    assert abs(float(q0.grad) - dq0_o) <= 1e-9 * abs(dq0_o)
    l2, mx = rel_err(q5t.grad.numpy(), dq5_o)
    assert l2 < 1e-9 and mx < 1e-9, (l2, mx)


def _pc4_loss(p, phi, q5, steps, lattice):
    with Sim(p, phi, q5, precision="fp64", lattice=lattice, fd_scheme="pc4") as s:
        zc0 = s.centre()[0][2]
        s.step(steps)
        zc = s.centre()[0][2]
    return (zc - zc0) ** 2


@pytest.mark.parametrize("lattice", ["d3q19", "d3q15"])
def test_droplet32_pc4_adjoint_vs_central_differences(lattice):
    """The 32^3 droplet (400 steps, checkpoints every 20) with the pc4 integrator
    (M = 0.05), on the D3Q19 and on the paper's D3Q15 scheme, in FP64: dL/dzeta,
    dL/dq0 and five Q entries inside the droplet against central differences of
    the forward rollout, each within 1e-4 of its difference quotient.  (In FP32
    the gradients of this small-displacement loss differ from FP64's by up to a
    few 1e-4, and by more for q0's small gradient, as the Euler integrator's do
    at the same mobility: the rounding of the FP32 trajectory; the FP32 reverse
    step itself is held to the oracle's VJP above.)

    The first-order upwind switch makes the loss only piecewise smooth in the
    parameters: a velocity that changes sign at some site and step puts a kink
    in L(zeta), and a central difference with step h averages the slopes of the
    kinks it straddles.  On this rollout, with h = 1e-6, that leaves a few 1e-5
    between the quotient for zeta and the adjoint, and the quotient converges
    to the adjoint as h shrinks (1e-6 at h = 1e-8) until its own rounding noise
    (~1e-17 absolute in L) dominates; zeta therefore takes h = 1e-8.  q0's
    gradient is small (~5e-7), so its quotient is noise-limited below
    h = 1e-6 and takes that step.  The Q entries take h = 1e-6 with a floor of
    three times the quotients' change from h to 2h, as in the Euler rollout
    check."""
    from paper_2011_00287_amd.autograd import backward_segments, run_segments
    w = inputs.WORKLOADS["droplet32_adjoint"]
    p = inputs.params_for("droplet32_adjoint", M=0.05)
    phi, q5 = inputs.workload_fields("droplet32_adjoint")
    steps, ck = w["steps"], w["checkpoint"]
    with Sim(p, phi, q5, precision="fp64", lattice=lattice, fd_scheme="pc4") as sim:
        zc0 = sim.centre()[0][2]
        ckpts = run_segments(sim, steps, ck)
        adj = sim.adjoint_buffer()
        L = sim.seed_centre(zc0, adj)
        dz, dq0 = backward_segments(sim, ckpts, steps, ck, adj)
        _, qbar, _ = sim.adjoint_parts(adj)
        qbar = qbar.double().cpu().numpy()
    assert L > 0
    hz, hq = 1e-8, 1e-6
    fd_z = (_pc4_loss(dict(p, zeta=p["zeta"] + hz), phi, q5, steps, lattice) -
            _pc4_loss(dict(p, zeta=p["zeta"] - hz), phi, q5, steps, lattice)) / (2 * hz)
    fd_q0 = (_pc4_loss(dict(p, q0=p["q0"] + hq), phi, q5, steps, lattice) -
             _pc4_loss(dict(p, q0=p["q0"] - hq), phi, q5, steps, lattice)) / (2 * hq)
    print(lattice, "zeta ad", dz, "fd", fd_z, "q0 ad", dq0, "fd", fd_q0)
    assert abs(dz - fd_z) <= 1e-4 * abs(fd_z), (dz, fd_z)
    assert abs(dq0 - fd_q0) <= 1e-4 * abs(fd_q0), (dq0, fd_q0)
    rng = np.random.default_rng(1)
    inside = np.argwhere(phi > p["phi_cr"])
    picks = inside[rng.choice(len(inside), 5, replace=False)]
    comps = rng.integers(0, 5, 5)

    def fd_q(c, z, y, x, hh):
        qp = q5.copy()
        qm = q5.copy()
        qp[c, z, y, x] += hh
        qm[c, z, y, x] -= hh
        return (_pc4_loss(p, phi, qp, steps, lattice) - _pc4_loss(p, phi, qm, steps, lattice)) / (2 * hh)

    ads, fds, fds2 = [], [], []
    for (z, y, x), c in zip(picks, comps):
        fds.append(fd_q(c, z, y, x, hq))
        fds2.append(fd_q(c, z, y, x, 2 * hq))
        ads.append(qbar[c, z, y, x])
    ads, fds, fds2 = np.array(ads), np.array(fds), np.array(fds2)
    noise = np.abs(fds - fds2).max()
    ratio = np.abs(ads - fds) / (1e-4 * np.abs(fds) + 3 * noise)
    print("Q entries: ad", ads, "fd", fds, "fd noise", noise, "worst |ad - fd| / bound", ratio.max())
    assert np.all(ratio <= 1.0), (ads, fds, ratio)
