"""GPU checks of the adjoint of the paper's own LB scheme (Sec. 3: D3Q15, the
symmetric stress in the equilibrium of Eqs. (9), (11), the antisymmetric stress
as the forcing term of Eq. (10)), through the C ABI, against the autograd of the
D3Q15 oracle step:

* one reverse step == the oracle's vector-Jacobian product (FP64, element by
  element, 1e-10 relative), with u, F recomputed and from a step record, on
  boxes of one tile and of ragged tiles on both in-plane axes;
* the same step in FP32 (1e-5 relative: float32 rounding of the forward values);
* a rollout's gradient w.r.t. zeta, q0 and the initial Q field == the oracle's
  autograd gradient of the same rollout, with checkpoints and with lean records.
"""
import math

import numpy as np
import pytest
import torch

from oracle import core, d3q15
from paper_2011_00287_amd import inputs
from paper_2011_00287_amd.autograd import displacement_loss
from paper_2011_00287_amd.sim import Sim

from helpers import rel_err

pytestmark = pytest.mark.gpu
DT = torch.float64


def _p(**kw):
    return dict(inputs.BASE_PARAMS, **kw)


def _oracle_vjp(p, g, q5, phi, ab_g, ab_q, ab_p):
    gt = torch.tensor(g, requires_grad=True)
    qt = torch.tensor(q5, requires_grad=True)
    pt = torch.tensor(phi, requires_grad=True)
    zt = torch.tensor(p["zeta"], dtype=DT, requires_grad=True)
    q0t = torch.tensor(p["q0"], dtype=DT, requires_grad=True)
    go, qo, pho = d3q15.step(gt, qt, pt, dict(p, zeta=zt, q0=q0t))
    s = (go * torch.tensor(ab_g)).sum() + (qo * torch.tensor(ab_q)).sum() + (pho * torch.tensor(ab_p)).sum()
    s.backward()
    return gt.grad.numpy(), qt.grad.numpy(), pt.grad.numpy(), float(zt.grad), float(q0t.grad)


def _inputs(shape, seed):
    nx, ny, nz = shape
    _, phi, q5 = inputs.random_fields(nx, ny, nz, seed=seed, q_amp=0.2)
    rng = np.random.default_rng(seed + 100)
    g = rng.uniform(-2e-3, 2e-3, (15, nz, ny, nx))
    ab = (rng.normal(size=g.shape), rng.normal(size=q5.shape), rng.normal(size=phi.shape))
    return g, phi, q5, ab


def _gpu_vjp(p, g, phi, q5, ab, precision, record):
    with Sim(p, phi, q5, precision=precision, lattice="d3q15") as sim:
        sim.set_fields(g=g)
        state = sim.get_state()
        adj = sim.adjoint_buffer()
        for part, a in zip(sim.adjoint_parts(adj), ab):
            part.copy_(torch.tensor(a, dtype=part.dtype))
        out = sim.adjoint_buffer()
        rec = None
        if record:
            rec = sim.record_buffer()
            sim.step_record(state, torch.empty_like(state), rec)
        zb, qb = sim.adjoint_step(state, adj, out, rec=rec)
        parts = tuple(t.double().cpu().numpy() for t in sim.adjoint_parts(out))
    return parts + (zb, qb)


@pytest.mark.parametrize("record", [False, True])
@pytest.mark.parametrize("shape", [(6, 5, 7), (34, 9, 5)])
def test_d3q15_single_step_vjp_matches_oracle(shape, record):
    """(34, 9, 5): FP64 tiles of 16 x 8 leave a two-column x tile and a one-row y tile."""
    p = _p(q0=2 * math.pi / 7, zeta=0.01)
    g, phi, q5, ab = _inputs(shape, seed=41 + shape[0])
    ref = _oracle_vjp(p, g, q5, phi, *ab)
    got = _gpu_vjp(p, g, phi, q5, ab, "fp64", record)
    for name, a, b in zip(("g", "q", "phi"), got[:3], ref[:3]):
        l2, mx = rel_err(a, b)
        assert l2 < 1e-10 and mx < 1e-10, (name, l2, mx)
    for a, b in zip(got[3:], ref[3:]):
        assert abs(a - b) <= 1e-10 * abs(b), (a, b)


def test_d3q15_single_step_vjp_fp32():
    p = _p(q0=2 * math.pi / 7, zeta=0.01)
    g, phi, q5, ab = _inputs((35, 10, 6), seed=77)
    ref = _oracle_vjp(p, g, q5, phi, *ab)
    got = _gpu_vjp(p, g, phi, q5, ab, "fp32", True)
    for name, a, b in zip(("g", "q", "phi"), got[:3], ref[:3]):
        l2, mx = rel_err(a, b)
        assert l2 < 1e-5 and mx < 1e-5, (name, l2, mx)
    for a, b in zip(got[3:], ref[3:]):
        assert abs(a - b) <= 1e-4 * abs(b), (a, b)


def _oracle_rollout_grad(p, phi, q5, steps):
    qt = torch.tensor(q5, requires_grad=True)
    zt = torch.tensor(p["zeta"], dtype=DT, requires_grad=True)
    q0t = torch.tensor(p["q0"], dtype=DT, requires_grad=True)
    po = dict(p, zeta=zt, q0=q0t)
    phit = torch.tensor(phi)
    zc0 = core.centre_linear(phit)[2].detach()
    g = torch.zeros((15,) + phi.shape, dtype=DT)
    g, q, ph = d3q15.run(g, qt, phit, po, steps)
    L = core.displacement_loss(ph, zc0)
    L.backward()
    return float(L.detach()), float(zt.grad), float(q0t.grad), qt.grad.numpy()


@pytest.mark.parametrize("checkpoint", [3, 0])
def test_d3q15_rollout_gradient_matches_oracle_autograd(checkpoint):
    p = _p(q0=2 * math.pi / 8, zeta=0.02)
    phi, q5 = inputs.droplet_fields(8, 8, 10, 2.5, p["q0"], seed=3)
    steps = 7
    L_o, dz_o, dq0_o, dq5_o = _oracle_rollout_grad(p, phi, q5, steps)
    zeta = torch.tensor(p["zeta"], dtype=DT, requires_grad=True)
    q0 = torch.tensor(p["q0"], dtype=DT, requires_grad=True)
    q5t = torch.tensor(q5, requires_grad=True)
    L = displacement_loss(zeta, q0, q5t, params=p, phi=phi, steps=steps, checkpoint=checkpoint,
                          precision="fp64", lattice="d3q15")
    L.backward()
    assert abs(float(L.detach()) - L_o) <= 1e-12 * abs(L_o)
    assert abs(float(zeta.grad) - dz_o) <= 1e-9 * abs(dz_o)
    assert abs(float(q0.grad) - dq0_o) <= 1e-9 * abs(dq0_o)
    l2, mx = rel_err(q5t.grad.numpy(), dq5_o)
    assert l2 < 1e-9 and mx < 1e-9, (l2, mx)
