"""Pins of the oracle's second LB scheme (the paper's, Sec. 3): D3Q15 with the
symmetric stress in the equilibrium (Eqs. (9), (11)) and the antisymmetric stress
as a forcing term (Eq. (10)).

* the D3Q15 tables: normalisation, isotropy up to fourth order, opposites;
* the equilibrium's moments are exactly those of Eqs. (8)-(9): sum f = rho,
  sum c f = rho u, sum c c f = rho/3 I + rho u u - S;
* the Guo source's moments;
* a stress in the equilibrium reaches the momentum, after one collide-and-stream
  from equilibrium at rest, as the central difference of S (closed form for a
  sinusoidal shear and normal stress);
* exact mass and momentum conservation on a periodic box, the uniform body
  force closed form, and the shear-wave viscosity (tau - 1/2)/3.
"""
import math

import numpy as np
import pytest
import torch

from oracle import core, d3q15
from paper_2011_00287_amd import inputs

DT = torch.float64


def _p(**kw):
    return dict(inputs.BASE_PARAMS, **kw)


def test_d3q15_tables():
    c = np.array(d3q15.C15, dtype=float)
    w = np.array(d3q15.W15)
    I = np.eye(3)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(np.einsum("i,ia->a", w, c), 0.0, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), I / 3.0, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib,ig->abg", w, c, c, c), 0.0, atol=1e-15)
    iso4 = (np.einsum("ab,gd->abgd", I, I) + np.einsum("ag,bd->abgd", I, I) + np.einsum("ad,bg->abgd", I, I)) / 9.0
    assert np.allclose(np.einsum("i,ia,ib,ig,id->abgd", w, c, c, c, c), iso4, atol=1e-15)
    for i, j in enumerate(d3q15.OPP15):
        assert np.array_equal(c[i], -c[j])
    assert len({tuple(v) for v in c}) == 15


def _random_state(shape, seed):
    rng = np.random.default_rng(seed)
    rho = torch.tensor(1.0 + 0.05 * rng.standard_normal(shape))
    u = torch.tensor(0.05 * rng.standard_normal((3,) + shape))
    S = rng.standard_normal((3, 3) + shape) * 0.01
    S = torch.tensor(0.5 * (S + S.transpose(1, 0, *range(2, S.ndim))))
    F = torch.tensor(1e-3 * rng.standard_normal((3,) + shape))
    return rho, u, S, F


def test_equilibrium_moments_with_stress():
    p = _p()
    rho, u, S, _ = _random_state((4, 3, 5), 1)
    g = d3q15.equilibrium_dev(rho, u, S, p)
    c, w = d3q15._c(), d3q15._w()
    f = g + w.reshape(15, 1, 1, 1) * p["rho0"]
    assert torch.allclose(f.sum(0), rho, atol=1e-14)
    assert torch.allclose(torch.einsum("ia,i...->a...", c, f), rho * u, atol=1e-14)
    m2 = torch.einsum("ia,ib,i...->ab...", c, c, f)
    want = rho / 3.0 * torch.eye(3, dtype=DT).reshape(3, 3, 1, 1, 1) + rho * torch.einsum("a...,b...->ab...", u, u) - S
    assert torch.allclose(m2, want, atol=1e-14)


def test_guo_source_moments():
    p = _p()
    _, u, _, F = _random_state((3, 4, 2), 2)
    src = d3q15.guo_source(u, F, p)
    c = d3q15._c()
    k = 1.0 - 0.5 / p["tau"]
    assert torch.allclose(src.sum(0), torch.zeros_like(src[0]), atol=1e-17)
    assert torch.allclose(torch.einsum("ia,i...->a...", c, src), k * F, atol=1e-16)
    m2 = torch.einsum("ia,ib,i...->ab...", c, c, src)
    want = k * (torch.einsum("a...,b...->ab...", u, F) + torch.einsum("a...,b...->ab...", F, u))
    assert torch.allclose(m2, want, atol=1e-16)


@pytest.mark.parametrize("comp", [(0, 2), (0, 0), (1, 2)])
def test_stress_reaches_momentum_as_central_difference(comp):
    """S_ab(r) = s sin(k r_b) (+ its transpose), u = 0, g at its equilibrium: after one
    collide-and-stream the momentum is sum_b D0_b S_ab, i.e. s sin(k) cos(k r_b), exactly."""
    a, b = comp
    p = _p()
    n = 12
    k = 2 * math.pi * 2 / n
    s = 3e-3
    shape = (n, n, n)
    coord = torch.arange(n, dtype=DT)
    prof = [coord.reshape(1, 1, n), coord.reshape(1, n, 1), coord.reshape(n, 1, 1)][b]  # x, y, z index
    S = torch.zeros((3, 3) + shape, dtype=DT)
    S[a, b] = s * torch.sin(k * prof).expand(shape)
    S[b, a] = S[a, b]
    rho = torch.full(shape, p["rho0"], dtype=DT)
    u = torch.zeros((3,) + shape, dtype=DT)
    g = d3q15.equilibrium_dev(rho, u, S, p)
    g1 = d3q15.stream(d3q15.collide(g, u, rho, S, torch.zeros_like(u), p))
    mom = torch.einsum("ia,i...->a...", d3q15._c(), g1)
    want = torch.zeros_like(mom)  # S_ba depends on r_b only, so the b-component (a != b) is zero
    want[a] = s * math.sin(k) * torch.cos(k * prof).expand(shape)
    assert torch.allclose(mom, want, atol=1e-16)


def test_random_state_conserves_mass_and_momentum():
    p = _p(q0=2 * math.pi / 7, zeta=0.02)
    g, phi, q5 = inputs.random_fields(6, 5, 7, seed=8, g_amp=2e-3, q_amp=0.2)
    g = torch.tensor(g[:15])
    phi, q5 = torch.tensor(phi), torch.tensor(q5)
    m0 = float(g.sum())
    j0 = torch.einsum("ia,i...->a", d3q15._c(), g)
    g1, q1, p1 = d3q15.step(g, q5, phi, p)
    assert abs(float(g1.sum()) - m0) < 1e-14
    j1 = torch.einsum("ia,i...->a", d3q15._c(), g1)
    _, _, _, F = d3q15.thermo(phi, core.q_full(q5), p)
    assert torch.allclose(F.sum((1, 2, 3)), torch.zeros(3, dtype=DT), atol=1e-14)
    assert torch.allclose(j1, j0, atol=1e-14)
    assert abs(float(p1.sum()) - float(phi.sum())) < 1e-12


def test_uniform_body_force_closed_form():
    p = _p(zeta=0.0, body_force=(2e-6, -1e-6, 5e-7))
    shape = (5, 4, 6)
    n = 5 * 4 * 6
    g = d3q15.init_populations(torch.zeros((3,) + shape, dtype=DT), p)
    phi = torch.zeros(shape, dtype=DT)
    q5 = torch.zeros((5,) + shape, dtype=DT)
    t = 9
    g, q5, phi = d3q15.run(g, q5, phi, p, t)
    rho, u = d3q15.observe(g, q5, phi, p)
    mom = (rho * u).sum((1, 2, 3))
    want = torch.tensor(p["body_force"], dtype=DT) * n * (t + 0.5)
    assert torch.allclose(mom, want, rtol=1e-12, atol=0)


def test_shear_wave_viscosity():
    """u_x = U0 sin(2 pi z / n) of the bare fluid (Q = phi = 0 held, free-energy constants 0)
    decays at the rate nu k^2 per step, nu = (tau - 1/2)/3 (n = 64: within 1.5 %)."""
    p = _p(A0=0.0, a=0.0, k_phi=0.0, K=0.0, W=0.0, zeta=0.0)
    n, U0 = 64, 1e-6
    shape = (n, 2, 2)
    z = torch.arange(n, dtype=DT).reshape(n, 1, 1)
    sinz = torch.sin(2 * math.pi * z / n)
    u0 = torch.zeros((3,) + shape, dtype=DT)
    u0[0] = U0 * sinz.expand(shape)
    g = d3q15.init_populations(u0, p)
    phi = torch.zeros(shape, dtype=DT)
    q5 = torch.zeros((5,) + shape, dtype=DT)
    amps = []
    for _ in range(61):
        _, u = d3q15.observe(g, q5, phi, p)
        amps.append(float((u[0] * sinz).sum()))
        g, _, _ = d3q15.step(g, q5, phi, p)
    rate = -math.log(amps[-1] / amps[-21]) / 20
    nu = (p["tau"] - 0.5) / 3.0
    assert abs(rate / (nu * (2 * math.pi / n) ** 2) - 1.0) < 0.015, rate
