"""Pins of the oracle's lattice-Boltzmann part against closed forms and invariants.

D3Q19 moment identities, Guo forcing moments (the conditions of Eq. (10) with
the whole stress as a body force), exact conservation (Eq. (8)), the closed
form of a uniform body force, and a shear wave against the exact eigenvalue of
the linearised 19x19 BGK operator and against the analytic viscosity
nu = (tau - 1/2)/3 (Sec. 3: tau sets the viscosity).
"""
import math

import numpy as np
import pytest
import torch

from oracle import core
from oracle.lattice import C19, OPP, W19
from paper_2011_00287_amd import inputs

DT = torch.float64


def test_lattice_tables():
    c = np.array(C19, dtype=float)
    w = np.array(W19)
    assert len(C19) == 19 and len(set(C19)) == 19
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w @ c, 0.0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(3) / 3, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0.0, atol=1e-16)
    d = np.eye(3)
    iso4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso4, atol=1e-16)
    for i in range(19):
        assert tuple(-x for x in C19[i]) == C19[OPP[i]]
        if i:
            assert OPP[i] == (i + 1 if i % 2 else i - 1)


def _rand(shape, seed, amp):
    return torch.tensor(np.random.default_rng(seed).uniform(-amp, amp, shape), dtype=DT)


def test_equilibrium_moments():
    p = dict(inputs.BASE_PARAMS)
    sh = (3, 4, 5)
    rho = 1.0 + _rand(sh, 1, 0.05)
    u = _rand((3,) + sh, 2, 0.1)
    geq = core.equilibrium_dev(rho, u, p)
    c = torch.tensor(C19, dtype=DT)
    w = torch.tensor(W19, dtype=DT).reshape(19, 1, 1, 1)
    feq = geq + w * p["rho0"]
    assert torch.allclose(geq.sum(0), rho - p["rho0"], atol=1e-15, rtol=0)
    assert torch.allclose(torch.einsum("ia,i...->a...", c, geq), rho * u, atol=1e-15, rtol=0)
    pi = torch.einsum("ia,ib,i...->ab...", c, c, feq)
    expect = rho * torch.eye(3, dtype=DT).reshape(3, 3, 1, 1, 1) / 3 + rho * torch.einsum("a...,b...->ab...", u, u)
    assert torch.allclose(pi, expect, atol=1e-15, rtol=0)


def test_guo_moments():
    p = dict(inputs.BASE_PARAMS)
    sh = (3, 3, 4)
    u = _rand((3,) + sh, 3, 0.1)
    F = _rand((3,) + sh, 4, 1e-3)
    src = core.guo_source(u, F, p)
    c = torch.tensor(C19, dtype=DT)
    k = 1 - 0.5 / p["tau"]
    assert torch.allclose(src.sum(0), torch.zeros(sh, dtype=DT), atol=1e-18, rtol=0)
    assert torch.allclose(torch.einsum("ia,i...->a...", c, src), k * F, atol=1e-18, rtol=0)
    second = torch.einsum("ia,ib,i...->ab...", c, c, src)
    uf = torch.einsum("a...,b...->ab...", u, F)
    assert torch.allclose(second, k * (uf + uf.transpose(0, 1)), atol=1e-18, rtol=0)


def test_stream_is_permutation_and_conserves():
    g = _rand((19, 5, 4, 6), 5, 1e-2)
    s = core.stream(g)
    for i in range(19):
        assert torch.equal(torch.sort(s[i].flatten()).values, torch.sort(g[i].flatten()).values)
        cx, cy, cz = C19[i]
        back = torch.roll(s[i], shifts=(-cz, -cy, -cx), dims=(-3, -2, -1))
        assert torch.equal(back, g[i])
    # a single population at one site moves to x + c_i
    one = torch.zeros(19, 5, 5, 5, dtype=DT)
    one[:, 2, 2, 2] = 1.0
    s = core.stream(one)
    for i, (cx, cy, cz) in enumerate(C19):
        assert s[i, 2 + cz, 2 + cy, 2 + cx] == 1.0 and s[i].sum() == 1.0


def test_collision_conserves_mass_and_momentum_without_force():
    p = dict(inputs.BASE_PARAMS)
    g = _rand((19, 4, 5, 3), 6, 5e-3)
    F = torch.zeros(3, 4, 5, 3, dtype=DT)
    rho, u = core.moments(g, F, p)
    gs = core.collide(g, u, rho, F, p)
    c = torch.tensor(C19, dtype=DT)
    assert torch.allclose(gs.sum(0), g.sum(0), atol=1e-16, rtol=0)
    assert torch.allclose(torch.einsum("ia,i...->a...", c, gs), torch.einsum("ia,i...->a...", c, g),
                          atol=1e-16, rtol=0)


def test_uniform_body_force_closed_form():
    """Sum of rho u grows by exactly N*f per step (u includes F/2)."""
    bf = (1e-5, -2e-5, 3e-5)
    p = dict(inputs.BASE_PARAMS, body_force=bf, zeta=0.0, W=0.0, K=0.0, A0=0.0, a=0.0, k_phi=0.0)
    n = (4, 5, 6)
    g = torch.zeros((19,) + n[::-1], dtype=DT)
    phi = torch.zeros(n[::-1], dtype=DT)
    q5 = torch.zeros((5,) + n[::-1], dtype=DT)
    N = 4 * 5 * 6
    for t in range(5):
        rho, u = core.observe(g, q5, phi, p)
        mom = (rho * u).sum((1, 2, 3))
        expect = torch.tensor(bf, dtype=DT) * N * (t + 0.5)
        assert torch.allclose(mom, expect, rtol=1e-12, atol=0)
        g, q5, phi = core.step(g, q5, phi, p)


def _linear_operator(k, tau):
    c = np.array(C19, dtype=float)
    w = np.array(W19)
    E = w[:, None] * (1.0 + 3.0 * c @ c.T)
    return np.diag(np.exp(-1j * (c @ k))) @ ((1 - 1 / tau) * np.eye(19) + E / tau)


def _shear_decay(nz, tau, steps, U0=1e-6):
    p = dict(inputs.BASE_PARAMS, tau=tau)
    u0 = torch.tensor(inputs.ic_shear_wave(nz, U0), dtype=DT)
    g = core.init_populations(u0, p)
    zero_q = torch.zeros((5,) + tuple(u0.shape[1:]), dtype=DT)
    zero_phi = torch.zeros(u0.shape[1:], dtype=DT)
    pa = dict(p, A0=0.0, a=0.0, k_phi=0.0, K=0.0, W=0.0, zeta=0.0)
    sinz = torch.sin(2 * math.pi * torch.arange(nz, dtype=DT) / nz)
    amps = []
    for _ in range(steps + 1):
        _, u = core.observe(g, zero_q, zero_phi, pa)
        amps.append(float((u[0].mean((1, 2)) * sinz).sum()))
        g, _, _ = core.step(g, zero_q, zero_phi, pa)
    return np.array(amps)


@pytest.mark.parametrize("nz,tau", [(16, 2.5), (12, 0.8)])
def test_shear_wave_exact_eigenvalue(nz, tau):
    """Decay per step equals the shear eigenvalue of the linearised step operator."""
    amps = _shear_decay(nz, tau, 80)
    ratio = amps[-1] / amps[-2]
    k = np.array([0.0, 0.0, 2 * math.pi / nz])
    ev, vec = np.linalg.eig(_linear_operator(k, tau))
    c = np.array(C19, dtype=float)
    jx = np.abs(c[:, 0] @ vec)
    lam = ev[np.argmax(jx / np.linalg.norm(vec, axis=0))]
    assert abs(lam.imag) < 1e-12
    assert abs(ratio - lam.real) / (1 - lam.real) < 1e-6


def test_shear_wave_analytic_viscosity():
    """At nz = 64 the decay rate matches nu k^2 with nu = (tau - 1/2)/3 within 1.5 %."""
    tau, nz = 2.5, 64
    amps = _shear_decay(nz, tau, 60)
    rate = -math.log(amps[-1] / amps[-21]) / 20
    nu = (tau - 0.5) / 3
    kk = 2 * math.pi / nz
    assert abs(rate / (nu * kk * kk) - 1) < 0.015
