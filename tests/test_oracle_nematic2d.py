"""Pins of the oracle's 2D bulk active nematic (D2Q9, 2x2 Q tensor), each
against something other than the oracle itself:

* D2Q9 tables: normalisation, isotropy to fourth order, opposite pairs;
  equilibrium and Guo moments; exact mass and momentum conservation; the
  uniform-body-force closed form; the shear-wave decay rate nu = (tau - 1/2)/3;
* the bulk order S_eq = sqrt(2 (chi/3 - 1)/chi) is stationary (H = 0) and
  vanishes for chi <= 3;
* H is the exact gradient of F_h (autograd): dF/dq_xx = -2 H_xx, dF/dq_xy = -2 H_xy;
* Gibbs-Duhem: the divergence of the passive (f delta + Ericksen) stress tends
  to -grad(Q):H at second order;
* the reactive identity sigma_react : W + H : S = xi (Q:H) div u at every site
  (a sign or transpose error in either fails it); rigid rotation gives
  S = Om Q - Q Om;
* the active force of a sinusoidal Q in closed form;
* defect charges of a synthetic +1/2 defect and of a +-1/2 pair.
"""
import math

import numpy as np
import pytest
import torch

from oracle import nematic2d as n2

DT = torch.float64

BASE = dict(tau=2.5, rho0=1.0, A0=0.1, chi=4.0, K=0.04, Gamma=0.3, xi=0.7, zeta=0.0)


def _p(**kw):
    return dict(BASE, **kw)


def _grid(ny, nx):
    y = torch.arange(ny, dtype=DT).reshape(ny, 1).expand(ny, nx)
    x = torch.arange(nx, dtype=DT).reshape(1, nx).expand(ny, nx)
    return x, y


def _rand_q2(ny, nx, seed, amp=0.3):
    return torch.tensor(np.random.default_rng(seed).uniform(-amp, amp, (2, ny, nx)))


def test_d2q9_tables():
    c = np.array(n2.C9, dtype=float)
    w = np.array(n2.W9)
    I = np.eye(2)
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), I / 3, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib,ig->abg", w, c, c, c), 0, atol=1e-15)
    iso4 = (np.einsum("ab,gd->abgd", I, I) + np.einsum("ag,bd->abgd", I, I) + np.einsum("ad,bg->abgd", I, I)) / 9
    assert np.allclose(np.einsum("i,ia,ib,ig,id->abgd", w, c, c, c, c), iso4, atol=1e-15)
    for i in range(1, 9, 2):
        assert np.array_equal(c[i], -c[i + 1])


def test_equilibrium_and_guo_moments():
    p = _p()
    rng = np.random.default_rng(1)
    rho = torch.tensor(1 + 0.05 * rng.standard_normal((3, 4)))
    u = torch.tensor(0.05 * rng.standard_normal((2, 3, 4)))
    F = torch.tensor(1e-3 * rng.standard_normal((2, 3, 4)))
    c, w = n2._c(), n2._w()
    f = n2.equilibrium_dev(rho, u, p) + w.reshape(9, 1, 1) * p["rho0"]
    assert torch.allclose(f.sum(0), rho, atol=1e-14)
    assert torch.allclose(torch.einsum("ia,i...->a...", c, f), rho * u, atol=1e-14)
    m2 = torch.einsum("ia,ib,i...->ab...", c, c, f)
    want = rho / 3 * n2._eye(rho) + rho * torch.einsum("a...,b...->ab...", u, u)
    assert torch.allclose(m2, want, atol=1e-14)
    src = n2.guo_source(u, F, p)
    k = 1 - 0.5 / p["tau"]
    assert torch.allclose(src.sum(0), torch.zeros_like(rho), atol=1e-17)
    assert torch.allclose(torch.einsum("ia,i...->a...", c, src), k * F, atol=1e-16)
    m2 = torch.einsum("ia,ib,i...->ab...", c, c, src)
    want = k * (torch.einsum("a...,b...->ab...", u, F) + torch.einsum("a...,b...->ab...", F, u))
    assert torch.allclose(m2, want, atol=1e-16)


def test_conservation_and_body_force():
    p = _p(zeta=0.01)
    rng = np.random.default_rng(2)
    g = torch.tensor(2e-3 * rng.standard_normal((9, 7, 6)))
    q2 = _rand_q2(7, 6, 3)
    j0 = torch.einsum("ia,i...->a", n2._c(), g)
    g1, q1 = n2.run(g, q2, p, 3)
    assert abs(float(g1.sum() - g.sum())) < 1e-14
    assert torch.allclose(torch.einsum("ia,i...->a", n2._c(), g1), j0, atol=1e-14)
    p = _p(A0=0.0, K=0.0, body_force=(2e-6, -1e-6))
    g = torch.zeros((9, 5, 8), dtype=DT)
    q2 = torch.zeros((2, 5, 8), dtype=DT)
    t = 7
    g, q2 = n2.run(g, q2, p, t)
    rho, u = n2.observe(g, q2, p)
    want = torch.tensor(p["body_force"], dtype=DT) * 40 * (t + 0.5)
    assert torch.allclose((rho * u).sum((1, 2)), want, rtol=1e-12, atol=0)


def test_shear_wave_viscosity():
    p = _p(A0=0.0, K=0.0)
    n, U0 = 64, 1e-6
    _, y = _grid(n, 2)
    siny = torch.sin(2 * math.pi * y / n)
    u0 = torch.zeros((2, n, 2), dtype=DT)
    u0[0] = U0 * siny
    g = n2.equilibrium_dev(torch.full((n, 2), p["rho0"], dtype=DT), u0, p)
    q2 = torch.zeros((2, n, 2), dtype=DT)
    amps = []
    for _ in range(61):
        _, u = n2.observe(g, q2, p)
        amps.append(float((u[0] * siny).sum()))
        g, q2 = n2.step(g, q2, p)
    rate = -math.log(amps[-1] / amps[-21]) / 20
    nu = (p["tau"] - 0.5) / 3
    assert abs(rate / (nu * (2 * math.pi / n) ** 2) - 1) < 0.015


@pytest.mark.parametrize("chi", [4.0, 3.5, 2.5])
def test_bulk_order_is_stationary(chi):
    p = _p(chi=chi)
    S = n2.s_eq(p)
    if chi <= 3:
        assert S == 0.0
    ang = 0.4
    n = torch.tensor([math.cos(ang), math.sin(ang)], dtype=DT)
    Q = (S * (torch.outer(n, n) - torch.eye(2, dtype=DT) / 2)).reshape(2, 2, 1, 1).expand(2, 2, 3, 4)
    H = n2.molecular_field(Q.clone(), p)
    assert float(H.abs().max()) < 1e-15
    if S > 0:  # a slightly different order is not stationary, and F is higher there
        Q2 = Q * 1.05
        assert float(n2.molecular_field(Q2.clone(), p).abs().max()) > 1e-5
        assert float(n2.free_energy(Q2.clone(), p)) > float(n2.free_energy(Q.clone(), p))


def test_h_is_exact_gradient_of_free_energy():
    p = _p()
    q2 = _rand_q2(6, 7, 4).requires_grad_(True)
    (gq,) = torch.autograd.grad(n2.free_energy(n2.q_full(q2), p), (q2,))
    with torch.no_grad():
        H = n2.molecular_field(n2.q_full(q2), p)
    want = torch.stack([-2 * H[0, 0], -2 * H[0, 1]])
    assert torch.allclose(want, gq, rtol=0, atol=1e-13)
    assert torch.allclose(H[0, 0] + H[1, 1], torch.zeros_like(H[0, 0]), atol=1e-16)


def test_gibbs_duhem_second_order():
    """div(f delta + Ericksen) + grad(Q):H -> 0 at second order on a smooth field."""
    errs = []
    for n in (32, 64, 128):
        x, y = _grid(n, n)
        k = 2 * math.pi / n
        q2 = torch.stack([0.2 * torch.sin(k * x) * torch.cos(k * y) + 0.1, 0.15 * torch.cos(k * x + 2 * k * y)])
        p = _p(xi=0.0, zeta=0.0)
        Q = n2.q_full(q2)
        H = n2.molecular_field(Q, p)
        sig = n2.stress(Q, p, H=H)  # xi = 0: passive + antisymmetric (Q H - H Q) part
        sig = sig - (torch.einsum("ac...,cb...->ab...", Q, H) - torch.einsum("ac...,cb...->ab...", H, Q))
        F = n2.force(sig, p)
        dQ = n2.grad_q(Q)
        target = -torch.einsum("agn...,gn...->a...", dQ, H)
        errs.append(float((F - target).abs().max()) / float(target.abs().max()))
    for a, b in zip(errs, errs[1:]):
        assert 3.4 < a / b < 4.5, errs


def test_reactive_identity_and_rigid_rotation():
    p = _p(A0=0.0, K=0.0, zeta=0.0, xi=0.7)
    ny, nx = 5, 6
    rng = np.random.default_rng(5)
    Q = n2.q_full(_rand_q2(ny, nx, 6))
    H = n2.q_full(torch.tensor(rng.uniform(-1, 1, (2, ny, nx))))
    u = torch.tensor(rng.uniform(-0.1, 0.1, (2, ny, nx)))
    Wt = n2.velocity_gradient(u)
    sig = n2.stress(Q, p, H=H)  # A0 = K = 0: f = 0, Ericksen = 0, only the reactive stress
    S = n2.corotation(u, Q, p)
    lhs = torch.einsum("ab...,ab...->...", sig, Wt) + torch.einsum("ab...,ab...->...", H, S)
    rhs = p["xi"] * torch.einsum("ab...,ab...->...", Q, H) * (Wt[0, 0] + Wt[1, 1])
    assert torch.allclose(lhs, rhs, atol=1e-14)
    om = 0.03
    Wrot = torch.zeros((2, 2, ny, nx), dtype=DT)
    Wrot[0, 1], Wrot[1, 0] = om, -om
    S = n2.corotation_from_w(Wrot, Q, p)
    Om = 0.5 * (Wrot - Wrot.transpose(0, 1))
    want = torch.einsum("ac...,cb...->ab...", Om, Q) - torch.einsum("ac...,cb...->ab...", Q, Om)
    assert torch.allclose(S, want, atol=1e-15)


def test_active_force_closed_form():
    """Q_xy = e sin(k y), nothing else: F_x = -zeta D0_y Q_xy = -zeta e sin(k) cos(k y), F_y = 0."""
    p = _p(A0=0.0, K=0.0, zeta=0.02)
    n, e = 12, 0.1
    k = 2 * math.pi * 2 / n
    _, y = _grid(n, n)
    q2 = torch.stack([torch.zeros((n, n), dtype=DT), e * torch.sin(k * y)])
    F = n2.force(n2.stress(n2.q_full(q2), p), p)
    assert torch.allclose(F[0], -p["zeta"] * e * math.sin(k) * torch.cos(k * y), atol=1e-16)
    assert float(F[1].abs().max()) < 1e-16


def test_defect_charges():
    n = 16
    x, y = _grid(n, n)
    # +1/2 defect centred inside a plaquette
    phi = torch.atan2(y - 7.5, x - 7.5)
    th = 0.5 * phi
    q2 = torch.stack([torch.cos(2 * th), torch.sin(2 * th)]) * 0.3
    q = n2.defect_charges(q2)
    assert abs(float(q[7, 7]) - 0.5) < 1e-12
    # the periodic box holds net zero charge: the rest sits on the box edges
    assert abs(float(q.sum())) < 1e-12
    # a +1/2, -1/2 pair
    th = 0.5 * torch.atan2(y - 7.5, x - 4.5) - 0.5 * torch.atan2(y - 7.5, x - 10.5)
    q = n2.defect_charges(torch.stack([torch.cos(2 * th), torch.sin(2 * th)]))
    assert abs(float(q[7, 4]) - 0.5) < 1e-12 and abs(float(q[7, 10]) + 0.5) < 1e-12
