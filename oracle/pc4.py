"""The paper's finite-difference integrator for the order parameters (Sec. 3):
predictor-corrector time stepping, first-order upwind advection and
fourth-order accurate stencils for the space derivatives of Eqs. (1)-(2).
TEST INFRASTRUCTURE ONLY: used by tests and the benchmark's CPU baseline,
never by the product path.

Readings (the paper names the three ingredients and nothing more):
* predictor-corrector = Heun's method: with R the right-hand side of
  Eqs. (1)-(2) at fixed velocity, X* = X + R(X) and X(t+1) = X + [R(X) + R(X*)]/2;
  u is the LB velocity at time t (with F/2) in both stages;
* fourth-order stencils for every space derivative inside the order-parameter
  dynamics: D4 f = [8(f(x+1) - f(x-1)) - (f(x+2) - f(x-2))]/12 and the 13-point
  Laplacian L4 f = sum_g [16(f(x+e) + f(x-e)) - (f(x+2e) + f(x-2e)) - 30 f]/12,
  used in mu, H, the velocity gradient W and the Laplacian of mu;
* first-order upwind advection: u.grad Q with the one-sided difference taken
  against the flow at each site, and for phi the donor-cell flux form
  div(u phi) with face velocity (u(x) + u(x+e))/2 and the upwind phi, which
  conserves sum phi exactly;
* the LB side (stress, force, collision, streaming) is that of core.py.
"""
from __future__ import annotations

import torch

from . import core
from .core import DT, EPS, shift

# ------------------------------------------------------------ 4th-order operators


def d4(a, axis):
    """Fourth-order central first derivative along axis (radius 2)."""
    return (8.0 * (shift(a, axis, 1) - shift(a, axis, -1)) - (shift(a, axis, 2) - shift(a, axis, -2))) / 12.0


def lap4(a):
    """Fourth-order 13-point Laplacian."""
    out = -7.5 * a
    for g in range(3):
        out = out + (16.0 * (shift(a, g, 1) + shift(a, g, -1)) - (shift(a, g, 2) + shift(a, g, -2))) / 12.0
    return out


def grad_phi4(phi):
    return torch.stack([d4(phi, g) for g in range(3)])


def grad_q4(Q):
    """dQ[g, a, b] = D4_g Q_ab."""
    return torch.stack([d4(Q, g) for g in range(3)])


def velocity_gradient4(u):
    """W_ab = D4_b u_a."""
    return torch.stack([torch.stack([d4(u[a], b) for b in range(3)]) for a in range(3)])


# ----------------------------------------------- thermodynamics with D4 and L4


def chemical_potential4(phi, Q, p):
    """mu of Eqs. (1), (5) with the gradient terms on the 4th-order stencils:
    double-well derivative + chi_s d(LdG bulk)/dchi - k_phi L4 phi - 2W D4_a(Q_ab D4_b phi)."""
    tr2, _, tr3 = core._invariants(Q)
    mu = p["a"] * phi * (phi - p["phi0"]) * (2.0 * phi - p["phi0"]) / p["phi_cr"] ** 2
    mu = mu + p["A0"] * p["chi_s"] * (-tr2 / 6.0 - tr3 / 3.0 + tr2 * tr2 / 4.0)
    mu = mu - p["k_phi"] * lap4(phi)
    v = torch.einsum("ab...,b...->a...", Q, grad_phi4(phi))
    return mu - 2.0 * p["W"] * sum(d4(v[a], a) for a in range(3))


def molecular_field4(phi, Q, p):
    """H of Eqs. (2), (5) with the gradient terms on the 4th-order stencils:
    bulk - ... + K L4 Q - 2Kq0 (C + C^T) - 4Kq0^2 Q - W (D4phi D4phi - I |D4phi|^2/3),
    C_ab = eps_agd D4_g Q_db."""
    chi = p["chi0"] + p["chi_s"] * phi
    tr2, Q2, _ = core._invariants(Q)
    I = core.eye_field(phi)
    dphi = grad_phi4(phi)
    Cq = torch.einsum("agd,gdb...->ab...", EPS, grad_q4(Q))
    H = -p["A0"] * ((1.0 - chi / 3.0) * Q - chi * (Q2 - I * tr2 / 3.0) + chi * Q * tr2)
    H = H + p["K"] * torch.stack([torch.stack([lap4(Q[a, b]) for b in range(3)]) for a in range(3)])
    H = H - 2.0 * p["K"] * p["q0"] * (Cq + Cq.transpose(0, 1))
    H = H - 4.0 * p["K"] * p["q0"] ** 2 * Q
    dd = torch.einsum("a...,b...->ab...", dphi, dphi)
    return H - p["W"] * (dd - I * (dphi * dphi).sum(0) / 3.0)


# --------------------------------------------------------------- upwind advection


def upwind_advection(u, X):
    """u_g dX/dx_g with first-order upwind differences: backward where u_g > 0,
    forward where u_g < 0."""
    out = torch.zeros_like(X)
    for g in range(3):
        back = X - shift(X, g, -1)
        fwd = shift(X, g, 1) - X
        out = out + torch.clamp(u[g], min=0.0) * back + torch.clamp(u[g], max=0.0) * fwd
    return out


def donor_cell_divergence(u, phi):
    """div(u phi) in flux form: flux through the face x + e_g/2 is
    uf phi(x) if uf > 0 else uf phi(x + e_g), uf = (u_g(x) + u_g(x + e_g))/2."""
    out = torch.zeros_like(phi)
    for g in range(3):
        uf = 0.5 * (u[g] + shift(u[g], g, 1))
        flux = torch.clamp(uf, min=0.0) * phi + torch.clamp(uf, max=0.0) * shift(phi, g, 1)
        out = out + flux - shift(flux, g, -1)
    return out


# ------------------------------------------------------------------ Heun stages


def rhs(Q, phi, u, p):
    """(dQ/dt, dphi/dt) of Eqs. (1)-(2) at fixed u."""
    H = molecular_field4(phi, Q, p)
    S = core.corotation_from_w(velocity_gradient4(u), Q, p)
    rq = -upwind_advection(u, Q) + S + p["Gamma"] * H
    rphi = -donor_cell_divergence(u, phi) + p["M"] * lap4(chemical_potential4(phi, Q, p))
    return rq, rphi


def update_pc(Q, phi, u, p):
    """Heun: predictor X* = X + R(X); corrector X(t+1) = X + (R(X) + R(X*))/2."""
    kq1, kp1 = rhs(Q, phi, u, p)
    kq2, kp2 = rhs(Q + kq1, phi + kp1, u, p)
    return Q + 0.5 * (kq1 + kq2), phi + 0.5 * (kp1 + kp2)


def step(g, q5, phi, p):
    """One coupled step: the LB part of core.py, then the predictor-corrector
    update of Q and phi driven by u at time t."""
    Q = core.q_full(q5)
    _, _, _, F = core.thermo(phi, Q, p)
    rho, u = core.moments(g, F, p)
    g_new = core.stream(core.collide(g, u, rho, F, p))
    Q_new, phi_new = update_pc(Q, phi, u, p)
    return g_new, core.q5_of(Q_new), phi_new


def run(g, q5, phi, p, nsteps):
    for _ in range(nsteps):
        g, q5, phi = step(g, q5, phi, p)
    return g, q5, phi
