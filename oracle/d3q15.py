"""The paper's own lattice-Boltzmann scheme (Sec. 3), as a second scheme of the
coupled step.  TEST INFRASTRUCTURE ONLY: used by tests and the benchmark's CPU
baseline, never by the product path.

* D3Q15 velocity set (Fig. 1): rest, the 6 axis vectors and the 8 body
  diagonals, weights 2/9, 1/9, 1/72.
* The symmetric part of the stress enters the second moment of the
  equilibrium (Eq. (9)): sum_i f_eq_i c_ia c_ib = rho/3 delta_ab + rho u_a u_b
  - S_ab, with S the symmetric part of the total stress of Eqs. (3)-(4) and
  rho/3 the lattice pressure.  With a fourth-order isotropic velocity set the
  second-order expansion of Eq. (11) that meets Eqs. (8)-(9) is
      f_eq_i = w_i [rho + 3 rho c_i.u + 9/2 (c_i c_i - I/3) : (rho u u - S)].
* The antisymmetric part A of the stress acts through the forcing term
  (Eq. (10)): F = div A (+ body force), applied with the same half-force
  velocity and source as the D3Q19 scheme.
* Populations are stored as deviations g_i = f_i - w_i rho0, as in core.py.
* The order-parameter updates (Eqs. (1)-(2)) are those of core.py, driven by
  the velocity u = (sum c g + F/2)/rho of this scheme.
"""
from __future__ import annotations

import torch

from . import core

DT = torch.float64

# Order: 0 rest; 1-6 = +x, -x, +y, -y, +z, -z; 7-14 = body diagonals in
# opposite pairs (+,+,+)/(-,-,-), (+,+,-)/(-,-,+), (+,-,+)/(-,+,-), (-,+,+)/(+,-,-).
C15 = (
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1),
    (1, -1, 1), (-1, 1, -1), (-1, 1, 1), (1, -1, -1),
)
W15 = (2.0 / 9.0,) + (1.0 / 9.0,) * 6 + (1.0 / 72.0,) * 8
OPP15 = tuple(0 if i == 0 else (i + 1 if i % 2 == 1 else i - 1) for i in range(15))


def _c():
    return torch.tensor(C15, dtype=DT)


def _w():
    return torch.tensor(W15, dtype=DT)


def split_stress(sig):
    """Symmetric and antisymmetric parts of sigma[a, b, ...]."""
    st = sig.transpose(0, 1)
    return 0.5 * (sig + st), 0.5 * (sig - st)


def force_antisymmetric(A, p):
    """F_a = sum_b D0_b A_ab + body force (Eq. (10))."""
    return core.force(A, p)


def moments(g, F, p):
    """rho = rho0 + sum g; u = (sum c g + F/2)/rho."""
    rho = p["rho0"] + g.sum(0)
    j = torch.einsum("ia,i...->a...", _c(), g)
    return rho, (j + 0.5 * F) / rho


def equilibrium_dev(rho, u, S, p):
    """g_eq_i = f_eq_i - w_i rho0 with the stress in the second moment (Eqs. (9), (11))."""
    c, w = _c(), _w()
    T = rho * torch.einsum("a...,b...->ab...", u, u) - S
    cTc = torch.einsum("ia,ib,ab...->i...", c, c, T)
    trT = T[0, 0] + T[1, 1] + T[2, 2]
    cu = torch.einsum("ia,a...->i...", c, u)
    shape = (15,) + (1,) * (u.dim() - 1)
    return w.reshape(shape) * ((rho - p["rho0"]) + 3.0 * rho * cu + 4.5 * cTc - 1.5 * trT)


def guo_source(u, F, p):
    """(1 - 1/(2tau)) w_i [3(c_i - u) + 9 (c_i.u) c_i] . F on D3Q15."""
    c, w = _c(), _w()
    cu = torch.einsum("ia,a...->i...", c, u)
    cF = torch.einsum("ia,a...->i...", c, F)
    uF = (u * F).sum(0)
    shape = (15,) + (1,) * (u.dim() - 1)
    return (1.0 - 0.5 / p["tau"]) * w.reshape(shape) * (3.0 * (cF - uF) + 9.0 * cu * cF)


def collide(g, u, rho, S, F, p):
    geq = equilibrium_dev(rho, u, S, p)
    return g - (g - geq) / p["tau"] + guo_source(u, F, p)


def stream(gs):
    """Pull streaming g_i(x, t+1) = g*_i(x - c_i) (Eq. (6))."""
    out = torch.empty_like(gs)
    for i, (cx, cy, cz) in enumerate(C15):
        out[i] = torch.roll(gs[i], shifts=(cz, cy, cx), dims=(-3, -2, -1))
    return out


def thermo(phi, Q, p):
    """mu, H, the symmetric stress S and the force of the antisymmetric stress."""
    mu = core.chemical_potential(phi, Q, p)
    H = core.molecular_field(phi, Q, p)
    S, A = split_stress(core.stress(phi, Q, p, H=H))
    return mu, H, S, force_antisymmetric(A, p)


def step(g, q5, phi, p):
    """One coupled step with the paper's LB scheme: returns (g(t+1), q5(t+1), phi(t+1))."""
    Q = core.q_full(q5)
    mu, H, S, F = thermo(phi, Q, p)
    rho, u = moments(g, F, p)
    g_new = stream(collide(g, u, rho, S, F, p))
    return g_new, core.q5_of(core.update_q(Q, u, H, p)), core.update_phi(phi, u, mu, p)


def run(g, q5, phi, p, nsteps):
    for _ in range(nsteps):
        g, q5, phi = step(g, q5, phi, p)
    return g, q5, phi


def observe(g, q5, phi, p):
    """rho and u at time t (u with F/2 of the antisymmetric force)."""
    _, _, _, F = thermo(phi, core.q_full(q5), p)
    return moments(g, F, p)


def init_populations(u0, p):
    """Deviations of the stress-free second-order equilibrium of (rho0, u0)."""
    rho = torch.full(u0.shape[1:], p["rho0"], dtype=DT)
    S = torch.zeros((3, 3) + u0.shape[1:], dtype=DT)
    return equilibrium_dev(rho, u0, S, p)
