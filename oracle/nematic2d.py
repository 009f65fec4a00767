"""Two-dimensional bulk active nematic on D2Q9: the 2D counterpart of the
coupled step, for the activity regimes of Fig. 4 and the 2D workload of
Fig. 3.  TEST INFRASTRUCTURE ONLY: used by tests and the benchmark's CPU
baseline, never by the product path.

The paper gives the regimes (quiescent, spontaneous flow, chaotic) but neither
the 2D equations nor parameters; this module states them (readings):
* D2Q9 (rest, +-x, +-y, then the diagonal pairs (+,+)/(-,-), (+,-)/(-,+)),
  weights 4/9, 1/9, 1/36; BGK with Guo forcing and pull streaming as in 3D,
  populations stored as deviations g_i = f_i - w_i rho0;
* Q a 2x2 traceless symmetric tensor, stored as (Q_xx, Q_xy);
* free energy: Landau-de Gennes bulk A0/2 (1 - chi/3) tr Q^2 + A0 chi/4 (tr Q^2)^2
  (the cubic invariant vanishes in 2D) and one elastic constant, K/2 |grad Q|^2;
  no concentration field (the bulk of Fig. 4);
* H = -dF/dQ = -A0 (1 - chi/3) Q - A0 chi tr(Q^2) Q + K lap Q;
* stress: f delta_ab - sum_gn D0_a Q_gn K D0_b Q_gn - xi (H P + P H)
  + 2 xi P (Q:H) + (Q H - H Q) - zeta Q with P = Q + I/2 (zeta > 0 extensile);
* Beris-Edwards: Q(t+1) = Q + [-u.D0 Q + S + Gamma H] with
  S = (xi D + Om) P + P (xi D - Om) - 2 xi P tr(Q W) made traceless, W_ab = D0_b u_a;
* explicit Euler, second-order central differences, 5-point Laplacian;
  arrays are [ny, nx] (x fastest).
"""
from __future__ import annotations

import math

import torch

DT = torch.float64
_DIM = {0: -1, 1: -2}

C9 = ((0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1))
W9 = (4.0 / 9.0,) + (1.0 / 9.0,) * 4 + (1.0 / 36.0,) * 4
EYE2 = torch.eye(2, dtype=DT)


def shift(a, axis, s):
    """Value at x + s e_axis (periodic)."""
    return torch.roll(a, shifts=-s, dims=_DIM[axis])


def d0(a, axis):
    return 0.5 * (shift(a, axis, 1) - shift(a, axis, -1))


def dplus(a, axis):
    return shift(a, axis, 1) - a


def lap(a):
    return sum(shift(a, g, 1) + shift(a, g, -1) for g in range(2)) - 4.0 * a


def q_full(q2):
    xx, xy = q2
    return torch.stack([torch.stack([xx, xy]), torch.stack([xy, -xx])])


def q2_of(Q):
    return torch.stack([Q[0, 0], Q[0, 1]])


def _eye(like):
    return EYE2.reshape(2, 2, 1, 1).to(like)


def _tr2(Q):
    return torch.einsum("ab...,ab...->...", Q, Q)


# ------------------------------------------------------------ thermodynamics
def bulk_density(Q, p):
    t2 = _tr2(Q)
    return 0.5 * p["A0"] * (1.0 - p["chi"] / 3.0) * t2 + 0.25 * p["A0"] * p["chi"] * t2 * t2


def molecular_field(Q, p):
    t2 = _tr2(Q)
    Hb = -p["A0"] * (1.0 - p["chi"] / 3.0) * Q - p["A0"] * p["chi"] * t2 * Q
    return Hb + p["K"] * torch.stack([torch.stack([lap(Q[a, b]) for b in range(2)]) for a in range(2)])


def free_energy(Q, p):
    """F_h with forward differences in the gradient term (H is its exact gradient)."""
    f = bulk_density(Q, p) + 0.5 * p["K"] * sum((dplus(Q, g) ** 2).sum((0, 1)) for g in range(2))
    return f.sum()


def grad_q(Q):
    """dQ[g, a, b] = D0_g Q_ab."""
    return torch.stack([d0(Q, g) for g in range(2)])


def stress(Q, p, H=None):
    if H is None:
        H = molecular_field(Q, p)
    I = _eye(Q[0, 0])
    dQ = grad_q(Q)
    fc = bulk_density(Q, p) + 0.5 * p["K"] * (dQ * dQ).sum((0, 1, 2))
    er = -p["K"] * torch.einsum("agn...,bgn...->ab...", dQ, dQ)
    P = Q + I / 2.0
    HP = torch.einsum("ac...,cb...->ab...", H, P)
    PH = torch.einsum("ac...,cb...->ab...", P, H)
    QH = torch.einsum("ac...,cb...->ab...", Q, H)
    HQ = torch.einsum("ac...,cb...->ab...", H, Q)
    qh = torch.einsum("ab...,ab...->...", Q, H)
    react = -p["xi"] * (HP + PH) + 2.0 * p["xi"] * P * qh + (QH - HQ)
    return I * fc + er + react - p["zeta"] * Q


def force(sig, p):
    bf = p.get("body_force", (0.0, 0.0))
    return torch.stack([sum(d0(sig[a, b], b) for b in range(2)) + float(bf[a]) for a in range(2)])


# ------------------------------------------------------------------------ LB
def _c():
    return torch.tensor(C9, dtype=DT)


def _w():
    return torch.tensor(W9, dtype=DT)


def moments(g, F, p):
    rho = p["rho0"] + g.sum(0)
    j = torch.einsum("ia,i...->a...", _c(), g)
    return rho, (j + 0.5 * F) / rho


def equilibrium_dev(rho, u, p, drho=None):
    """g_eq = f_eq - w rho0; drho = rho - rho0 (taken as sum g when given, which keeps
    the precision that storing deviations is for)."""
    c, w = _c(), _w()
    cu = torch.einsum("ia,a...->i...", c, u)
    uu = (u * u).sum(0)
    shape = (9,) + (1,) * (u.dim() - 1)
    if drho is None:
        drho = rho - p["rho0"]
    return w.reshape(shape) * (drho + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu))


def guo_source(u, F, p):
    c, w = _c(), _w()
    cu = torch.einsum("ia,a...->i...", c, u)
    cF = torch.einsum("ia,a...->i...", c, F)
    uF = (u * F).sum(0)
    shape = (9,) + (1,) * (u.dim() - 1)
    return (1.0 - 0.5 / p["tau"]) * w.reshape(shape) * (3.0 * (cF - uF) + 9.0 * cu * cF)


def collide(g, u, rho, F, p):
    return g - (g - equilibrium_dev(rho, u, p, drho=g.sum(0))) / p["tau"] + guo_source(u, F, p)


def stream(gs):
    out = torch.empty_like(gs)
    for i, (cx, cy) in enumerate(C9):
        out[i] = torch.roll(gs[i], shifts=(cy, cx), dims=(-2, -1))
    return out


# ---------------------------------------------------------------- Q dynamics
def velocity_gradient(u):
    """W_ab = D0_b u_a."""
    return torch.stack([torch.stack([d0(u[a], b) for b in range(2)]) for a in range(2)])


def corotation(u, Q, p):
    return corotation_from_w(velocity_gradient(u), Q, p)


def corotation_from_w(Wt, Q, p):
    xi = p["xi"]
    I = _eye(Q[0, 0])
    D = 0.5 * (Wt + Wt.transpose(0, 1))
    Om = 0.5 * (Wt - Wt.transpose(0, 1))
    P = Q + I / 2.0
    trQW = torch.einsum("ab...,ba...->...", Q, Wt)
    S = (torch.einsum("ac...,cb...->ab...", xi * D + Om, P) + torch.einsum("ac...,cb...->ab...", P, xi * D - Om)
         - 2.0 * xi * P * trQW)
    return S - I * (S[0, 0] + S[1, 1]) / 2.0


def update_q(Q, u, H, p):
    adv = sum(u[g] * d0(Q, g) for g in range(2))
    return Q + (-adv + corotation(u, Q, p) + p["Gamma"] * H)


# ------------------------------------------------------------------ the step
def step(g, q2, p):
    """One coupled step: returns (g(t+1), q2(t+1)); g holds post-stream deviations at t."""
    Q = q_full(q2)
    H = molecular_field(Q, p)
    F = force(stress(Q, p, H=H), p)
    rho, u = moments(g, F, p)
    g_new = stream(collide(g, u, rho, F, p))
    return g_new, q2_of(update_q(Q, u, H, p))


def run(g, q2, p, nsteps):
    for _ in range(nsteps):
        g, q2 = step(g, q2, p)
    return g, q2


def observe(g, q2, p):
    """rho and u (with F/2) at time t."""
    Q = q_full(q2)
    return moments(g, force(stress(Q, p), p), p)


def totals(g, q2, p):
    rho, u = observe(g, q2, p)
    return dict(mass=g[0].numel() * p["rho0"] + float(g.sum()),
                momentum=[float((rho * u[a]).sum()) for a in range(2)],
                free_energy=float(free_energy(q_full(q2), p)),
                kinetic_energy=float((0.5 * rho * (u * u).sum(0)).sum()))


def s_eq(p):
    """Bulk order S of Q = S (n n - I/2) at the minimum of the bulk density (0 if isotropic)."""
    a = p["chi"] / 3.0 - 1.0
    return math.sqrt(2.0 * a / p["chi"]) if a > 0 else 0.0


def defect_charges(q2):
    """Winding of the director angle theta = atan2(Q_xy, Q_xx)/2 around each unit plaquette,
    in units of 2 pi (+-1/2 at half-integer defects, 0 elsewhere); [ny, nx]."""
    th = 0.5 * torch.atan2(q2[1], q2[0])

    def dth(a, b):  # angle difference wrapped into (-pi/2, pi/2]
        d = b - a
        return d - math.pi * torch.round(d / math.pi)

    t00 = th
    t10 = shift(th, 0, 1)
    t11 = shift(t10, 1, 1)
    t01 = shift(th, 1, 1)
    w = dth(t00, t10) + dth(t10, t11) + dth(t11, t01) + dth(t01, t00)
    return w / (2.0 * math.pi)
