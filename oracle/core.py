"""Plain FP64 CPU oracle of the coupled hybrid lattice-Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
calls it.  It shares no code with the HIP path.

What it computes (Carenza, Gonnella, Negro, "Lattice Boltzmann simulations of
self-propelling chiral active droplets"):

* free energy F[phi, Q] of Eq. (5): double well in phi, gradient term, the
  Landau-de Gennes bulk with chi(phi) = chi0 + chi_s*phi, one elastic constant
  with the cholesteric q0 term, and the anchoring W grad(phi).Q.grad(phi);
* chemical potential mu = dF/dphi and molecular field H = -(dF/dQ) projected
  traceless (Sec. 2, Eqs. (1)-(2));
* the stress of Eq. (3): the passive (interfacial + Ericksen + Beris-Edwards
  reactive + antisymmetric) part and the active part of Eq. (4), taken as
  -zeta*phi*Q so that activity lives inside the droplet;
* one D3Q19 BGK collide-and-stream (Eqs. (6)-(8), (11) with G = 0), forced
  by F = div(sigma) in the Guo form, which meets the force-moment conditions
  of Eq. (10) with the whole stress as a body force;
* explicit Euler finite-difference updates of Q (Beris-Edwards, Eq. (2),
  advection + co-rotation + Gamma*H) and phi (Cahn-Hilliard, Eq. (1), in
  conservative flux form).

Every right-hand side uses time-t fields.  Units: lattice spacing = time step
= 1, periodic box.  Fields are torch float64 tensors shaped [nz, ny, nx]
(x fastest).  The full Q tensor is a [3, 3, nz, ny, nx] tensor; the 5 stored
components are (xx, xy, xz, yy, yz).  Populations are stored as deviations
g_i = f_i - w_i*rho0 ([19, nz, ny, nx]).

Discrete operators: D0 central difference, D+ forward difference, 7-point
Laplacian, C_ab = eps_agd D0_g Q_db (discrete curl of Q), P = Q + I/3.
"""
from __future__ import annotations

import torch

from .lattice import C19, W19

DT = torch.float64
_DIM = {0: -1, 1: -2, 2: -3}  # x, y, z -> tensor dimension


# ---------------------------------------------------------------- operators
def shift(a: torch.Tensor, axis: int, s: int) -> torch.Tensor:
    """Value at x + s*e_axis (periodic)."""
    return torch.roll(a, shifts=-s, dims=_DIM[axis])


def d0(a, axis):
    """Central difference [a(x+e) - a(x-e)]/2."""
    return 0.5 * (shift(a, axis, 1) - shift(a, axis, -1))


def dplus(a, axis):
    """Forward difference a(x+e) - a(x)."""
    return shift(a, axis, 1) - a


def lap(a):
    """7-point Laplacian."""
    return sum(shift(a, g, 1) + shift(a, g, -1) for g in range(3)) - 6.0 * a


def levi_civita():
    e = torch.zeros(3, 3, 3, dtype=DT)
    e[0, 1, 2] = e[1, 2, 0] = e[2, 0, 1] = 1.0
    e[0, 2, 1] = e[2, 1, 0] = e[1, 0, 2] = -1.0
    return e


EPS = levi_civita()
EYE = torch.eye(3, dtype=DT)


def q_full(q5):
    """[5,...] stored components -> [3,3,...] traceless symmetric tensor."""
    xx, xy, xz, yy, yz = q5
    zz = -xx - yy
    return torch.stack([torch.stack([xx, xy, xz]), torch.stack([xy, yy, yz]), torch.stack([xz, yz, zz])])


def q5_of(Q):
    return torch.stack([Q[0, 0], Q[0, 1], Q[0, 2], Q[1, 1], Q[1, 2]])


def eye_field(like):
    """Identity tensor broadcast over the lattice: [3,3,1,1,1]."""
    return EYE.reshape(3, 3, 1, 1, 1).to(like)


def grad_phi(phi):
    """D0_g phi, [3, ...]."""
    return torch.stack([d0(phi, g) for g in range(3)])


def grad_q(Q):
    """dQ[g, a, b] = D0_g Q_ab, [3, 3, 3, ...]."""
    return torch.stack([d0(Q, g) for g in range(3)])


def curl_q(dQ):
    """C_ab = eps_agd D0_g Q_db."""
    return torch.einsum("agd,gdb...->ab...", EPS, dQ)


def _invariants(Q):
    tr2 = torch.einsum("ab...,ab...->...", Q, Q)
    Q2 = torch.einsum("ac...,cb...->ab...", Q, Q)
    tr3 = torch.einsum("ab...,ba...->...", Q2, Q)
    return tr2, Q2, tr3


# ------------------------------------------------------ thermodynamics (Eq. 5)
def chemical_potential(phi, Q, p):
    """mu = dF/dphi (Eqs. (1), (5)).

    double-well derivative + chi_s * d(LdG bulk)/dchi - k_phi lap(phi)
    - 2W D0_a(Q_ab D0_b phi)  (the anchoring term, since D0^T = -D0).
    """
    tr2, _, tr3 = _invariants(Q)
    dphi = grad_phi(phi)
    mu = p["a"] * phi * (phi - p["phi0"]) * (2.0 * phi - p["phi0"]) / p["phi_cr"] ** 2
    mu = mu + p["A0"] * p["chi_s"] * (-tr2 / 6.0 - tr3 / 3.0 + tr2 * tr2 / 4.0)
    mu = mu - p["k_phi"] * lap(phi)
    v = torch.einsum("ab...,b...->a...", Q, dphi)
    mu = mu - 2.0 * p["W"] * sum(d0(v[a], a) for a in range(3))
    return mu


def molecular_field(phi, Q, p):
    """H = -(dF/dQ) projected onto traceless symmetric tensors (Eqs. (2), (5)).

    bulk: -A0[(1 - chi/3)Q - chi(Q^2 - I tr(Q^2)/3) + chi Q tr(Q^2)]
    elastic: K lap(Q) - 2 K q0 (C + C^T) - 4 K q0^2 Q
    anchoring: -W (D0phi D0phi - I |D0phi|^2/3)
    """
    chi = p["chi0"] + p["chi_s"] * phi
    tr2, Q2, _ = _invariants(Q)
    I = eye_field(phi)
    dphi = grad_phi(phi)
    dQ = grad_q(Q)
    Cq = curl_q(dQ)
    H = -p["A0"] * ((1.0 - chi / 3.0) * Q - chi * (Q2 - I * tr2 / 3.0) + chi * Q * tr2)
    H = H + p["K"] * torch.stack([torch.stack([lap(Q[a, b]) for b in range(3)]) for a in range(3)])
    H = H - 2.0 * p["K"] * p["q0"] * (Cq + Cq.transpose(0, 1))
    H = H - 4.0 * p["K"] * p["q0"] ** 2 * Q
    dd = torch.einsum("a...,b...->ab...", dphi, dphi)
    H = H - p["W"] * (dd - I * (dphi * dphi).sum(0) / 3.0)
    return H


def bulk_density(phi, Q, p):
    """Local (non-gradient) part of the Eq. (5) integrand, incl. 2Kq0^2 tr(Q^2)."""
    chi = p["chi0"] + p["chi_s"] * phi
    tr2, _, tr3 = _invariants(Q)
    f = 0.5 * p["a"] * phi ** 2 * (phi - p["phi0"]) ** 2 / p["phi_cr"] ** 2
    f = f + p["A0"] * (0.5 * (1.0 - chi / 3.0) * tr2 - chi / 3.0 * tr3 + chi / 4.0 * tr2 * tr2)
    f = f + 2.0 * p["K"] * p["q0"] ** 2 * tr2
    return f


def free_energy_density_c(phi, Q, p):
    """Local free-energy density with central differences (used in the stress).

    The one-constant form of the elastic term of Eq. (5) on a periodic box:
    (K/2)|grad Q|^2 + 2 K q0 Q:curl Q + 2 K q0^2 Q:Q.
    """
    dphi = grad_phi(phi)
    dQ = grad_q(Q)
    Cq = curl_q(dQ)
    f = bulk_density(phi, Q, p)
    f = f + 0.5 * p["k_phi"] * (dphi * dphi).sum(0)
    f = f + 0.5 * p["K"] * (dQ * dQ).sum((0, 1, 2))
    f = f + 2.0 * p["K"] * p["q0"] * torch.einsum("ab...,ab...->...", Q, Cq)
    f = f + p["W"] * torch.einsum("a...,ab...,b...->...", dphi, Q, dphi)
    return f


def free_energy(phi, Q, p):
    """Discrete free energy F_h (Eq. (5) summed over the lattice).

    Gradient-squared terms use forward differences so that mu and H of this
    module are the exact gradients of F_h: dF_h/dphi(x) = mu(x) and
    dF_h/dq_k(x) = -H(x):B_k for the stored components q_k.
    """
    dphi = grad_phi(phi)
    dQ = grad_q(Q)
    Cq = curl_q(dQ)
    f = bulk_density(phi, Q, p)
    f = f + 0.5 * p["k_phi"] * sum(dplus(phi, g) ** 2 for g in range(3))
    f = f + 0.5 * p["K"] * sum((dplus(Q, g) ** 2).sum((0, 1)) for g in range(3))
    f = f + 2.0 * p["K"] * p["q0"] * torch.einsum("ab...,ab...->...", Q, Cq)
    f = f + p["W"] * torch.einsum("a...,ab...,b...->...", dphi, Q, dphi)
    return f.sum()


# ------------------------------------------------------------ stress (Eq. 3-4)
def stress_interfacial(phi, Q, fc, p):
    """f delta_ab - D0_a phi (k_phi D0_b phi + 2W Q_bg D0_g phi).

    Index a is the force component, b the derivative index (F_a = D0_b s_ab).
    Its divergence tends to mu grad(phi) (plus the Q part of the Ericksen
    stress: -grad(Q):H), the thermodynamic force of Eq. (3) written with the
    free-energy density as the isotropic part; the form with (f - phi mu)
    differs by the gradient of phi*mu, which the pressure of the
    incompressible flow absorbs.
    """
    dphi = grad_phi(phi)
    I = eye_field(phi)
    t = p["k_phi"] * dphi + 2.0 * p["W"] * torch.einsum("bg...,g...->b...", Q, dphi)
    return I * fc - torch.einsum("a...,b...->ab...", dphi, t)


def stress_ericksen_q(Q, p):
    """-sum_gn D0_a Q_gn (K D0_b Q_gn + 2 K q0 eps_lbg Q_ln)."""
    dQ = grad_q(Q)
    dfd = p["K"] * dQ + 2.0 * p["K"] * p["q0"] * torch.einsum("lbg,ln...->bgn...", EPS, Q)
    return -torch.einsum("agn...,bgn...->ab...", dQ, dfd)


def stress_reactive(Q, H, p):
    """Beris-Edwards reactive stress + antisymmetric part.

    -xi (H P + P H) + 2 xi P (Q:H) + (Q H - H Q), with P = Q + I/3.
    """
    I = eye_field(Q[0, 0])
    P = Q + I / 3.0
    HP = torch.einsum("ac...,cb...->ab...", H, P)
    PH = torch.einsum("ac...,cb...->ab...", P, H)
    QH = torch.einsum("ac...,cb...->ab...", Q, H)
    HQ = torch.einsum("ac...,cb...->ab...", H, Q)
    qh = torch.einsum("ab...,ab...->...", Q, H)
    return -p["xi"] * (HP + PH) + 2.0 * p["xi"] * P * qh + (QH - HQ)


def stress_active(phi, Q, p):
    """Active stress of Eq. (4) confined to the droplet: -zeta phi Q."""
    return -p["zeta"] * phi * Q


def stress(phi, Q, p, H=None):
    """Total stress: interfacial + Ericksen (Q) + reactive + active."""
    if H is None:
        H = molecular_field(phi, Q, p)
    fc = free_energy_density_c(phi, Q, p)
    return (stress_interfacial(phi, Q, fc, p) + stress_ericksen_q(Q, p)
            + stress_reactive(Q, H, p) + stress_active(phi, Q, p))


def force(sig, p):
    """F_a = sum_b D0_b sigma_ab + body force."""
    bf = p.get("body_force", (0.0, 0.0, 0.0))
    return torch.stack([sum(d0(sig[a, b], b) for b in range(3)) + float(bf[a]) for a in range(3)])


# ----------------------------------------------------------------- LB (6-11)
def _c():
    return torch.tensor(C19, dtype=DT)


def _w():
    return torch.tensor(W19, dtype=DT)


def moments(g, F, p):
    """rho = rho0 + sum g; u = (sum c g + F/2)/rho (Eq. (8), Guo half-force)."""
    c = _c()
    rho = p["rho0"] + g.sum(0)
    j = torch.einsum("ia,i...->a...", c, g)
    u = (j + 0.5 * F) / rho
    return rho, u


def equilibrium_dev(rho, u, p):
    """g_eq_i = f_eq_i - w_i rho0 with the second-order f_eq of Eq. (11), G = 0."""
    c, w = _c(), _w()
    cu = torch.einsum("ia,a...->i...", c, u)
    uu = (u * u).sum(0)
    shape = (19,) + (1,) * (u.dim() - 1)
    return w.reshape(shape) * ((rho - p["rho0"]) + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu))


def guo_source(u, F, p):
    """(1 - 1/(2tau)) w_i [3(c_i - u) + 9 (c_i.u) c_i] . F."""
    c, w = _c(), _w()
    cu = torch.einsum("ia,a...->i...", c, u)
    cF = torch.einsum("ia,a...->i...", c, F)
    uF = (u * F).sum(0)
    shape = (19,) + (1,) * (u.dim() - 1)
    return (1.0 - 0.5 / p["tau"]) * w.reshape(shape) * (3.0 * (cF - uF) + 9.0 * cu * cF)


def collide(g, u, rho, F, p):
    geq = equilibrium_dev(rho, u, p)
    return g - (g - geq) / p["tau"] + guo_source(u, F, p)


def stream(gs):
    """Pull streaming: g_i(x, t+1) = g*_i(x - c_i) (Eq. (6))."""
    out = torch.empty_like(gs)
    for i, (cx, cy, cz) in enumerate(C19):
        out[i] = torch.roll(gs[i], shifts=(cz, cy, cx), dims=(-3, -2, -1))
    return out


# ----------------------------------------------------- order parameters (1-2)
def velocity_gradient(u):
    """W_ab = D0_b u_a."""
    return torch.stack([torch.stack([d0(u[a], b) for b in range(3)]) for a in range(3)])


def corotation(u, Q, p):
    """Traceless co-rotational term of the Beris-Edwards material derivative.

    S = (xi D + Om)(Q + I/3) + (Q + I/3)(xi D - Om) - 2 xi (Q + I/3) tr(Q W),
    D, Om the symmetric / antisymmetric parts of W; returned as S - I tr(S)/3.
    """
    Wt = velocity_gradient(u)
    return corotation_from_w(Wt, Q, p)


def corotation_from_w(Wt, Q, p):
    xi = p["xi"]
    I = eye_field(Q[0, 0])
    D = 0.5 * (Wt + Wt.transpose(0, 1))
    Om = 0.5 * (Wt - Wt.transpose(0, 1))
    P = Q + I / 3.0
    trQW = torch.einsum("ab...,ba...->...", Q, Wt)
    A = xi * D + Om
    B = xi * D - Om
    S = torch.einsum("ac...,cb...->ab...", A, P) + torch.einsum("ac...,cb...->ab...", P, B) - 2.0 * xi * P * trQW
    trS = S[0, 0] + S[1, 1] + S[2, 2]
    return S - I * trS / 3.0


def advection_q(u, Q):
    """u_g D0_g Q."""
    return sum(u[g] * d0(Q, g) for g in range(3))


def update_q(Q, u, H, p):
    """Q(t+1) = Q + [-u.D0 Q + S + Gamma H] (Eq. (2), explicit Euler)."""
    return Q + (-advection_q(u, Q) + corotation(u, Q, p) + p["Gamma"] * H)


def update_phi(phi, u, mu, p):
    """phi(t+1) = phi - D0_g(u_g phi) + M lap(mu) (Eq. (1), explicit Euler)."""
    return phi - sum(d0(u[g] * phi, g) for g in range(3)) + p["M"] * lap(mu)


# ------------------------------------------------------------------ the step
def thermo(phi, Q, p):
    """mu, H, sigma, F at time t."""
    mu = chemical_potential(phi, Q, p)
    H = molecular_field(phi, Q, p)
    sig = stress(phi, Q, p, H=H)
    F = force(sig, p)
    return mu, H, sig, F


def step(g, q5, phi, p):
    """One coupled step: returns (g(t+1), q5(t+1), phi(t+1)).

    g holds post-stream deviations at time t.
    """
    Q = q_full(q5)
    mu, H, _, F = thermo(phi, Q, p)
    rho, u = moments(g, F, p)
    gs = collide(g, u, rho, F, p)
    g_new = stream(gs)
    Q_new = update_q(Q, u, H, p)
    phi_new = update_phi(phi, u, mu, p)
    return g_new, q5_of(Q_new), phi_new


def run(g, q5, phi, p, nsteps):
    for _ in range(nsteps):
        g, q5, phi = step(g, q5, phi, p)
    return g, q5, phi


def observe(g, q5, phi, p):
    """rho and u at time t (u includes F/2), as the moments call reports them."""
    Q = q_full(q5)
    _, _, _, F = thermo(phi, Q, p)
    return moments(g, F, p)


def init_populations(u0, p, rho=None):
    """Post-stream deviations of a state at rest density rho0 (or rho) and velocity u0."""
    if rho is None:
        rho = torch.full(u0.shape[1:], p["rho0"], dtype=DT)
    return equilibrium_dev(rho, u0, p)


# ---------------------------------------------------------------- observables
def totals(g, q5, phi, p):
    """mass, momentum (sum rho u with F/2), sum phi, F_h, kinetic energy."""
    rho, u = observe(g, q5, phi, p)
    n = phi.numel()
    return dict(
        mass=n * p["rho0"] + float(g.sum()),
        momentum=[float((rho * u[a]).sum()) for a in range(3)],
        phi_total=float(phi.sum()),
        free_energy=float(free_energy(phi, q_full(q5), p)),
        kinetic_energy=float((0.5 * rho * (u * u).sum(0)).sum()),
    )


def centre_linear(phi):
    """phi-weighted centre (x, y, z) with coordinates in [0, n)."""
    nz, ny, nx = phi.shape
    tot = phi.sum()
    zc = (phi.sum((1, 2)) * torch.arange(nz, dtype=DT)).sum() / tot
    yc = (phi.sum((0, 2)) * torch.arange(ny, dtype=DT)).sum() / tot
    xc = (phi.sum((0, 1)) * torch.arange(nx, dtype=DT)).sum() / tot
    return torch.stack([xc, yc, zc])


def centre_circular(phi):
    """Circular-mean centre per axis: n/(2pi) atan2(sum phi sin, sum phi cos) in [0, n)."""
    import math
    out = []
    for dim, n in ((2, phi.shape[2]), (1, phi.shape[1]), (0, phi.shape[0])):
        other = tuple(d for d in range(3) if d != dim)
        prof = phi.sum(other)
        th = 2 * math.pi * torch.arange(n, dtype=DT) / n
        ang = torch.atan2((prof * torch.sin(th)).sum(), (prof * torch.cos(th)).sum())
        out.append(torch.remainder(ang * n / (2 * math.pi), n))
    return torch.stack(out)


def displacement_loss(phi_T, zc0):
    """Squared displacement of the linear phi-weighted centre along z."""
    return (centre_linear(phi_T)[2] - zc0) ** 2
