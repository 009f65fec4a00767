"""Pins of the oracle's free energy, chemical potential and molecular field (Eq. (5)).

* the Landau-de Gennes bulk: its ordered minimum S_eq(chi) in closed form,
  H = 0 there, and the isotropic-nematic coexistence at chi = 2.7 that the
  paper states as the liquid-crystal threshold;
* the double well: minima at phi = 0 and phi0, and the tanh interface of the
  continuum theory (mu = 0 on it); the excess free energy of planar
  interfaces tends to the closed-form surface tension sqrt(a k_phi) phi0^3 / 6
  per unit area, at second order in the interface resolution;
* mu and H are the exact lattice gradients of the discrete free energy
  (brute-force central differences on a 4^3 box);
* the cholesteric term: free energy per site of a lattice helix in closed
  form, its minimum at tan 2k = 2 q0, and the closed-form H of a helix;
* tangential anchoring for W > 0.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import core
from paper_2011_00287_amd import inputs

DT = torch.float64
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _p(**kw):
    return dict(inputs.BASE_PARAMS, **kw)


def _uniaxial(S, n, shape):
    n = np.asarray(n, dtype=float)
    n = n / np.linalg.norm(n)
    Q = S * (np.outer(n, n) - np.eye(3) / 3)
    q5 = np.array([Q[0, 0], Q[0, 1], Q[0, 2], Q[1, 1], Q[1, 2]])
    return torch.tensor(np.broadcast_to(q5[:, None, None, None], (5,) + shape).copy(), dtype=DT)


def s_eq(chi):
    """Ordered minimum of the LdG bulk of Eq. (5) for a uniaxial Q (closed form)."""
    return 0.25 + 0.75 * math.sqrt(1.0 - 8.0 / (3.0 * chi))


def test_parameters_match_paper_threshold():
    p = _p()
    chi_cr = p["chi0"] + p["chi_s"] * GOLD["phi_cr"]["value"]
    assert abs(chi_cr - GOLD["chi_liquid_crystal_threshold"]["value"]) < 1e-12
    assert abs(s_eq(p["chi0"] + p["chi_s"] * p["phi0"]) - 0.5) < 1e-12


@pytest.mark.parametrize("chi", [2.8, 3.0, 3.5])
def test_uniform_nematic_is_stationary(chi):
    """phi uniform, q0 = 0, Q = S_eq(nn - I/3): H = 0 and mu is uniform."""
    shape = (4, 4, 4)
    phi0 = 2.0
    p = _p(chi0=chi - 0.3 * phi0, q0=0.0)
    phi = torch.full(shape, phi0, dtype=DT)
    for n in ((1, 0, 0), (1, 2, -0.5)):
        Q = core.q_full(_uniaxial(s_eq(chi), n, shape))
        H = core.molecular_field(phi, Q, p)
        assert float(H.abs().max()) < 1e-15
        mu = core.chemical_potential(phi, Q, p)
        assert float((mu - mu.mean()).abs().max()) < 1e-15


def test_isotropic_nematic_coexistence_at_threshold():
    """At chi = 2.7 the ordered minimum has the same bulk free energy as Q = 0."""
    chi = GOLD["chi_liquid_crystal_threshold"]["value"]
    p = _p(q0=0.0, a=0.0, K=0.0, W=0.0, k_phi=0.0, chi0=chi, chi_s=0.0)
    phi = torch.zeros((3, 3, 3), dtype=DT)
    S = s_eq(chi)
    assert abs(S - 1.0 / 3.0) < 1e-12
    f_ord = core.free_energy(phi, core.q_full(_uniaxial(S, (0, 0, 1), (3, 3, 3))), p)
    assert abs(float(f_ord)) < 1e-14
    # just above the threshold the ordered state is lower; just below, higher
    for dchi, sign in ((0.05, -1), (-0.01, 1)):
        pc = dict(p, chi0=chi + dchi)
        c = chi + dchi
        S = 0.25 + 0.75 * math.sqrt(1 - 8 / (3 * c))
        f = float(core.free_energy(phi, core.q_full(_uniaxial(S, (0, 0, 1), (3, 3, 3))), pc))
        assert f * sign > 0


def test_double_well_minima():
    p = _p(A0=0.0, W=0.0)
    q = torch.zeros((5, 3, 3, 3), dtype=DT)
    for v in (0.0, p["phi0"]):
        phi = torch.full((3, 3, 3), v, dtype=DT)
        assert float(core.chemical_potential(phi, core.q_full(q), p).abs().max()) == 0.0
        assert float(core.free_energy(phi, core.q_full(q), p)) == 0.0
    phi = torch.full((3, 3, 3), 0.5 * p["phi0"], dtype=DT)
    assert float(core.free_energy(phi, core.q_full(q), p)) > 0


def test_tanh_interface_has_zero_mu():
    """The continuum flat interface phi0/2 [1 + tanh(kappa x)], kappa = phi0 sqrt(a/k_phi)/(2 phi_cr).

    On a lattice the residual mu is O(kappa^4); with a weak double well it is
    tiny compared with the bulk scale a phi0^3.
    """
    p = _p(a=0.07 / 64, A0=0.0, W=0.0)
    kappa = p["phi0"] * math.sqrt(p["a"] / p["k_phi"]) / (2 * p["phi_cr"])
    nx = 256
    x = np.arange(nx) - nx / 2
    prof = 0.5 * p["phi0"] * (1 + np.tanh(kappa * x) * (np.abs(x) < nx / 4) + np.sign(x) * (np.abs(x) >= nx / 4))
    # single interface region: compare well away from the clamped edges
    phi = torch.tensor(np.broadcast_to(prof, (3, 3, nx)).copy(), dtype=DT)
    mu = core.chemical_potential(phi, core.q_full(torch.zeros((5, 3, 3, nx), dtype=DT)), p)[0, 0]
    core_region = slice(nx // 2 - 20, nx // 2 + 20)
    scale = p["a"] * p["phi0"] ** 3
    assert float(mu[core_region].abs().max()) < 2e-3 * scale
    # and a wrong width is clearly not stationary
    prof2 = 0.5 * p["phi0"] * (1 + np.tanh(1.3 * kappa * x))
    phi2 = torch.tensor(np.broadcast_to(prof2, (3, 3, nx)).copy(), dtype=DT)
    mu2 = core.chemical_potential(phi2, core.q_full(torch.zeros((5, 3, 3, nx), dtype=DT)), p)[0, 0]
    assert float(mu2[core_region].abs().max()) > 0.05 * scale


BASIS = [np.array(m, dtype=float) for m in (
    [[1, 0, 0], [0, 0, 0], [0, 0, -1]],
    [[0, 1, 0], [1, 0, 0], [0, 0, 0]],
    [[0, 0, 1], [0, 0, 0], [1, 0, 0]],
    [[0, 0, 0], [0, 1, 0], [0, 0, -1]],
    [[0, 0, 0], [0, 0, 1], [0, 1, 0]],
)]


def _planar_interfaces_ratio(k_phi):
    """F_h of two planar tanh interfaces (Q = 0) over 2 sigma A, sigma = sqrt(a k_phi) phi0^3 / 6."""
    p = _p(q0=0.0, zeta=0.0, W=0.0, k_phi=k_phi)
    kappa = p["phi0"] * math.sqrt(p["a"] / p["k_phi"]) / 2.0
    sigma = math.sqrt(p["a"] * p["k_phi"]) * p["phi0"] ** 3 / 6.0
    nx, ny, nz = 128, 3, 3
    x = np.arange(nx)
    prof = 0.5 * p["phi0"] * (np.tanh(kappa * (x - nx / 4 - 0.3)) - np.tanh(kappa * (x - 3 * nx / 4 - 0.3)))
    phi = torch.tensor(np.broadcast_to(prof[None, None, :], (nz, ny, nx)).copy(), dtype=DT)
    Q = core.q_full(torch.zeros((5, nz, ny, nx), dtype=DT))
    return float(core.free_energy(phi, Q, p)) / (2.0 * sigma * ny * nz), kappa


def test_interface_tension_closed_form():
    """Bulk phases at phi = 0 and phi0 cost nothing, so F_h is the interfaces' excess:
    2 sigma A in the continuum.  On the lattice the error is O(kappa^2): it must
    shrink about 4-fold each time the interface width doubles (k_phi x 4)."""
    errs = []
    for k_phi in (0.1, 0.4, 1.6):
        ratio, kappa = _planar_interfaces_ratio(k_phi)
        errs.append(abs(ratio - 1.0))
    assert errs[0] < 0.03 and errs[2] < 2e-3, errs
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.5 < e0 / e1 < 4.5, errs


def test_mu_and_h_are_exact_gradients_of_free_energy():
    """Brute force on 4^3: central differences of F_h at every (site, field)."""
    p = _p(q0=2 * math.pi / 5)
    _, phi_np, q5_np = inputs.random_fields(4, 4, 4, seed=11, q_amp=0.3)
    phi = torch.tensor(phi_np, dtype=DT)
    q5 = torch.tensor(q5_np, dtype=DT)
    mu = core.chemical_potential(phi, core.q_full(q5), p)
    H = core.molecular_field(phi, core.q_full(q5), p)
    h = 1e-5
    rng = np.random.default_rng(0)
    sites = [tuple(s) for s in rng.integers(0, 4, size=(12, 3))]
    for s in sites:
        e = torch.zeros_like(phi)
        e[s] = h
        num = (core.free_energy(phi + e, core.q_full(q5), p) - core.free_energy(phi - e, core.q_full(q5), p)) / (2 * h)
        assert abs(float(num) - float(mu[s])) < 1e-8 * max(1.0, abs(float(mu[s])))
        for k in range(5):
            e5 = torch.zeros_like(q5)
            e5[(k,) + s] = h
            num = (core.free_energy(phi, core.q_full(q5 + e5), p) - core.free_energy(phi, core.q_full(q5 - e5), p)) / (2 * h)
            ana = -float((H[(slice(None), slice(None)) + s] * torch.tensor(BASIS[k], dtype=DT)).sum())
            assert abs(float(num) - ana) < 1e-8 * max(1.0, abs(ana))


def test_h_is_traceless_symmetric():
    p = _p(q0=0.7)
    _, phi_np, q5_np = inputs.random_fields(5, 4, 6, seed=3, q_amp=0.3)
    H = core.molecular_field(torch.tensor(phi_np), core.q_full(torch.tensor(q5_np)), p)
    assert float((H - H.transpose(0, 1)).abs().max()) < 1e-15
    assert float((H[0, 0] + H[1, 1] + H[2, 2]).abs().max()) < 1e-14


def _helix(k, S, nz, nxy=3):
    z = np.arange(nz, dtype=float)
    q5 = np.zeros((5, nz, nxy, nxy))
    c, s = np.cos(k * z), np.sin(k * z)
    q5[0] = (S * (c * c - 1 / 3))[:, None, None]
    q5[1] = (S * c * s)[:, None, None]
    q5[3] = (S * (s * s - 1 / 3))[:, None, None]
    return torch.tensor(q5, dtype=DT)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_helix_free_energy_closed_form(m):
    """Per site: bulk + K S^2 (sin^2 k - q0 sin 2k) + (4/3) K q0^2 S^2 for n = (cos kz, sin kz, 0)."""
    nz = 24
    k = 2 * math.pi * m / nz
    q0 = 2 * math.pi / 16
    S = 0.5
    p = _p(q0=q0, W=0.0)
    phi = torch.full((nz, 3, 3), p["phi0"], dtype=DT)
    Fh = float(core.free_energy(phi, core.q_full(_helix(k, S, nz)), p)) / phi.numel()
    chi = p["chi0"] + p["chi_s"] * p["phi0"]
    bulk = p["A0"] * ((1 - chi / 3) * S * S / 3 - 2 * chi * S ** 3 / 27 + chi * S ** 4 / 9)
    expect = bulk + p["K"] * S * S * (math.sin(k) ** 2 - q0 * math.sin(2 * k)) + 4 / 3 * p["K"] * q0 * q0 * S * S
    assert abs(Fh - expect) < 1e-14


def test_helix_pitch_minimises_free_energy():
    """Among lattice helices the free energy is lowest at tan 2k = 2 q0, which tends to k = q0
    (pitch 2 pi / q0) as q0 -> 0; at q0 = 2 pi/16 the second-order stencils already shift it by 15 %."""
    for q0, nz in ((2 * math.pi / 16, 64), (2 * math.pi / 48, 96)):
        p = _p(q0=q0, W=0.0)
        phi = torch.full((nz, 3, 3), p["phi0"], dtype=DT)
        ks = [2 * math.pi * m / nz for m in range(0, 9)]
        fs = [float(core.free_energy(phi, core.q_full(_helix(k, 0.5, nz)), p)) for k in ks]
        best = ks[int(np.argmin(fs))]
        kstar = 0.5 * math.atan(2 * q0)
        assert abs(best - kstar) <= math.pi / nz
        if q0 < 0.2:
            assert abs(best - q0) <= math.pi / nz
        # negative twist is penalised: the chiral term selects the handedness
        fneg = float(core.free_energy(phi, core.q_full(_helix(-best, 0.5, nz)), p))
        assert fneg > min(fs)


def test_helix_molecular_field_closed_form():
    """Elastic part of H on a helix: -4K[sin^2 k - q0 sin 2k + q0^2] Q_osc - 4 K q0^2 Q_const."""
    nz = 24
    k = 2 * math.pi * 2 / nz
    q0 = 2 * math.pi / 16
    S = 0.5
    p = _p(q0=q0, A0=0.0, W=0.0)
    phi = torch.full((nz, 3, 3), p["phi0"], dtype=DT)
    Q = core.q_full(_helix(k, S, nz))
    H = core.molecular_field(phi, Q, p)
    Qc = core.q_full(_helix(0.0, 0.0, nz))  # zeros
    Qconst = torch.zeros_like(Q)
    Qconst[0, 0] = Qconst[1, 1] = S / 6
    Qconst[2, 2] = -S / 3
    Qosc = Q - Qconst
    expect = -4 * p["K"] * (math.sin(k) ** 2 - q0 * math.sin(2 * k) + q0 * q0) * Qosc - 4 * p["K"] * q0 * q0 * Qconst
    assert float((H - expect).abs().max()) < 1e-15
    del Qc


def test_anchoring_is_tangential_for_positive_w():
    """A flat interface normal to z: W > 0 prefers the director in the interface plane."""
    assert GOLD["anchoring_tangential_for_positive_W"]["value"]
    nz = 32
    z = np.arange(nz) - nz / 2
    prof = 1 + np.tanh(z / 2.0) * (np.abs(z) < nz / 4) + np.sign(z) * (np.abs(z) >= nz / 4)
    phi = torch.tensor(np.broadcast_to(prof[:, None, None], (nz, 3, 3)).copy(), dtype=DT)
    for W, tangential_wins in ((0.02, True), (-0.02, False)):
        p = _p(W=W, q0=0.0)
        f_par = float(core.free_energy(phi, core.q_full(_uniaxial(0.5, (1, 0, 0), phi.shape)), p))
        f_nrm = float(core.free_energy(phi, core.q_full(_uniaxial(0.5, (0, 0, 1), phi.shape)), p))
        assert (f_par < f_nrm) == tangential_wins
