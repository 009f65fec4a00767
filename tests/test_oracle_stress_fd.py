"""Pins of the oracle's stress (Eqs. (3)-(4)) and order-parameter updates (Eqs. (1)-(2)).

* momentum: the force sums to zero on a periodic box for any Q, phi;
* Gibbs-Duhem: div of the interfacial + Ericksen stress converges at second
  order to mu grad(phi) - grad(Q):H, the continuum identity for the
  thermodynamic stress of Eq. (5) with the free-energy density as its
  isotropic part;
* reactive couplings conserve energy: sigma_react : W + H : S equals the
  isotropic term (2 xi/3)(Q:H) tr(W), for random tensors;
* co-rotation: a rigid rotation rotates Q (S = Om Q - Q Om for any xi);
  extensional flow on an isotropic state gives S = (2 xi/3) D (rods align
  with the stretching axis for xi > 0);
* active stress: closed-form force of a sinusoidal Q;
* Cahn-Hilliard: sum of phi is conserved;
* relaxation: with u = 0 the explicit step decreases F_h monotonically;
  a cholesteric helix with noise keeps its pitch while the noise decays.
"""
import math

import numpy as np
import pytest
import torch

from oracle import brute, core
from paper_2011_00287_amd import inputs

DT = torch.float64


def _p(**kw):
    return dict(inputs.BASE_PARAMS, **kw)


def _t(a):
    return torch.tensor(a, dtype=DT)


def test_total_force_vanishes():
    p = _p(q0=0.9, zeta=0.01)
    _, phi, q5 = inputs.random_fields(5, 6, 4, seed=21, q_amp=0.3)
    sig = core.stress(_t(phi), core.q_full(_t(q5)), p)
    F = core.force(sig, p)
    scale = float(sig.abs().max())
    assert float(F.sum((1, 2, 3)).abs().max()) < 1e-13 * scale * phi.size


def _gd_error(n, p, seed=5, transpose=False):
    phi_np, q5_np = inputs.smooth_fields(n, n, n, seed, q_amp=0.15, phi_mean=1.0, phi_amp=0.6)
    phi, Q = _t(phi_np), core.q_full(_t(q5_np))
    mu = core.chemical_potential(phi, Q, p)
    H = core.molecular_field(phi, Q, p)
    fc = core.free_energy_density_c(phi, Q, p)
    sig = core.stress_interfacial(phi, Q, fc, p) + core.stress_ericksen_q(Q, p)
    if transpose:
        sig = sig.transpose(0, 1)
    F = core.force(sig, dict(p, body_force=(0, 0, 0)))
    dQ = core.grad_q(Q)
    expect = torch.stack([mu * core.d0(phi, a) - (dQ[a] * H).sum((0, 1)) for a in range(3)])
    return float((F - expect).abs().max()) / float(expect.abs().max())


@pytest.mark.parametrize("bulk", [True, False])
def test_gibbs_duhem_second_order(bulk):
    """Refining a smooth field by 2 cuts the mismatch by ~4.

    q0 scales with the box so that the continuum problem is the same at both
    resolutions.  Without the bulk terms every force term is third order in
    gradients, which makes the check sensitive to the gradient terms alone.
    """
    over = {} if bulk else dict(a=0.0, A0=0.0, W=0.1)
    p = _p(**over)
    e1 = _gd_error(12, dict(p, q0=2 * math.pi / 12))
    e2 = _gd_error(24, dict(p, q0=2 * math.pi / 24))
    assert e2 < 0.05
    assert 3.0 < e1 / e2 < 5.0


def test_gibbs_duhem_detects_transposed_index():
    """The force index order matters: sigma transposed misses by O(1) and does not converge."""
    p = _p(a=0.0, A0=0.0, W=0.1, q0=2 * math.pi / 24)
    good = _gd_error(24, p)
    bad = _gd_error(24, p, transpose=True)
    bad12 = _gd_error(12, dict(p, q0=2 * math.pi / 12), transpose=True)
    assert bad > 5 * good and bad > 0.8 * bad12


def _sym_traceless(rng):
    A = rng.normal(size=(3, 3))
    A = 0.5 * (A + A.T)
    return A - np.eye(3) * np.trace(A) / 3


def test_reactive_stress_energy_identity():
    rng = np.random.default_rng(7)
    p = _p(xi=0.7)
    for _ in range(5):
        Q = _sym_traceless(rng) * 0.3
        H = _sym_traceless(rng)
        Wt = rng.normal(size=(3, 3)) * 0.1
        Qt = _t(Q).reshape(3, 3, 1, 1, 1)
        Ht = _t(H).reshape(3, 3, 1, 1, 1)
        Wtt = _t(Wt).reshape(3, 3, 1, 1, 1)
        sig = core.stress_reactive(Qt, Ht, p)
        S = core.corotation_from_w(Wtt, Qt, p)
        lhs = float((sig * Wtt).sum() + (Ht * S).sum())
        rhs = 2 * p["xi"] / 3 * float((Qt * Ht).sum()) * np.trace(Wt)
        assert abs(lhs - rhs) < 1e-14


def test_corotation_rigid_rotation():
    rng = np.random.default_rng(8)
    for xi in (0.0, 0.7, -0.4):
        Q = _sym_traceless(rng) * 0.3
        A = rng.normal(size=(3, 3))
        Om = 0.5 * (A - A.T) * 0.1
        S = core.corotation_from_w(_t(Om).reshape(3, 3, 1, 1, 1), _t(Q).reshape(3, 3, 1, 1, 1), _p(xi=xi))
        assert np.allclose(S.reshape(3, 3).numpy(), Om @ Q - Q @ Om, atol=1e-15)


def test_corotation_extension_aligns_rods():
    D = np.diag([1.0, -0.5, -0.5]) * 1e-2
    S = core.corotation_from_w(_t(D).reshape(3, 3, 1, 1, 1), torch.zeros(3, 3, 1, 1, 1, dtype=DT), _p(xi=0.7))
    assert np.allclose(S.reshape(3, 3).numpy(), 2 * 0.7 / 3 * D, atol=1e-16)
    assert S[0, 0].item() > 0


def test_active_force_closed_form():
    """phi uniform, Q_xz = A sin(kz): F_x = -zeta phi A sin(k) cos(kz), other components 0."""
    nz, A, zeta = 16, 0.1, 0.01
    k = 2 * math.pi / nz
    p = _p(zeta=zeta, A0=0.0, K=0.0, W=0.0, xi=0.0, a=0.0, k_phi=0.0)
    q5 = np.zeros((5, nz, 3, 3))
    z = np.arange(nz)
    q5[2] = (A * np.sin(k * z))[:, None, None]
    phi = torch.full((nz, 3, 3), 2.0, dtype=DT)
    F = core.force(core.stress(phi, core.q_full(_t(q5)), p), p)
    expect = -zeta * 2.0 * A * math.sin(k) * np.cos(k * z)
    assert np.allclose(F[0, :, 0, 0].numpy(), expect, atol=1e-17)
    assert float(F[1].abs().max()) == 0.0 and float(F[2].abs().max()) < 1e-18


def test_phi_is_conserved_and_q_stays_traceless():
    p = _p(q0=0.6, zeta=0.01)
    g, phi, q5 = inputs.random_fields(5, 4, 6, seed=9, q_amp=0.2, g_amp=1e-3)
    g, q5, phi = core.run(_t(g), _t(q5), _t(phi), p, 3)
    phi0 = inputs.random_fields(5, 4, 6, seed=9)[1].sum()
    assert abs(float(phi.sum()) - phi0) < 1e-12 * phi0
    assert q5.shape[0] == 5


def _relax_step(q5, phi, p):
    Q = core.q_full(q5)
    mu = core.chemical_potential(phi, Q, p)
    H = core.molecular_field(phi, Q, p)
    u = torch.zeros((3,) + tuple(phi.shape), dtype=DT)
    return core.q5_of(core.update_q(Q, u, H, p)), core.update_phi(phi, u, mu, p)


def test_relaxation_decreases_free_energy():
    """u = 0: the explicit Gamma*H and M*lap(mu) steps are gradient steps of F_h."""
    p = _p(q0=2 * math.pi / 8, zeta=0.0)
    phi_np, q5_np = inputs.droplet_fields(12, 12, 12, 3.5, p["q0"], seed=2)
    phi, q5 = _t(phi_np), _t(q5_np)
    F_prev = float(core.free_energy(phi, core.q_full(q5), p))
    for _ in range(40):
        q5, phi = _relax_step(q5, phi, p)
        F = float(core.free_energy(phi, core.q_full(q5), p))
        assert F <= F_prev + 1e-13 * abs(F_prev)
        F_prev = F


def test_cholesteric_keeps_pitch_and_noise_decays():
    """Bulk phi = phi0, zeta = 0: a helix at the lattice-optimal wavenumber plus noise relaxes."""
    nz = 32
    q0 = 2 * math.pi / 16
    p = _p(q0=q0, zeta=0.0)
    m = 2  # k = 2 pi m / nz = q0
    phi_np = np.full((nz, 4, 4), p["phi0"])
    z = np.arange(nz)
    k = 2 * math.pi * m / nz
    q5_np = np.zeros((5, nz, 4, 4))
    c, s = np.cos(k * z), np.sin(k * z)
    q5_np[0] = (0.5 * (c * c - 1 / 3))[:, None, None]
    q5_np[1] = (0.5 * c * s)[:, None, None]
    q5_np[3] = (0.5 * (s * s - 1 / 3))[:, None, None]
    q5_np += np.random.default_rng(0).uniform(-0.01, 0.01, q5_np.shape)
    g = torch.zeros((19, nz, 4, 4), dtype=DT)
    q5, phi = _t(q5_np), _t(phi_np)

    def noise(q):
        qm = q.mean((2, 3), keepdim=True)
        return float((q - qm).abs().max())

    def phase_mode(q):
        prof = q[1].mean((1, 2)).numpy()
        spec = np.abs(np.fft.rfft(prof))
        return int(np.argmax(spec[1:]) + 1)

    n0 = noise(q5)
    g, q5, phi = core.run(g, q5, phi, p, 60)
    assert noise(q5) < 0.3 * n0
    assert phase_mode(q5) == 2 * m  # Q_xy ~ sin(2kz): 2m periods along z
    rho, u = core.observe(g, q5, phi, p)
    assert float(u.abs().max()) < 1e-3


def test_whole_step_matches_per_site_loops():
    """O2 (per-site loops) == O1 (rolled tensors) on small odd boxes."""
    p = _p(q0=2 * math.pi / 5, zeta=0.01, body_force=(1e-4, -2e-4, 3e-4))
    for shape in ((4, 4, 4), (5, 3, 4), (6, 6, 6)):
        g, phi, q5 = inputs.random_fields(*shape, seed=sum(shape), q_amp=0.3, g_amp=2e-3)
        gb, qb, pb = brute.step(g, q5, phi, p)
        go, qo, po = core.step(_t(g), _t(q5), _t(phi), p)
        for a, b in ((gb, go), (qb, qo), (pb, po)):
            b = b.numpy()
            assert np.abs(a - b).max() <= 1e-14 * max(1e-3, np.abs(b).max())
