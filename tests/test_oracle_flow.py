"""Pins of the oracle's flow coupling (Sec. 2, Eqs. (1)-(2)) and of its observables.

Each check moves or measures a field with a known velocity or a known
position, so that a plausible slip in the oracle fails it:

* advection: under a uniform velocity u0 with every force and mobility
  switched off (Gamma = M = 0, no free-energy term, so the stress and F
  vanish and u = u0 exactly), one whole coupled step multiplies a Fourier
  mode e^{ikx} of phi and of each Q component by exactly 1 - i u0 sin k (the
  central-difference symbol of the material derivative -u.grad).  A flipped
  sign of the advection of Q or of the phi flux, or a dropped axis, fails;
* velocity gradient: W_ab = D0_b u_a for a shear u_x = U sin(ky) gives
  W_xy = U sin k cos(ky) and W_yx = 0;
* co-rotation under a rigid rotation u = w x (r - c): a uniform nematic
  Q = S0(nn - I/3) turns at the angular velocity w, i.e. its rate is
  S0[(w x n)n + n(w x n)] (director kinematics dn/dt = w x n, half the
  vorticity), for any xi.  A transposed W reverses the sense and fails;
* centres: phi concentrated at one site, and a droplet translated by a
  periodic shift, give that site and the shifted centre (linear and circular
  means), and the displacement loss of a shift s along z is s^2;
* totals: mass, momentum and kinetic energy of a uniform flow are
  N rho0, N rho0 u0 and N rho0 |u0|^2 / 2.
"""
import math

import numpy as np
import pytest
import torch

from oracle import core
from paper_2011_00287_amd import inputs

DT = torch.float64


def _still(**kw):
    """Parameters with every thermodynamic force and both mobilities off.

    a = k_phi = A0 = K = W = zeta = 0 make mu, H, the stress and F vanish
    identically; Gamma = M = 0 leave only the advection and co-rotation of
    the order parameters.
    """
    p = dict(inputs.BASE_PARAMS)
    p.update(a=0.0, k_phi=0.0, A0=0.0, K=0.0, W=0.0, zeta=0.0, q0=0.0, Gamma=0.0, M=0.0)
    p.update(kw)
    return p


def _uniform_flow_state(shape, u0, p):
    u = torch.stack([torch.full(shape, float(c), dtype=DT) for c in u0])
    return core.init_populations(u, p)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_uniform_advection_multiplies_modes_by_exact_symbol(axis, sign):
    shape = (6, 10, 8)  # [nz, ny, nx]: a different length per axis
    n = shape[2 - axis]
    m = 2
    k = 2 * math.pi * m / n
    U = sign * 0.03
    u0 = [0.011, -0.007, 0.005]  # components across the mode do not change it
    u0[axis] = U
    p = _still()
    g = _uniform_flow_state(shape, u0, p)
    coord = torch.arange(n, dtype=DT)
    view = [1, 1, 1]
    view[2 - axis] = n
    xa = coord.reshape(view).expand(shape)
    # phi = 1 + 0.2 cos(k x + 0.3); Q components with their own phase
    phases = [0.3, 1.1, -0.4, 2.0, 0.7, -1.3]
    amps = [0.2, 0.05, -0.03, 0.04, 0.02, -0.06]
    modes = [a * torch.cos(k * xa + th) for a, th in zip(amps, phases)]
    phi = 1.0 + modes[0]
    q5 = torch.stack(modes[1:])
    g1, q5_1, phi_1 = core.step(g, q5, phi, p)
    # exact: Re[(1 - i U sin k) A e^{i(kx + th)}] = A cos(kx + th) + U sin k A sin(kx + th)
    expect = [a * (torch.cos(k * xa + th) + U * math.sin(k) * torch.sin(k * xa + th)) for a, th in zip(amps, phases)]
    assert torch.allclose(phi_1, 1.0 + expect[0], rtol=0, atol=1e-15)
    assert torch.allclose(q5_1, torch.stack(expect[1:]), rtol=0, atol=1e-15)
    # and the opposite sign of the symbol is far off (the pin can tell them apart)
    wrong = 1.0 + amps[0] * (torch.cos(k * xa + phases[0]) - U * math.sin(k) * torch.sin(k * xa + phases[0]))
    assert float((phi_1 - wrong).abs().max()) > 1e-3
    # the flow itself is untouched: populations of a uniform flow stream into themselves
    assert torch.allclose(g1, g, rtol=0, atol=1e-16)


def test_advection_of_phi_is_the_conservative_flux():
    """With a non-uniform u the flux form -D0.(u phi) differs from -u.D0 phi by -phi D0.u.

    A compressive velocity u_x = U sin(kx) at rest density (forces off) moves
    phi = const by exactly -phi0 U sin k cos(kx) in one step; the advective form
    would leave a uniform phi unchanged.
    """
    shape = (4, 5, 12)
    n = shape[2]
    k = 2 * math.pi / n
    U = 0.02
    p = _still()
    x = torch.arange(n, dtype=DT).reshape(1, 1, n).expand(shape)
    u = torch.stack([U * torch.sin(k * x), torch.zeros(shape, dtype=DT), torch.zeros(shape, dtype=DT)])
    g = core.init_populations(u, p)
    phi = torch.full(shape, 1.5, dtype=DT)
    q5 = torch.zeros((5,) + shape, dtype=DT)
    _, _, phi_1 = core.step(g, q5, phi, p)
    expect = 1.5 - 1.5 * U * math.sin(k) * torch.cos(k * x)
    assert torch.allclose(phi_1, expect, rtol=0, atol=1e-15)


def test_velocity_gradient_index_order_on_a_shear():
    shape = (3, 8, 5)
    ny = shape[1]
    k = 2 * math.pi / ny
    U = 0.04
    y = torch.arange(ny, dtype=DT).reshape(1, ny, 1).expand(shape)
    u = torch.stack([U * torch.sin(k * y), torch.zeros(shape, dtype=DT), torch.zeros(shape, dtype=DT)])
    W = core.velocity_gradient(u)
    assert torch.allclose(W[0, 1], U * math.sin(k) * torch.cos(k * y), rtol=0, atol=1e-16)
    for a in range(3):
        for b in range(3):
            if (a, b) != (0, 1):
                assert float(W[a, b].abs().max()) == 0.0, (a, b)


def _cross(w, n):
    return np.array([w[1] * n[2] - w[2] * n[1], w[2] * n[0] - w[0] * n[2], w[0] * n[1] - w[1] * n[0]])


@pytest.mark.parametrize("xi", [0.0, 0.7, -0.4])
def test_corotation_turns_a_nematic_with_the_rotation(xi):
    """u = w x (r - c) is linear, so D0 is exact at sites whose stencil does not wrap."""
    n_side = 9
    shape = (n_side, n_side, n_side)
    c = (n_side - 1) / 2
    w = np.array([0.003, -0.002, 0.005])
    idx = torch.arange(n_side, dtype=DT) - c
    z, y, x = torch.meshgrid(idx, idx, idx, indexing="ij")
    r = [x, y, z]
    u = torch.stack([w[1] * r[2] - w[2] * r[1], w[2] * r[0] - w[0] * r[2], w[0] * r[1] - w[1] * r[0]])
    nvec = np.array([0.6, 0.48, 0.64])
    nvec /= np.linalg.norm(nvec)
    S0 = 0.5
    Qm = S0 * (np.outer(nvec, nvec) - np.eye(3) / 3)
    Q = torch.tensor(Qm, dtype=DT).reshape(3, 3, 1, 1, 1).expand(3, 3, *shape).clone()
    S = core.corotation(u, Q, dict(inputs.BASE_PARAMS, xi=xi))
    wn = _cross(w, nvec)
    expect = S0 * (np.outer(wn, nvec) + np.outer(nvec, wn))  # traceless already: 2 S0 (w x n).n = 0
    inner = S[:, :, 1:-1, 1:-1, 1:-1]
    err = (inner - torch.tensor(expect, dtype=DT).reshape(3, 3, 1, 1, 1)).abs().max()
    assert float(err) < 1e-16, float(err)
    # the reverse sense (a transposed velocity gradient) is far off
    assert float((inner + torch.tensor(expect, dtype=DT).reshape(3, 3, 1, 1, 1)).abs().max()) > 1e-4


@pytest.mark.parametrize("site", [(0, 0, 0), (3, 5, 2), (6, 1, 4)])
def test_centres_of_a_point_mass(site):
    shape = (7, 8, 9)
    phi = torch.zeros(shape, dtype=DT)
    x, y, z = site
    phi[z, y, x] = 2.0
    assert torch.allclose(core.centre_linear(phi), torch.tensor([x, y, z], dtype=DT), rtol=0, atol=1e-15)
    assert torch.allclose(core.centre_circular(phi), torch.tensor([x, y, z], dtype=DT), rtol=0, atol=1e-12)


def test_centres_of_a_translated_droplet_and_the_loss():
    n = 24
    # a compact droplet, phi = 2 (1 - r^2/R^2) inside r < R, symmetric about
    # the box centre n/2 on every axis (a tanh tail would wrap round the box)
    idx = torch.arange(n, dtype=DT) - n / 2
    z, y, x = torch.meshgrid(idx, idx, idx, indexing="ij")
    phi0 = torch.clamp(2.0 * (1.0 - (x * x + y * y + z * z) / 36.0), min=0.0)
    assert torch.allclose(core.centre_linear(phi0), torch.full((3,), n / 2, dtype=DT), rtol=0, atol=1e-12)
    assert torch.allclose(core.centre_circular(phi0), torch.full((3,), n / 2, dtype=DT), rtol=0, atol=1e-12)
    for s in (1, 3, -2):
        phiT = torch.roll(phi0, shifts=s, dims=0)  # shift along z (no wrap of the droplet)
        zc = core.centre_linear(phiT)
        assert abs(float(zc[2]) - (n / 2 + s)) < 1e-12
        assert abs(float(zc[0]) - n / 2) < 1e-12 and abs(float(zc[1]) - n / 2) < 1e-12
        assert abs(float(core.displacement_loss(phiT, n / 2)) - s * s) < 1e-11
    # circular mean follows a shift across the periodic boundary
    big = 11
    phiW = torch.roll(phi0, shifts=(big, -big, 2 * big), dims=(2, 1, 0))
    expect = torch.remainder(torch.tensor([n / 2 + big, n / 2 - big, n / 2 + 2 * big], dtype=DT), n)
    got = core.centre_circular(phiW)
    d = torch.remainder(got - expect + n / 2, n) - n / 2
    assert float(d.abs().max()) < 1e-10


def test_totals_of_a_uniform_flow():
    shape = (4, 6, 5)
    u0 = (0.02, -0.01, 0.015)
    p = dict(inputs.BASE_PARAMS)
    g = _uniform_flow_state(shape, u0, p)
    # a phi at the double-well minimum 0 and Q = 0: no stress, u = u0 exactly
    phi = torch.zeros(shape, dtype=DT)
    q5 = torch.zeros((5,) + shape, dtype=DT)
    t = core.totals(g, q5, phi, p)
    n = phi.numel()
    assert abs(t["mass"] - n * p["rho0"]) < 1e-12
    for a in range(3):
        assert abs(t["momentum"][a] - n * p["rho0"] * u0[a]) < 1e-14
    assert abs(t["kinetic_energy"] - n * p["rho0"] * sum(c * c for c in u0) / 2) < 1e-15
    assert t["phi_total"] == 0.0 and t["free_energy"] == 0.0
