"""Seeded synthetic inputs: parameter sets and initial fields.

This module is shared by the HIP path, its tests, the benchmark and the
CPU oracle's tests.  It holds no step arithmetic of the method: only the
parameter values of the droplet workloads and the construction of the
initial droplet (phi), the cholesteric helix inside it (Q) and the seeded
noise, plus plain random fields for parity tests.  It depends on numpy only.

Field layout everywhere: numpy float64 arrays shaped [nz, ny, nx] (x fastest);
the 5 stored Q components are ordered (xx, xy, xz, yy, yz) and Q_zz = -Q_xx - Q_yy.
"""
from __future__ import annotations

import math

import numpy as np

# Model constants shared by every droplet workload (free energy Eq. (5),
# Cahn-Hilliard Eq. (1), Beris-Edwards Eq. (2), BGK Eq. (7)).  chi0 and chi_s
# are chosen so that chi(phi_cr = 1) = 2.7 (the liquid-crystal threshold of
# Sec. 2) and chi(phi0 = 2) = 3, whose bulk order parameter is S = 0.5.
BASE_PARAMS = dict(
    tau=2.5, rho0=1.0,
    a=0.07, phi0=2.0, phi_cr=1.0, k_phi=0.1, M=0.1,
    A0=1.0, chi0=2.4, chi_s=0.3, K=0.02, q0=0.0, W=0.02,
    Gamma=0.3, xi=0.7, zeta=0.0,
    body_force=(0.0, 0.0, 0.0),
)

# The droplet workloads: periodic cubic box of side n, droplet radius R,
# cholesteric wavenumber q0, activity zeta, steps and precision(s).
WORKLOADS = {
    "droplet16": dict(n=16, R=5.0, q0=2 * math.pi / 8, zeta=0.005, steps=100, precisions=("fp64",)),
    "droplet64": dict(n=64, R=16.0, q0=2 * math.pi / 16, zeta=0.005, steps=2000, precisions=("fp64", "fp32"),
                      zetas=(0.0, 0.005, 0.01)),
    "droplet128": dict(n=128, R=32.0, q0=2 * math.pi / 24, zeta=0.008, steps=5000, precisions=("fp32", "fp16s")),
    "droplet32_adjoint": dict(n=32, R=8.0, q0=2 * math.pi / 12, zeta=0.006, steps=400, checkpoint=20,
                              precisions=("fp32",)),
    "droplet256": dict(n=256, R=64.0, q0=2 * math.pi / 32, zeta=0.01, steps=1000, adjoint_steps=50,
                       checkpoint=10, precisions=("fp32",)),
}


def params_for(workload: str, **overrides) -> dict:
    """Parameter dict of a named workload, with optional overrides."""
    w = WORKLOADS[workload]
    p = dict(BASE_PARAMS)
    p["q0"] = w["q0"]
    p["zeta"] = w["zeta"]
    p.update(overrides)
    return p


def droplet_fields(nx: int, ny: int, nz: int, R: float, q0: float, *, S0: float = 0.5,
                   noise: float = 0.01, seed: int = 0, phi0: float = 2.0, phi_cr: float = 1.0,
                   width: float = 1.0):
    """Initial droplet: returns (phi [nz,ny,nx], q5 [5,nz,ny,nx]) in float64.

    phi = (phi0/2)[1 + tanh((R - r)/width)] around the box centre
    (nx/2, ny/2, nz/2) with r the plain Euclidean distance (R <= n/4, so no
    periodic image is needed).  Where phi > phi_cr the order is a cholesteric
    helix along z: Q = S0 (n n - I/3) with n = (cos q0 z, sin q0 z, 0), z the
    integer lattice index, plus independent uniform noise in [-noise, noise)
    on each of the 5 stored components drawn as
    default_rng(seed).uniform(-noise, noise, (5, nz, ny, nx)); Q = 0 elsewhere.
    """
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    r = np.sqrt((x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - nz / 2) ** 2)
    phi = 0.5 * phi0 * (1.0 + np.tanh((R - r) / width))
    inside = phi > phi_cr
    c, s = np.cos(q0 * z), np.sin(q0 * z)
    q5 = np.empty((5, nz, ny, nx))
    q5[0] = S0 * (c * c - 1.0 / 3.0)
    q5[1] = S0 * c * s
    q5[2] = 0.0
    q5[3] = S0 * (s * s - 1.0 / 3.0)
    q5[4] = 0.0
    if noise:
        q5 += np.random.default_rng(seed).uniform(-noise, noise, (5, nz, ny, nx))
    q5 *= inside[None]
    return phi, q5


def workload_fields(workload: str, seed: int = 0):
    """(phi, q5) of a named workload's initial droplet."""
    w = WORKLOADS[workload]
    n = w["n"]
    return droplet_fields(n, n, n, w["R"], w["q0"], seed=seed)


def random_fields(nx: int, ny: int, nz: int, seed: int, *, g_amp: float = 1e-3, q_amp: float = 0.2,
                  phi_lo: float = 0.0, phi_hi: float = 2.0, u_amp: float = 0.0):
    """Plain random state for parity tests: (g [19,nz,ny,nx] deviations, phi, q5).

    g deviations are uniform in [-g_amp, g_amp); phi uniform in [phi_lo, phi_hi);
    the 5 stored Q components uniform in [-q_amp, q_amp).
    """
    rng = np.random.default_rng(seed)
    g = rng.uniform(-g_amp, g_amp, (19, nz, ny, nx))
    phi = rng.uniform(phi_lo, phi_hi, (nz, ny, nx))
    q5 = rng.uniform(-q_amp, q_amp, (5, nz, ny, nx))
    return g, phi, q5


def smooth_fields(nx: int, ny: int, nz: int, seed: int, *, modes: int = 3, q_amp: float = 0.2,
                  phi_mean: float = 1.0, phi_amp: float = 0.5):
    """Smooth periodic fields (a few low Fourier modes with seeded phases).

    Returns (phi, q5); used where a continuum limit is compared.
    """
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    kx, ky, kz = 2 * np.pi / nx, 2 * np.pi / ny, 2 * np.pi / nz

    def field(amp):
        f = np.zeros((nz, ny, nx))
        for _ in range(modes):
            mx, my, mz = rng.integers(0, 2, size=3)
            if mx == my == mz == 0:
                mx = 1
            ph = rng.uniform(0, 2 * np.pi)
            f += rng.uniform(0.5, 1.0) * np.cos(mx * kx * x + my * ky * y + mz * kz * z + ph)
        return amp * f / modes

    phi = phi_mean + field(phi_amp)
    q5 = np.stack([field(q_amp) for _ in range(5)])
    return phi, q5


def ic_shear_wave(n_z: int, U0: float, nx: int = 3, ny: int = 3):
    """u_x = U0 sin(2 pi z / n_z) on an nx x ny x n_z box (float64, [3,nz,ny,nx])."""
    z = np.arange(n_z, dtype=np.float64)
    u = np.zeros((3, n_z, ny, nx))
    u[0] = U0 * np.sin(2 * np.pi * z / n_z)[:, None, None]
    return u


# ----------------------------------------------------------------- 2D nematic
# Bulk active nematic on D2Q9 (the regimes of Fig. 4; the paper gives no 2D
# parameters, so these stand in): chi = 4 puts the bulk in the nematic phase
# with S_eq = sqrt(2 (chi/3 - 1)/chi) = 0.408.
NEMATIC2D_PARAMS = dict(tau=2.5, rho0=1.0, A0=0.1, chi=4.0, K=0.04, Gamma=0.3, xi=0.7, zeta=0.0)

# Director along x with +-0.05 rad of seeded noise, S0 = S_eq.  The regimes of
# Fig. 4 on these parameters: quiescent below the finite-box threshold
# (zeta = 0.0005 on 64^2), a stationary spontaneous flow (zeta = 0.002 on
# 128^2), active turbulence with +-1/2 defects (zeta >= 0.01).
NEMATIC2D_WORKLOADS = {
    "nematic64": dict(n=64, zeta=0.005, S0=0.408, noise=0.05, steps=200),      # FP64 parity
    "quiescent64": dict(n=64, zeta=0.0005, S0=0.408, noise=0.05, steps=10000),
    "flow128": dict(n=128, zeta=0.002, S0=0.408, noise=0.05, steps=10000),
    "chaos128": dict(n=128, zeta=0.02, S0=0.408, noise=0.05, steps=10000),
    "nematic512": dict(n=512, zeta=0.02, S0=0.408, noise=0.05, steps=2000),    # benchmark (Fig. 3 2D size)
}


def nematic2d_params(workload: str, **overrides) -> dict:
    p = dict(NEMATIC2D_PARAMS)
    p["zeta"] = NEMATIC2D_WORKLOADS[workload]["zeta"]
    p.update(overrides)
    return p


def nematic_fields(nx: int, ny: int, S0: float, noise: float, seed: int = 0) -> np.ndarray:
    """q2 [2, ny, nx] of a director along x with uniform angle noise in
    [-noise, noise] radians: Q = S0 (n n - I/2)."""
    th = np.random.default_rng(seed).uniform(-noise, noise, (ny, nx))
    return np.stack([0.5 * S0 * np.cos(2 * th), 0.5 * S0 * np.sin(2 * th)])


def nematic2d_workload_fields(workload: str, seed: int = 0) -> np.ndarray:
    w = NEMATIC2D_WORKLOADS[workload]
    return nematic_fields(w["n"], w["n"], w["S0"], w["noise"], seed)
