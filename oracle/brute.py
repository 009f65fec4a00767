"""Per-site loop version of the coupled step, for tiny boxes (4^3 - 6^3).

TEST INFRASTRUCTURE ONLY.  It computes the same step as core.py, written
independently with explicit periodic neighbour indices and explicit index
loops instead of rolled whole-field tensors, so that a wrong shift direction,
a transposed index or a dropped term in either version shows up as a
mismatch.  Plain Python floats throughout; arrays are numpy [nz, ny, nx].
"""
from __future__ import annotations

import numpy as np

from .lattice import C19, W19

LC = {(0, 1, 2): 1.0, (1, 2, 0): 1.0, (2, 0, 1): 1.0, (0, 2, 1): -1.0, (2, 1, 0): -1.0, (1, 0, 2): -1.0}


def eps(a, b, c):
    return LC.get((a, b, c), 0.0)


def _qmat(q5, z, y, x):
    xx, xy, xz, yy, yz = (float(q5[k, z, y, x]) for k in range(5))
    return [[xx, xy, xz], [xy, yy, yz], [xz, yz, -xx - yy]]


def step(g, q5, phi, p):
    """One coupled step on numpy float64 arrays; returns (g, q5, phi) at t+1."""
    nz, ny, nx = phi.shape
    sites = [(z, y, x) for z in range(nz) for y in range(ny) for x in range(nx)]

    def nb(s, d, sgn):
        z, y, x = s
        off = [0, 0, 0]
        off[d] = sgn
        return ((z + off[2]) % nz, (y + off[1]) % ny, (x + off[0]) % nx)

    Qs = {s: _qmat(q5, *s) for s in sites}
    ph = {s: float(phi[s]) for s in sites}

    def d0s(val, s, d):
        return 0.5 * (val[nb(s, d, 1)] - val[nb(s, d, -1)])

    def lap_s(val, s):
        return sum(val[nb(s, d, 1)] + val[nb(s, d, -1)] for d in range(3)) - 6.0 * val[s]

    # gradients
    dphi, dQ, lphi, lQ = {}, {}, {}, {}
    for s in sites:
        dphi[s] = [d0s(ph, s, d) for d in range(3)]
        lphi[s] = lap_s(ph, s)
        dq = [[[0.0] * 3 for _ in range(3)] for _ in range(3)]
        lq = [[0.0] * 3 for _ in range(3)]
        for a in range(3):
            for b in range(3):
                comp = {t: Qs[t][a][b] for t in (s,) + tuple(nb(s, d, k) for d in range(3) for k in (1, -1))}
                for d in range(3):
                    dq[d][a][b] = 0.5 * (comp[nb(s, d, 1)] - comp[nb(s, d, -1)])
                lq[a][b] = sum(comp[nb(s, d, 1)] + comp[nb(s, d, -1)] for d in range(3)) - 6.0 * comp[s]
        dQ[s], lQ[s] = dq, lq

    # anchoring vector v_a = Q_ab D0_b phi
    vvec = {s: [sum(Qs[s][a][b] * dphi[s][b] for b in range(3)) for a in range(3)] for s in sites}

    mu, H, fc = {}, {}, {}
    for s in sites:
        Q = Qs[s]
        f = ph[s]
        chi = p["chi0"] + p["chi_s"] * f
        tr2 = sum(Q[a][b] * Q[a][b] for a in range(3) for b in range(3))
        Q2 = [[sum(Q[a][c] * Q[c][b] for c in range(3)) for b in range(3)] for a in range(3)]
        tr3 = sum(Q2[a][b] * Q[b][a] for a in range(3) for b in range(3))
        divv = sum(0.5 * (vvec[nb(s, a, 1)][a] - vvec[nb(s, a, -1)][a]) for a in range(3))
        mu[s] = (p["a"] * f * (f - p["phi0"]) * (2 * f - p["phi0"]) / p["phi_cr"] ** 2
                 + p["A0"] * p["chi_s"] * (-tr2 / 6 - tr3 / 3 + tr2 * tr2 / 4)
                 - p["k_phi"] * lphi[s] - 2 * p["W"] * divv)
        Cq = [[sum(eps(a, gg, d) * dQ[s][gg][d][b] for gg in range(3) for d in range(3)) for b in range(3)]
              for a in range(3)]
        gp2 = sum(x * x for x in dphi[s])
        h = [[0.0] * 3 for _ in range(3)]
        for a in range(3):
            for b in range(3):
                de = 1.0 if a == b else 0.0
                h[a][b] = (-p["A0"] * ((1 - chi / 3) * Q[a][b] - chi * (Q2[a][b] - de * tr2 / 3) + chi * Q[a][b] * tr2)
                           + p["K"] * lQ[s][a][b] - 2 * p["K"] * p["q0"] * (Cq[a][b] + Cq[b][a])
                           - 4 * p["K"] * p["q0"] ** 2 * Q[a][b]
                           - p["W"] * (dphi[s][a] * dphi[s][b] - de * gp2 / 3))
        H[s] = h
        gq2 = sum(dQ[s][gg][a][b] ** 2 for gg in range(3) for a in range(3) for b in range(3))
        qc = sum(Q[a][b] * Cq[a][b] for a in range(3) for b in range(3))
        anch = sum(dphi[s][a] * Q[a][b] * dphi[s][b] for a in range(3) for b in range(3))
        fc[s] = (0.5 * p["a"] * f * f * (f - p["phi0"]) ** 2 / p["phi_cr"] ** 2
                 + p["A0"] * (0.5 * (1 - chi / 3) * tr2 - chi / 3 * tr3 + chi / 4 * tr2 * tr2)
                 + 2 * p["K"] * p["q0"] ** 2 * tr2 + 0.5 * p["k_phi"] * gp2 + 0.5 * p["K"] * gq2
                 + 2 * p["K"] * p["q0"] * qc + p["W"] * anch)

    sig = {}
    for s in sites:
        Q, h, f, dp_, dq = Qs[s], H[s], ph[s], dphi[s], dQ[s]
        P = [[Q[a][b] + (1.0 / 3.0 if a == b else 0.0) for b in range(3)] for a in range(3)]
        qh = sum(Q[a][b] * h[a][b] for a in range(3) for b in range(3))
        sg = [[0.0] * 3 for _ in range(3)]
        for a in range(3):
            for b in range(3):
                de = 1.0 if a == b else 0.0
                t = p["k_phi"] * dp_[b] + 2 * p["W"] * sum(Q[b][gg] * dp_[gg] for gg in range(3))
                val = fc[s] * de - dp_[a] * t
                for gg in range(3):
                    for n in range(3):
                        dfd = p["K"] * dq[b][gg][n] + 2 * p["K"] * p["q0"] * sum(
                            eps(lam, b, gg) * Q[lam][n] for lam in range(3))
                        val -= dq[a][gg][n] * dfd
                hp = sum(h[a][c] * P[c][b] for c in range(3))
                pH = sum(P[a][c] * h[c][b] for c in range(3))
                qH = sum(Q[a][c] * h[c][b] for c in range(3))
                hQ = sum(h[a][c] * Q[c][b] for c in range(3))
                val += -p["xi"] * (hp + pH) + 2 * p["xi"] * P[a][b] * qh + (qH - hQ)
                val += -p["zeta"] * f * Q[a][b]
                sg[a][b] = val
        sig[s] = sg

    bf = p.get("body_force", (0.0, 0.0, 0.0))
    F = {}
    for s in sites:
        F[s] = [sum(0.5 * (sig[nb(s, b, 1)][a][b] - sig[nb(s, b, -1)][a][b]) for b in range(3)) + bf[a]
                for a in range(3)]

    tau = p["tau"]
    gstar = np.empty_like(g)
    U = {}
    for s in sites:
        gi = [float(g[i][s]) for i in range(19)]
        rho = p["rho0"] + sum(gi)
        u = [(sum(gi[i] * C19[i][a] for i in range(19)) + 0.5 * F[s][a]) / rho for a in range(3)]
        U[s] = u
        uu = sum(x * x for x in u)
        uF = sum(u[a] * F[s][a] for a in range(3))
        for i in range(19):
            cu = sum(C19[i][a] * u[a] for a in range(3))
            cF = sum(C19[i][a] * F[s][a] for a in range(3))
            geq = W19[i] * ((rho - p["rho0"]) + rho * (3 * cu + 4.5 * cu * cu - 1.5 * uu))
            src = (1 - 0.5 / tau) * W19[i] * (3 * (cF - uF) + 9 * cu * cF)
            gstar[i][s] = gi[i] - (gi[i] - geq) / tau + src
    g_new = np.empty_like(g)
    for s in sites:
        z, y, x = s
        for i in range(19):
            cx, cy, cz = C19[i]
            g_new[i][s] = gstar[i][(z - cz) % nz, (y - cy) % ny, (x - cx) % nx]

    q5_new = np.empty_like(q5)
    phi_new = np.empty_like(phi)
    xi = p["xi"]
    for s in sites:
        Q, h, u = Qs[s], H[s], U[s]
        Wt = [[0.5 * (U[nb(s, b, 1)][a] - U[nb(s, b, -1)][a]) for b in range(3)] for a in range(3)]
        D = [[0.5 * (Wt[a][b] + Wt[b][a]) for b in range(3)] for a in range(3)]
        Om = [[0.5 * (Wt[a][b] - Wt[b][a]) for b in range(3)] for a in range(3)]
        P = [[Q[a][b] + (1.0 / 3.0 if a == b else 0.0) for b in range(3)] for a in range(3)]
        trQW = sum(Q[a][b] * Wt[b][a] for a in range(3) for b in range(3))
        S = [[sum((xi * D[a][c] + Om[a][c]) * P[c][b] + P[a][c] * (xi * D[c][b] - Om[c][b]) for c in range(3))
              - 2 * xi * P[a][b] * trQW for b in range(3)] for a in range(3)]
        trS = S[0][0] + S[1][1] + S[2][2]
        Qn = [[0.0] * 3 for _ in range(3)]
        for a in range(3):
            for b in range(3):
                adv = sum(u[gg] * dQ[s][gg][a][b] for gg in range(3))
                Qn[a][b] = Q[a][b] + (-adv + S[a][b] - (trS / 3 if a == b else 0.0) + p["Gamma"] * h[a][b])
        q5_new[0][s], q5_new[1][s], q5_new[2][s] = Qn[0][0], Qn[0][1], Qn[0][2]
        q5_new[3][s], q5_new[4][s] = Qn[1][1], Qn[1][2]
        flux = sum(0.5 * (U[nb(s, gg, 1)][gg] * ph[nb(s, gg, 1)] - U[nb(s, gg, -1)][gg] * ph[nb(s, gg, -1)])
                   for gg in range(3))
        phi_new[s] = ph[s] - flux + p["M"] * lap_s(mu, s)
    return g_new, q5_new, phi_new
