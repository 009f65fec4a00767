"""Shared test helpers: error norms and oracle wrappers on numpy arrays."""
import numpy as np
import torch

from oracle import core

DT = torch.float64


def t64(a):
    return torch.tensor(np.asarray(a), dtype=DT)


def rel_err(x, ref):
    """(l2 relative, max-abs / max|ref|); both 0 when ref and x are exactly zero."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = x - ref
    n2 = np.linalg.norm(ref)
    m = np.abs(ref).max()
    l2 = np.linalg.norm(d) / n2 if n2 > 0 else np.linalg.norm(d)
    mx = np.abs(d).max() / m if m > 0 else np.abs(d).max()
    return float(l2), float(mx)


def oracle_run(p, g, q5, phi, nsteps):
    """Run the oracle; returns numpy (g, q5, phi)."""
    g, q5, phi = core.run(t64(g), t64(q5), t64(phi), p, nsteps)
    return g.numpy(), q5.numpy(), phi.numpy()


def oracle_observe(p, g, q5, phi):
    rho, u = core.observe(t64(g), t64(q5), t64(phi), p)
    return rho.numpy(), u.numpy()


def field_errors(sim_out, orc_out, rho0=1.0):
    """Per-field errors (R22 norm) between (rho, u, phi, q5) tuples."""
    names = ("rho-rho0", "u", "phi", "Q")
    res = {}
    for n, a, b in zip(names, sim_out, orc_out):
        if n == "rho-rho0":
            a, b = np.asarray(a) - rho0, np.asarray(b) - rho0
        res[n] = rel_err(a, b)
    return res
