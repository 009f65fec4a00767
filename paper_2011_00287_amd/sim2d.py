"""Python handle on one 2D active-nematic context of the HIP library
(include/lb_nematic2d.h).  Argument marshalling only: every step runs in the
library's kernels."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import Lb2dParams, Lb2dTotals, check2, lib

_KEYS = ("tau", "rho0", "A0", "chi", "K", "Gamma", "xi", "zeta")


def make_params2d(p: dict, shape, precision: str = "fp64") -> Lb2dParams:
    """Lb2dParams from a parameter dict and a field shape (ny, nx)."""
    ny, nx = shape
    lp = Lb2dParams()
    lp.nx, lp.ny = int(nx), int(ny)
    lp.prec = _lib.PRECISIONS[precision]
    for k in _KEYS:
        setattr(lp, k, float(p[k]))
    bf = p.get("body_force", (0.0, 0.0))
    lp.body_force[0], lp.body_force[1] = float(bf[0]), float(bf[1])
    return lp


def _dptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Nematic2D:
    """One periodic ny x nx box.  q2: [2, ny, nx] (Q_xx, Q_xy); u0: [2, ny, nx] or None.
    precision: 'fp64' or 'fp32'.  stream: a torch.cuda.Stream, a raw hipStream_t as
    int, or None for the default stream."""

    def __init__(self, params: dict, q2, u0=None, precision: str = "fp64", stream=None):
        q2 = _c64(q2)
        if q2.ndim != 3 or q2.shape[0] != 2:
            raise ValueError(f"q2 shape {q2.shape}, expected (2, ny, nx)")
        self.shape = q2.shape[1:]
        u0 = None if u0 is None else _c64(u0)
        if u0 is not None and u0.shape != q2.shape:
            raise ValueError("u0 shape mismatch")
        self.params = dict(params)
        self.precision = precision
        self._lp = make_params2d(params, self.shape, precision)
        s = None if stream is None else ctypes.c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)
        h = ctypes.c_void_p()
        check2(lib().lb2d_init(ctypes.byref(self._lp), _dptr(q2), _dptr(u0), s, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().lb2d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def n_sites(self) -> int:
        return int(self.shape[0] * self.shape[1])

    def step(self, n: int = 1):
        check2(lib().lb2d_step(self._h, int(n)))

    def sync(self):
        check2(lib().lb2d_sync(self._h))

    def moments(self):
        """(rho, u, q2) at the current time."""
        rho = np.empty(self.shape)
        u = np.empty((2,) + self.shape)
        q2 = np.empty((2,) + self.shape)
        check2(lib().lb2d_moments(self._h, _dptr(rho), _dptr(u), _dptr(q2)))
        return rho, u, q2

    def q(self):
        q2 = np.empty((2,) + self.shape)
        check2(lib().lb2d_moments(self._h, None, None, _dptr(q2)))
        return q2

    def populations(self):
        g = np.empty((9,) + self.shape)
        check2(lib().lb2d_populations(self._h, _dptr(g)))
        return g

    def set_fields(self, g=None, q2=None):
        g = None if g is None else _c64(g)
        q2 = None if q2 is None else _c64(q2)
        if g is not None and g.shape != (9,) + self.shape:
            raise ValueError(f"g shape {g.shape}")
        if q2 is not None and q2.shape != (2,) + self.shape:
            raise ValueError(f"q2 shape {q2.shape}")
        check2(lib().lb2d_set_fields(self._h, _dptr(g), _dptr(q2)))

    def totals(self) -> dict:
        t = Lb2dTotals()
        check2(lib().lb2d_free_energy(self._h, ctypes.byref(t)))
        return dict(mass=t.mass, momentum=list(t.momentum), free_energy=t.free_energy,
                    kinetic_energy=t.kinetic_energy, step=t.step)

    def profile(self, nsteps: int):
        """{kernel name: average ms per launch} over nsteps steps (state advances)."""
        ms = (ctypes.c_double * 4)()
        cnt = ctypes.c_int32()
        check2(lib().lb2d_profile_step(self._h, int(nsteps), ms, ctypes.byref(cnt)))
        return {lib().lb2d_kernel_name(self._h, i).decode(): ms[i] for i in range(cnt.value)}
