"""Python handle on one simulation context of the HIP library.

Argument marshalling only: every step of the method runs in the library's
kernels.  torch is used for the device memory of checkpoints and for the
stream the kernels run on.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _lib
from ._lib import LbParams, LbTotals, check, lib

_PARAM_KEYS = ("tau", "rho0", "a", "phi0", "phi_cr", "k_phi", "M", "A0", "chi0", "chi_s", "K", "q0", "W",
               "Gamma", "xi", "zeta")


def make_params(p: dict, shape, precision: str = "fp64", lattice: str = "d3q19",
                fd_scheme: str = "euler2") -> LbParams:
    """LbParams from a parameter dict and a field shape (nz, ny, nx)."""
    nz, ny, nx = shape
    lp = LbParams()
    lp.nx, lp.ny, lp.nz = int(nx), int(ny), int(nz)
    lp.prec = _lib.PRECISIONS[precision]
    lp.lattice = _lib.LATTICES[lattice]
    lp.fd_scheme = _lib.FD_SCHEMES[fd_scheme]
    for k in _PARAM_KEYS:
        setattr(lp, k, float(p[k]))
    bf = p.get("body_force", (0.0, 0.0, 0.0))
    for a in range(3):
        lp.body_force[a] = float(bf[a])
    return lp


def make_tuning(tuning: Optional[dict]) -> "_lib.LbTuning":
    """lb_tuning from a dict: path ('default', 'one', 'two', 'site' or the lb_path
    value), tile indices (1-based, 0 = default) and slab depths (0 = automatic)."""
    t = _lib.LbTuning()
    for k, v in (tuning or {}).items():
        if k == "path" and isinstance(v, str):
            v = _lib.PATHS[v]
        if k not in dict(_lib.LbTuning._fields_):
            raise KeyError(f"unknown tuning field {k!r}")
        setattr(t, k, int(v))
    return t


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Sim:
    """One periodic box on the GPU.

    phi: [nz, ny, nx]; q5: [5, nz, ny, nx] (xx, xy, xz, yy, yz); u0: [3, nz, ny, nx]
    or None.  precision: 'fp64', 'fp32' or 'fp16s'.  lattice: 'd3q19' (stress as a
    forcing term) or 'd3q15' (symmetric stress in the equilibrium, antisymmetric
    stress as a forcing term; fp64 and fp32).  fd_scheme: 'euler2'
    (explicit Euler, second-order stencils) or 'pc4' (the paper's predictor-corrector
    with upwind advection and fourth-order stencils).  tuning: launch
    configuration (see make_tuning; None = the defaults).  stream: a torch.cuda.Stream,
    a raw hipStream_t as int, or None for the default stream.  The device tensors
    this class allocates (state, adjoint and record buffers) are created and
    zero-filled on torch's current stream, so pass that stream (or None while
    torch uses the default stream) to keep them ordered with the library's work.
    """

    def __init__(self, params: dict, phi, q5, u0=None, precision: str = "fp64", stream=None,
                 lattice: str = "d3q19", fd_scheme: str = "euler2", tuning: Optional[dict] = None):
        phi = _c64(phi)
        q5 = _c64(q5)
        if q5.shape != (5,) + phi.shape:
            raise ValueError(f"q5 shape {q5.shape} does not match phi {phi.shape}")
        u0 = None if u0 is None else _c64(u0)
        if u0 is not None and u0.shape != (3,) + phi.shape:
            raise ValueError("u0 shape mismatch")
        self.shape = phi.shape
        self.precision = precision
        self.lattice = lattice
        self.fd_scheme = fd_scheme
        self.n_populations = _lib.N_POPULATIONS[lattice]
        self.params = dict(params)
        self._lp = make_params(params, phi.shape, precision, lattice, fd_scheme)
        self._stream = stream
        h = ctypes.c_void_p()
        self._tuning = make_tuning(tuning)
        check(lib().lb_init_tuned(ctypes.byref(self._lp), ctypes.byref(self._tuning), _dptr(phi), _dptr(q5),
                                  _dptr(u0), _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    @property
    def n_sites(self) -> int:
        nz, ny, nx = self.shape
        return nx * ny * nz

    def close(self):
        if getattr(self, "_h", None):
            lib().lb_destroy(self._h)
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

    # ------------------------------------------------------------------ stepping
    def step(self, n: int = 1):
        check(lib().lb_step(self._h, int(n)))

    def sync(self):
        check(lib().lb_sync(self._h))

    def run_logged(self, nsteps: int, every: int, path: str):
        """Advance nsteps steps, appending one JSON line to `path` at the start and
        every `every` steps: step, float64 totals (mass, momentum, sum phi, F_h,
        kinetic energy) and the droplet centre (linear and circular mean).  A
        non-finite total raises (LbError, LB_ENONFINITE) with the last good line
        already written."""
        import json
        if every <= 0:
            raise ValueError("every must be positive")
        with open(path, "a") as fh:
            done = 0
            while True:
                t = self.totals()
                lin, circ, _ = self.centre()
                fh.write(json.dumps({"step": t["step"], "mass": t["mass"], "momentum": t["momentum"],
                                     "phi_total": t["phi_total"], "free_energy": t["free_energy"],
                                     "kinetic_energy": t["kinetic_energy"], "centre_linear": lin.tolist(),
                                     "centre_circular": circ.tolist()}) + "\n")
                fh.flush()
                if done >= nsteps:
                    break
                n = min(every, nsteps - done)
                self.step(n)
                done += n

    def set_params(self, **changes):
        """Change model parameters (not the box, precision, lattice or integrator); kept only if
        the library accepts them."""
        new = dict(self.params, **changes)
        lp = make_params(new, self.shape, self.precision, self.lattice, self.fd_scheme)
        check(lib().lb_set_params(self._h, ctypes.byref(lp)))
        self.params, self._lp = new, lp

    # --------------------------------------------------------------- observation
    def moments(self):
        """(rho, u, phi, q5) at the current time as float64 numpy arrays."""
        rho = np.empty(self.shape)
        u = np.empty((3,) + self.shape)
        phi = np.empty(self.shape)
        q5 = np.empty((5,) + self.shape)
        check(lib().lb_moments(self._h, _dptr(rho), _dptr(u), _dptr(phi), _dptr(q5)))
        return rho, u, phi, q5

    def fields(self):
        """(phi, q5) at the current time."""
        phi = np.empty(self.shape)
        q5 = np.empty((5,) + self.shape)
        check(lib().lb_moments(self._h, None, None, _dptr(phi), _dptr(q5)))
        return phi, q5

    def populations(self) -> np.ndarray:
        g = np.empty((self.n_populations,) + self.shape)
        check(lib().lb_populations(self._h, _dptr(g)))
        return g

    def set_fields(self, g=None, phi=None, q5=None):
        g = None if g is None else _c64(g)
        phi = None if phi is None else _c64(phi)
        q5 = None if q5 is None else _c64(q5)
        for name, a, lead in (("g", g, (self.n_populations,)), ("phi", phi, ()), ("q5", q5, (5,))):
            if a is not None and a.shape != lead + self.shape:
                raise ValueError(f"{name} shape {a.shape}, expected {lead + self.shape}")
        check(lib().lb_set_fields(self._h, _dptr(g), _dptr(phi), _dptr(q5)))

    def totals(self) -> dict:
        t = LbTotals()
        check(lib().lb_free_energy(self._h, ctypes.byref(t)))
        return dict(mass=t.mass, momentum=list(t.momentum), phi_total=t.phi_total, free_energy=t.free_energy,
                    kinetic_energy=t.kinetic_energy, step=t.step)

    def centre(self):
        """(linear centre xyz, circular centre xyz, sum phi)."""
        out = (ctypes.c_double * 6)()
        tot = ctypes.c_double()
        check(lib().lb_centre(self._h, out, ctypes.byref(tot)))
        return np.array(out[:3]), np.array(out[3:]), tot.value

    # ---------------------------------------------------------------- checkpoint
    def state_bytes(self) -> int:
        return int(lib().lb_state_bytes(self._h))

    def get_state(self, buf=None):
        """Copy the state into a torch uint8 device tensor (allocated if None)."""
        import torch
        nb = self.state_bytes()
        if buf is None:
            buf = torch.empty(nb, dtype=torch.uint8, device="cuda")
        check(lib().lb_get_state(self._h, ctypes.c_void_p(buf.data_ptr()), nb))
        return buf

    def set_state(self, buf):
        check(lib().lb_set_state(self._h, ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()))

    # ------------------------------------------------------------------- adjoint
    @property
    def compute_dtype(self):
        import torch
        return torch.float64 if self.precision == "fp64" else torch.float32

    def adjoint_buffer(self):
        """Zeroed device tensor holding (g_bar [Q][N], q_bar [5][N], phi_bar [N]); Q = 19 or 15."""
        import torch
        nb = int(lib().lb_adjoint_bytes(self._h))
        esz = 8 if self.precision == "fp64" else 4
        return torch.zeros(nb // esz, dtype=self.compute_dtype, device="cuda")

    def adjoint_parts(self, adj):
        """Views (g_bar [Q,nz,ny,nx], q_bar [5,...], phi_bar [...]) of an adjoint buffer (Q populations)."""
        n, nq = self.n_sites, self.n_populations
        return (adj[:nq * n].view((nq,) + self.shape), adj[nq * n:(nq + 5) * n].view((5,) + self.shape),
                adj[(nq + 5) * n:].view(self.shape))

    def seed_centre(self, z_ref: float, adj) -> float:
        """adj <- dL/d(state) of L = (z_c - z_ref)^2 at the current state; returns L."""
        loss = ctypes.c_double()
        check(lib().lb_adjoint_seed_centre(self._h, ctypes.c_double(z_ref), ctypes.c_void_p(adj.data_ptr()),
                                           adj.numel() * adj.element_size(), ctypes.byref(loss)))
        return loss.value

    def record_buffer(self):
        """Device tensor for one step record (u [3][N], F [3][N], drho [N]; with the pc4
        integrator also the predictor state X*)."""
        import torch
        nb = int(lib().lb_record_bytes(self._h))
        esz = 8 if self.precision == "fp64" else 4
        return torch.empty(nb // esz, dtype=self.compute_dtype, device="cuda")

    def step_record(self, state_in, state_out, rec_out):
        """state_out <- one step of state_in (None: record only); rec_out <- (u, F, drho) of
        state_in's time."""
        out = None if state_out is None else ctypes.c_void_p(state_out.data_ptr())
        check(lib().lb_step_record(self._h, ctypes.c_void_p(state_in.data_ptr()),
                                   out, ctypes.c_void_p(rec_out.data_ptr()),
                                   state_in.numel() * state_in.element_size(),
                                   rec_out.numel() * rec_out.element_size()))

    def adjoint_step(self, state, adj_in, adj_out, rec=None, zeta_bar: float = 0.0, q0_bar: float = 0.0,
                     fetch: bool = True):
        """adj_out <- adjoint at t from adj_in (adjoint at t+1), given the forward state at t
        (and its step record, or None to recompute).  Returns the updated (zeta_bar, q0_bar).

        fetch=False leaves this step's parameter contributions summed on the
        device (no synchronisation) and returns the inputs unchanged; the next
        call with fetch=True adds every kept contribution."""
        recp = ctypes.c_void_p(rec.data_ptr()) if rec is not None else None
        recb = rec.numel() * rec.element_size() if rec is not None else 0
        zb = ctypes.c_double(zeta_bar)
        qb = ctypes.c_double(q0_bar)
        check(lib().lb_adjoint_step(self._h, ctypes.c_void_p(state.data_ptr()), state.numel() * state.element_size(),
                                    recp, recb, ctypes.c_void_p(adj_in.data_ptr()),
                                    ctypes.c_void_p(adj_out.data_ptr()), adj_in.numel() * adj_in.element_size(),
                                    ctypes.byref(zb) if fetch else None, ctypes.byref(qb) if fetch else None))
        return zb.value, qb.value

    def lean_record_buffer(self):
        """uint8 device tensor for one lean step record (Q, phi of time t; drho, u, F of its step;
        with the pc4 integrator also the predictor state X*)."""
        import torch
        return torch.empty(int(lib().lb_lean_record_bytes(self._h)), dtype=torch.uint8, device="cuda")

    def step_record_lean(self, rec):
        """Record the current time into rec (lean format) and advance the state by one step."""
        check(lib().lb_step_record_lean(self._h, ctypes.c_void_p(rec.data_ptr()), rec.numel() * rec.element_size()))

    def adjoint_step_lean(self, rec, adj_in, adj_out, zeta_bar: float = 0.0, q0_bar: float = 0.0,
                          fetch: bool = True):
        """adj_out <- adjoint at t from adj_in (adjoint at t+1), given the lean record of the
        step from t; parameter sums as in adjoint_step."""
        zb = ctypes.c_double(zeta_bar)
        qb = ctypes.c_double(q0_bar)
        check(lib().lb_adjoint_step_lean(self._h, ctypes.c_void_p(rec.data_ptr()), rec.numel() * rec.element_size(),
                                         ctypes.c_void_p(adj_in.data_ptr()), ctypes.c_void_p(adj_out.data_ptr()),
                                         adj_in.numel() * adj_in.element_size(),
                                         ctypes.byref(zb) if fetch else None, ctypes.byref(qb) if fetch else None))
        return zb.value, qb.value

    # ----------------------------------------------------------------- profiling
    def profile(self, nsteps: int):
        """{kernel name: average ms per launch} over nsteps steps (state advances)."""
        ms = (ctypes.c_double * _lib.LB_MAX_KERNELS)()
        cnt = ctypes.c_int32()
        check(lib().lb_profile_step(self._h, int(nsteps), ms, ctypes.byref(cnt)))
        return {lib().lb_kernel_name(self._h, i).decode(): ms[i] for i in range(cnt.value)}
