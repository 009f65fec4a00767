"""ctypes declarations of the C ABI in include/lb_chiral.h and include/lb_nematic2d.h
(marshalling only)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "liblbchiral.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_ENONFINITE, LB_ESTATE = 0, -1, -2, -3, -4, -5
LB_FP64, LB_FP32, LB_FP16S = 0, 1, 2
PRECISIONS = {"fp64": LB_FP64, "fp32": LB_FP32, "fp16s": LB_FP16S}
LB_D3Q19, LB_D3Q15 = 0, 1
LATTICES = {"d3q19": LB_D3Q19, "d3q15": LB_D3Q15}
N_POPULATIONS = {"d3q19": 19, "d3q15": 15}
LB_FD_EULER2, LB_FD_PC4 = 0, 1
FD_SCHEMES = {"euler2": LB_FD_EULER2, "pc4": LB_FD_PC4}
LB_MAX_KERNELS = 8


class LbParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("prec", ctypes.c_int32),
        ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
        ("a", ctypes.c_double), ("phi0", ctypes.c_double), ("phi_cr", ctypes.c_double),
        ("k_phi", ctypes.c_double), ("M", ctypes.c_double),
        ("A0", ctypes.c_double), ("chi0", ctypes.c_double), ("chi_s", ctypes.c_double),
        ("K", ctypes.c_double), ("q0", ctypes.c_double), ("W", ctypes.c_double),
        ("Gamma", ctypes.c_double), ("xi", ctypes.c_double), ("zeta", ctypes.c_double),
        ("body_force", ctypes.c_double * 3), ("lattice", ctypes.c_int32),
        ("fd_scheme", ctypes.c_int32),
    ]


LB_PATH_DEFAULT, LB_PATH_ONE_LAUNCH, LB_PATH_TWO_LAUNCHES, LB_PATH_SITE = 0, 1, 2, 3
PATHS = {"default": LB_PATH_DEFAULT, "one": LB_PATH_ONE_LAUNCH, "two": LB_PATH_TWO_LAUNCHES, "site": LB_PATH_SITE}


class LbTuning(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in (
        "path", "lb_tile", "order_tile", "pc_tile", "pcmu_tile", "adj_tile", "adj_order_tile", "step_tile", "tz_step", "tz_lb", "tz_order", "tz_pc",
        "tz_pcmu", "tz_adj", "tz_adj_order", "tz_pc_adj", "pc_adj")]


class LbTotals(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3), ("phi_total", ctypes.c_double),
        ("free_energy", ctypes.c_double), ("kinetic_energy", ctypes.c_double), ("step", ctypes.c_int64),
    ]


class LbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lb status {status}: {msg}")
        self.status = status


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)

SIGNATURES = {
    "lb_init": (ctypes.c_int, [ctypes.POINTER(LbParams), _D, _D, _D, _P, ctypes.POINTER(_P)]),
    "lb_init_tuned": (ctypes.c_int, [ctypes.POINTER(LbParams), ctypes.POINTER(LbTuning), _D, _D, _D, _P,
                                     ctypes.POINTER(_P)]),
    "lb_step": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lb_set_params": (ctypes.c_int, [_P, ctypes.POINTER(LbParams)]),
    "lb_moments": (ctypes.c_int, [_P, _D, _D, _D, _D]),
    "lb_populations": (ctypes.c_int, [_P, _D]),
    "lb_set_fields": (ctypes.c_int, [_P, _D, _D, _D]),
    "lb_free_energy": (ctypes.c_int, [_P, ctypes.POINTER(LbTotals)]),
    "lb_centre": (ctypes.c_int, [_P, _D, _D]),
    "lb_centre_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P,
                                         _P]),
    "lb_state_bytes": (ctypes.c_size_t, [_P]),
    "lb_get_state": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "lb_set_state": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "lb_adjoint_bytes": (ctypes.c_size_t, [_P]),
    "lb_record_bytes": (ctypes.c_size_t, [_P]),
    "lb_step_record": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_size_t, ctypes.c_size_t]),
    "lb_adjoint_step": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P, ctypes.c_size_t, _P, _P, ctypes.c_size_t,
                                        _D, _D]),
    "lb_lean_record_bytes": (ctypes.c_size_t, [_P]),
    "lb_step_record_lean": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "lb_adjoint_step_lean": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P, _P, ctypes.c_size_t, _D, _D]),
    "lb_adjoint_seed_centre": (ctypes.c_int, [_P, ctypes.c_double, _P, ctypes.c_size_t, _D]),
    "lb_profile_step": (ctypes.c_int, [_P, ctypes.c_int32, _D, ctypes.POINTER(ctypes.c_int32)]),
    "lb_kernel_name": (ctypes.c_char_p, [_P, ctypes.c_int32]),
    "lb_sync": (ctypes.c_int, [_P]),
    "lb_destroy": (None, [_P]),
    "lb_last_error": (ctypes.c_char_p, []),
}


class Lb2dParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("prec", ctypes.c_int32),
        ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
        ("A0", ctypes.c_double), ("chi", ctypes.c_double), ("K", ctypes.c_double),
        ("Gamma", ctypes.c_double), ("xi", ctypes.c_double), ("zeta", ctypes.c_double),
        ("body_force", ctypes.c_double * 2),
    ]


class Lb2dTotals(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("momentum", ctypes.c_double * 2), ("free_energy", ctypes.c_double),
        ("kinetic_energy", ctypes.c_double), ("step", ctypes.c_int64),
    ]


SIGNATURES_2D = {
    "lb2d_init": (ctypes.c_int, [ctypes.POINTER(Lb2dParams), _D, _D, _P, ctypes.POINTER(_P)]),
    "lb2d_step": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lb2d_sync": (ctypes.c_int, [_P]),
    "lb2d_moments": (ctypes.c_int, [_P, _D, _D, _D]),
    "lb2d_populations": (ctypes.c_int, [_P, _D]),
    "lb2d_set_fields": (ctypes.c_int, [_P, _D, _D]),
    "lb2d_free_energy": (ctypes.c_int, [_P, ctypes.POINTER(Lb2dTotals)]),
    "lb2d_profile_step": (ctypes.c_int, [_P, ctypes.c_int32, _D, ctypes.POINTER(ctypes.c_int32)]),
    "lb2d_kernel_name": (ctypes.c_char_p, [_P, ctypes.c_int32]),
    "lb2d_destroy": (None, [_P]),
    "lb2d_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load the built HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} missing "
                               "(run python -m paper_2011_00287_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in list(SIGNATURES.items()) + list(SIGNATURES_2D.items()):
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != LB_OK:
        msg = lib().lb_last_error()
        raise LbError(status, msg.decode() if msg else "")


def check2(status: int) -> None:
    if status != LB_OK:
        msg = lib().lb2d_last_error()
        raise LbError(status, msg.decode() if msg else "")
