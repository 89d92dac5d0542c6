"""ctypes binding of ``libdgsrhd.so`` (the C ABI in include/dgsrhd.h).

Argument marshalling only: every step of the DG path runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgsrhd.so")

DG_OK, DG_EINVAL, DG_ENOMEM, DG_EHIP, DG_ECON2PRIM, DG_EAVERAGE, DG_ESTATE = 0, -1, -2, -3, -4, -5, -6
ERROR_NAMES = {DG_EINVAL: "DG_EINVAL", DG_ENOMEM: "DG_ENOMEM", DG_EHIP: "DG_EHIP",
               DG_ECON2PRIM: "DG_ECON2PRIM", DG_EAVERAGE: "DG_EAVERAGE", DG_ESTATE: "DG_ESTATE"}
CONSERVED, PRIMITIVE = 0, 1


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("p", ctypes.c_int),
        ("n_elem", ctypes.c_int * 3),
        ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
        ("bc", ctypes.c_int * 3),
        ("eos", ctypes.c_int),
        ("gamma_ad", ctypes.c_double), ("c_light", ctypes.c_double),
        ("c2p", ctypes.c_int), ("precision", ctypes.c_int),
        ("phys", ctypes.c_int), ("phys_eps", ctypes.c_double),
        ("sync_mode", ctypes.c_int),
        ("flux", ctypes.c_int),
        ("bc_hi", ctypes.c_int * 3),
        ("bc_state", ctypes.c_double * 30),
        ("c2p_iters", ctypes.c_int),
        ("limiter", ctypes.c_int),
    ]


class Diag(ctypes.Structure):
    _fields_ = [(n, ctypes.c_longlong) for n in (
        "c2p_fail", "c2p_noconv", "trace_fallback", "flagged", "smoothed", "bad_average",
        "bad_input", "first_bad_elem", "limited")]


_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int

SIGNATURES = {
    "dg_init_mesh": (_I, [ctypes.POINTER(MeshDesc), _P, ctypes.POINTER(_P)]),
    "dg_set_stream": (_I, [_P, _P]),
    "dg_state_size": (ctypes.c_size_t, [_P]),
    "dg_set_state": (_I, [_P, _I, _P, _P]),
    "dg_con2prim": (_I, [_P, _P, _P]),
    "dg_rhs": (_I, [_P, _P, _P]),
    "dg_enforce_physical": (_I, [_P, _P]),
    "dg_ssprk3_step": (_I, [_P, _P, _D]),
    "dg_ssprk3_run": (_I, [_P, _P, _D, _I]),
    "dg_ssprk_step": (_I, [_P, _P, _D, _I]),
    "dg_ssprk_run": (_I, [_P, _P, _D, _I, _I]),
    "dg_rhs_vjp": (_I, [_P, _P, _P, _P]),
    "dg_ssprk3_step_vjp": (_I, [_P, _P, _D, _P, _P]),
    "dg_tape_size": (ctypes.c_size_t, [_P]),
    "dg_ssprk3_step_tape": (_I, [_P, _P, _D, _P]),
    "dg_ssprk3_step_vjp_tape": (_I, [_P, _P, _D, _P, _P]),
    "dg_ssprk3_run_tape": (_I, [_P, _P, _D, _I, _P]),
    "dg_ssprk3_run_vjp_tape": (_I, [_P, _P, _D, _I, _P]),
    "dg_objective_vy2": (_I, [_P, _P, ctypes.POINTER(_D), _P]),
    "dg_set_state_vjp": (_I, [_P, _P, _P, _P]),
    "dg_get_diagnostics": (_I, [_P, ctypes.POINTER(Diag)]),
    "dg_reset_diagnostics": (_I, [_P]),
    "dg_last_error": (ctypes.c_char_p, [_P]),
    "dg_destroy": (None, [_P]),
    "dg_rhs_noalloc": (_I, [ctypes.POINTER(MeshDesc), _P, _P, _P, ctypes.POINTER(Diag)]),
}

# primitive staging the allocation-free right-hand side holds (DG_RHS_NOALLOC_MAX_STATE)
RHS_NOALLOC_MAX_STATE = 8380416

_lib = None


def load() -> ctypes.CDLL:
    """Load the built HIP library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950) first")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class DGError(RuntimeError):
    def __init__(self, code: int, where: str, message: str):
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)} ({message})")
        self.code = code
