"""ctypes binding of librbicg.so: the C ABI declared in include/rbicg.h and
include/rbicg_hostla.h, with the same names.  Argument marshalling only; every
step of the solver runs in the library.  Loading fails loudly if the library
has not been built (python -m paper_1010_0762_amd.build)."""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbicg.so")

RBICG_OK = 0
RBICG_NOT_CONVERGED = 1
RBICG_EINVAL = -1
RBICG_ENOMEM = -2
RBICG_BREAKDOWN = -3
RBICG_EHIP = -4

RBICG_F64 = 0
RBICG_C128 = 1
RBICG_F32_IN_F64_OUT = 2


class rbicg_csr(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("nnz", ct.c_int64), ("rowptr", ct.c_void_p),
                ("colind", ct.c_void_p), ("values", ct.c_void_p),
                ("values_complex", ct.c_int32), ("on_device", ct.c_int32)]


class rbicg_opts(ct.Structure):
    _fields_ = [("k", ct.c_int32), ("s", ct.c_int32), ("maxit", ct.c_int32),
                ("max_restarts", ct.c_int32), ("update", ct.c_int32),
                ("svd_tol", ct.c_double), ("seed", ct.c_uint64), ("prec", ct.c_int),
                ("inner_tol", ct.c_double), ("max_outer", ct.c_int32),
                ("stream", ct.c_void_p), ("chunk", ct.c_int32), ("profile", ct.c_int32),
                ("stall_window", ct.c_int32), ("pencil_setup", ct.c_int32),
                ("blocks", ct.c_int32)]


class rbicg_stats(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("iters", ct.c_int32), ("restarts", ct.c_int32),
                ("outer_steps", ct.c_int32), ("cycles", ct.c_int32), ("k_used", ct.c_int32),
                ("reseeds", ct.c_int32), ("relres", ct.c_double), ("relres_dual", ct.c_double),
                ("time_ms", ct.c_double), ("alg_bytes", ct.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = ct.c_void_p
_I = ct.c_int32
_D = ct.c_double
_DP = ct.POINTER(ct.c_double)

# name -> (restype, argtypes)
SIGNATURES = {
    "rbicg_default_opts": (None, [ct.POINTER(rbicg_opts)]),
    "rbicg_create": (ct.c_int, [ct.POINTER(rbicg_csr), ct.POINTER(rbicg_csr),
                                ct.POINTER(rbicg_opts), ct.POINTER(_P)]),
    "rbicg_solve_dual": (ct.c_int, [_P, _P, _P, _P, _P, _D, ct.POINTER(rbicg_stats)]),
    "rbicg_solve_sequence": (ct.c_int, [_P, _I, ct.POINTER(_P), ct.POINTER(_P), ct.POINTER(_P),
                                        ct.POINTER(_P), ct.POINTER(_P), _I, _D,
                                        ct.POINTER(rbicg_stats)]),
    "rbicg_update_recycle": (ct.c_int, [_P, ct.POINTER(rbicg_csr), ct.POINTER(rbicg_csr)]),
    "rbicg_bilinear": (ct.c_int, [_P, _P, _P, _D, _P, _DP, ct.POINTER(rbicg_stats)]),
    "rbicg_destroy": (ct.c_int, [_P]),
    "rbicg_last_error": (ct.c_char_p, []),
    "rbicg_set_recycle": (ct.c_int, [_P, _P, _P, _I]),
    "rbicg_get_recycle": (ct.c_int, [_P, _P, _P, _P, _P, _I, _I, ct.POINTER(_I)]),
    "rbicg_get_log": (ct.c_int, [_P, _DP, _I, ct.POINTER(_I)]),
    "rbicg_solve_shifted": (ct.c_int, [_P, _I, _DP, _P, _P, _P, _P, _D, _I,
                                       ct.POINTER(rbicg_stats)]),
    "rbicg_matrix_create": (ct.c_int, [ct.POINTER(rbicg_csr), ct.POINTER(rbicg_csr),
                                       ct.POINTER(_P)]),
    "rbicg_matrix_destroy": (ct.c_int, [_P]),
    "rbicg_matrix_info": (ct.c_int, [_P, ct.POINTER(ct.c_int64)]),
    "rbicg_matrix_pencil": (ct.c_int, [_P, _P, _DP, _DP, _P, ct.POINTER(_P)]),
    "rbicg_rbilu_create": (ct.c_int, [ct.POINTER(rbicg_csr), ct.POINTER(_P), ct.POINTER(_P),
                                      ct.POINTER(ct.c_int32)]),
    "rbicg_rbilu_rhs": (ct.c_int, [_P, _P, _P, _P, _P, _P]),
    "rbicg_rbilu_refresh": (ct.c_int, [_P, ct.POINTER(rbicg_csr), _P]),
    "rbicg_rbilu_refresh_values": (ct.c_int, [_P, _P, _P]),
    "rbicg_rbilu_solution": (ct.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "rbicg_rbilu_destroy": (ct.c_int, [_P]),
    "rbicg_create_on": (ct.c_int, [_P, ct.POINTER(rbicg_opts), ct.POINTER(_P)]),
    "rbicg_update_recycle_on": (ct.c_int, [_P, _P]),
    "rbicg_profile": (ct.c_int, [_P, _I, _DP]),
    "rbicg_project": (ct.c_int, [_P, _I, _P, _P, _P, _P, _DP, _DP, _DP, _DP]),
    "rbicg_bilinear_batch": (ct.c_int, [_P, _I, _P, _P, _D, _DP, _DP, ct.POINTER(rbicg_stats)]),
    "rbicg_batch_create": (ct.c_int, [_I, _D, ct.POINTER(_P)]),
    "rbicg_batch_attach": (ct.c_int, [_P, _P]),
    "rbicg_batch_stats": (ct.c_int, [_P, _DP]),
    "rbicg_batch_destroy": (ct.c_int, [_P]),
    "rbicg_batch_use_graphs": (ct.c_int, [_P, _I]),
    "rbicg_solve_dual_noalloc": (ct.c_int, [_P, ct.POINTER(rbicg_opts), _P, _P, _P, _P, _D,
                                            ct.POINTER(rbicg_stats)]),
    "rbicg_ilut_create": (ct.c_int, [ct.POINTER(rbicg_csr), _D, _I, _D, ct.POINTER(_P)]),
    "rbicg_ilu_attach": (ct.c_int, [_P, _P]),
    "rbicg_ilu_rhs": (ct.c_int, [_P, _P, _P, _P, _P, _I, _P]),
    "rbicg_ilu_solution": (ct.c_int, [_P, _P, _P, _P, _P, _I, _P]),
    "rbicg_ilu_info": (ct.c_int, [_P, ct.POINTER(ct.c_int64)]),
    "rbicg_ilu_set_waves": (ct.c_int, [_P, _I]),
    "rbicg_ilu_destroy": (ct.c_int, [_P]),
    "rbicg_host_ilut": (ct.c_int, [_I, _P, _P, _DP, _D, _I, _D, ct.POINTER(ct.c_int64), _P, _P,
                                   _DP, _P, _P, _DP, _P]),
    "rbicg_host_levels": (ct.c_int, [_I, _P, _P, _I, _I, _P, ct.POINTER(ct.c_int64)]),
    "rbicg_host_eig": (ct.c_int, [_I, _DP, _DP, _DP, _DP, _DP]),
    "rbicg_host_select": (ct.c_int, [_I, _DP, _DP, _DP, _I, _I, _DP, _DP]),
    "rbicg_host_eig_select": (ct.c_int, [_I, _DP, _DP, _I, _I, _DP, _DP]),
    "rbicg_host_svd": (ct.c_int, [_I, _I, _DP, _DP, _DP, _DP]),
    "rbicg_host_heig": (ct.c_int, [_I, _DP, _DP, _DP]),
    "rbicg_host_biorth": (ct.c_int, [_I, _DP, _DP, _DP, _D, _DP, _DP]),
}

_lib = None


def load() -> ct.CDLL:
    """Load librbicg.so (once).  Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                           "`python -m paper_1010_0762_amd.build` (hipcc, gfx950)")
    lib = ct.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().rbicg_last_error().decode(errors="replace")


class RBiCGError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where} failed with code {code}: {last_error()}")
        self.code = code


def check(code, where, ok=(RBICG_OK,)):
    if code not in ok:
        raise RBiCGError(code, where)
    return code


def dptr(a) -> ct.POINTER(ct.c_double):
    """ctypes double* of a contiguous numpy array."""
    return a.ctypes.data_as(_DP)
