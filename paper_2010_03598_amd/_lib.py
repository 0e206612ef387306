"""ctypes view of libkgrape.so (the C ABI declared in include/kgrape.h).

Loading fails loudly: there is no fallback implementation of any entry point.
"""

from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; KG_LIBRARY names another build of the same sources (the
# host-sanitizer build that the CPU tests load in a child process)
LIB_PATH = os.environ.get("KG_LIBRARY") or os.path.join(_PKG, "libkgrape.so")

KG_OK = 0
KG_EINVAL = -1
KG_EWORKSPACE = -3
KG_EDEVICE = -4

KG_C128 = 0
KG_C64 = 1

KG_HC_SX = 0
KG_HC_SZ = 1

KG_MAX_M = 64
KG_MIN_L = 2
KG_MAX_L = 30
KG_PE_MAX_L = 32

KG_GRAD_ZEROTH = 0
KG_GRAD_CENTRED = 1
KG_GRAD_FIRST_ORDER = 2
KG_GRAD_QUADRATURE = 3


class KgXxz(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("hc_kind", ctypes.c_int32), ("J", ctypes.c_double),
                ("Delta", ctypes.c_double), ("hc_sites", ctypes.c_uint64)]


class KgKrylov(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("reorth", ctypes.c_int32),
                ("breakdown_tol", ctypes.c_double)]


class KgChain(ctypes.Structure):
    _fields_ = [("h", KgXxz), ("N", ctypes.c_int32), ("m", ctypes.c_int32),
                ("reorth", ctypes.c_int32), ("team_first", ctypes.c_int32),
                ("team_size", ctypes.c_int32), ("pad_", ctypes.c_int32), ("dt", ctypes.c_double),
                ("breakdown_tol", ctypes.c_double), ("off_u", ctypes.c_int64),
                ("off_vec", ctypes.c_int64), ("off_states", ctypes.c_int64),
                ("off_ws", ctypes.c_int64)]


class KgBatchPlan(ctypes.Structure):
    _fields_ = [("u_len", ctypes.c_int64), ("vec_len", ctypes.c_int64),
                ("states_len", ctypes.c_int64), ("ws_bytes", ctypes.c_uint64),
                ("blocks_used", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class KgPe(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("K", ctypes.c_int32), ("dim", ctypes.c_int64),
                ("tables", ctypes.c_void_p)]


class KgError(RuntimeError):
    def __init__(self, fn: str, status: int, message: str):
        super().__init__(f"{fn} failed with status {status}: {message}")
        self.status = status


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_U32 = ctypes.c_uint32
_D = ctypes.c_double
_SZ = ctypes.c_size_t
_PX = ctypes.POINTER(KgXxz)
_PK = ctypes.POINTER(KgKrylov)
_PPE = ctypes.POINTER(KgPe)

# name -> (restype, argtypes); mirrors include/kgrape.h
SIGNATURES = {
    "kg_last_error": (ctypes.c_char_p, []),
    "kg_version": (_I32, []),
    "kg_workspace_bytes": (_SZ, [_PX, _PK, _I32]),
    "kg_extended_workspace_bytes": (_SZ, [_PX, _PK, _I32]),
    "kg_states_bytes": (_SZ, [_PX, _I32, _I32, _I32]),
    "xxz_apply": (_I32, [_PX, _D, _I32, _P, _P, _P]),
    "krylov_expv": (_I32, [_PX, _D, _D, _PK, _I32, _P, _P, _P, _SZ, _P, _P]),
    "grape_forward": (_I32, [_PX, _P, _I32, _D, _PK, _I32, _P, _P, _P, _P, _P, _I32, _P, _SZ, _P]),
    "grape_gradient": (_I32, [_PX, _P, _I32, _D, _PK, _I32, _P, _P, _P, _P, _P, _P, _I32, _I32,
                              _P, _SZ, _P]),
    "grape_gradient_centred": (_I32, [_PX, _P, _I32, _D, _PK, _I32, _P, _P, _P, _P, _P, _P, _I32,
                                      _I32, _P, _SZ, _P]),
    "grape_gradient_quadrature": (_I32, [_PX, _P, _I32, _D, _PK, _I32, _P, _P, _P, _P, _P, _P,
                                         _I32, _I32, _I32, _P, _SZ, _P]),
    "grape_gradient_first_order": (_I32, [_PX, _P, _I32, _D, _PK, _I32, _P, _P, _P, _P, _P, _P,
                                          _I32, _I32, _P, _SZ, _P]),
    "grape_ascent_update": (_I32, [_P, _P, _I32, _D, _P]),
    "kg_debug_index_map": (_I32, [_I32, _U32, _U32, _P, _P, _P]),
    "kg_profile_begin": (_I32, [_I32, _I32]),
    "kg_batched_chain_ws_bytes": (_SZ, [_I32, _I32, _I32]),
    "grape_gradient_batched": (_I32, [_P, _P, _I32, _I32, _P, ctypes.c_int64, _P, _P, ctypes.c_int64,
                                      _P, ctypes.c_int64, _P, _P, _P, _P, _SZ, _P, _P]),
    "kg_batched_plan": (_I32, [_P, _I32, _P, _I32, _I32, _I32, _D, _I32, _I32, _P]),
    "kg_batched_autotune": (_I32, [_P, _P, _I32, _I32, _P, _I32, _I32, _P, ctypes.c_int64, _P, _P,
                                   ctypes.c_int64, _P, ctypes.c_int64, _P, _P, _P, _P, _SZ, _P,
                                   _P, _P, _P]),
    "kg_profile_end": (_I32, [_P, _P, _P]),
    "kg_static_scratch_bytes": (_SZ, []),
    "krylov_expv_static": (_I32, [_PX, _D, _D, _PK, _I32, _P, _P, _P, _P]),
    "kg_columns_states_bytes": (_SZ, [_PX, _I32, _I32, _I32, _I32]),
    "grape_gradient_columns": (_I32, [_PX, _P, _I32, _D, _PK, _I32, _I32, _P, _P, _P, _P, _P, _P,
                                      _P, _I32, _I32, _P, _SZ, _P]),
    "grape_gradient_columns_pe": (_I32, [_PX, _PPE, _P, _I32, _D, _PK, _I32, _I32, _P, _P, _P, _P,
                                         _P, _P, _P, _I32, _I32, _P, _SZ, _P]),
    "kg_pe_dim": (ctypes.c_int64, [_I32, _I32]),
    "kg_pe_tables_bytes": (_SZ, [_I32, _I32]),
    "kg_pe_tables_host": (_I32, [_I32, _I32, _P, _SZ]),
    "kg_pe_build": (_I32, [_I32, _I32, _P, _SZ, _PPE]),
    "kg_pe_workspace_bytes": (_SZ, [_PPE, _PK, _I32, _I32]),
    "kg_pe_states_bytes": (_SZ, [_PPE, _I32, _I32, _I32]),
    "xxz_pe_apply": (_I32, [_PX, _PPE, _D, _I32, _P, _P, _P]),
    "krylov_expv_pe": (_I32, [_PX, _PPE, _D, _D, _PK, _I32, _P, _P, _P, _SZ, _P, _P]),
    "grape_forward_pe": (_I32, [_PX, _PPE, _P, _I32, _D, _PK, _I32, _P, _P, _P, _P, _P, _I32, _P,
                                _SZ, _P]),
    "grape_gradient_pe": (_I32, [_PX, _PPE, _P, _I32, _D, _PK, _I32, _P, _P, _P, _P, _P, _P, _I32,
                                 _I32, _I32, _I32, _P, _SZ, _P]),
}

PROF_CLASSES = ["pass_a", "pass_b", "combine", "bracket", "overlap", "hv"]

_lib = None


def load() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2010_03598_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().kg_last_error().decode()


def check(fn: str, status: int) -> None:
    if status != KG_OK:
        raise KgError(fn, status, last_error())
