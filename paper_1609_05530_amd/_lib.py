"""ctypes binding of libcpc.so (include/cpc.h). Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpc.so")


class CpcError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"libcpc error {code}: {message}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [
        ("prec", ctypes.c_int32),
        ("ties", ctypes.c_int32),
        ("var", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("n_min", ctypes.c_int64),
        ("schedule", ctypes.c_int32),
        ("flags", ctypes.c_int32),
    ]


# Every symbol include/cpc.h declares, with its ctypes signature.
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
SIGNATURES = {
    "cpc_create": (_I32, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "cpc_destroy": (_I32, [_P]),
    "cpc_default_options": (None, [ctypes.POINTER(Options)]),
    "cpc_workspace_bytes": (_SZ, [_I64, _I64, _I64, _I32, ctypes.POINTER(Options)]),
    "cpc_workspace_bytes_for": (_SZ, [_P, _I64, _I64, _I32, ctypes.POINTER(Options)]),
    "cpc_fit": (_I32, [_P, _P, _P, _I32, _I64, _P, _I64, _I32, ctypes.POINTER(Options), _P, _SZ, _P, _P, _P]),
    "cpc_fit_batched": (_I32, [_P, _P, _P, _I32, _I64, _P, _I64, _P, _I64, _P, ctypes.POINTER(Options), _P, _SZ,
                               _P, _P, _P]),
    "cpc_fit_batched_noalloc": (_I32, [_P, _P, _P, _I32, _I64, _P, _I64, _P, _I64, _P, ctypes.POINTER(Options), _P,
                                       _P, _P]),
    "cpc_rank": (_I32, [_P, _P, _P, _I32, _I64, _P, _I64, ctypes.POINTER(Options), _P, _SZ, _P, _P, _P]),
    "cpc_eval": (_I32, [_P, _P, _P, _I64, _P, _I64, _I32, _P, ctypes.POINTER(Options), _P, _SZ, _P, _P]),
    "cpc_variance": (_I32, [_P, _P, _P, _I64, _P, _I64, _I32, _P, ctypes.POINTER(Options), _P, _SZ, _P, _P]),
    "cpc_sample": (_I32, [_P, _I32, ctypes.c_double, ctypes.c_uint64, _I64, _I64, _I32, _P, _P, _P]),
    "cpc_density_distance": (_I32, [_P, _I32, _I64, _P, _P, ctypes.c_double, _I32, _P, _SZ, _P, _P]),
    "cpc_replicate_summary": (_I32, [_P, _I64, _P, _P, _P, _P]),
    "cpc_partition_workspace_bytes": (_SZ, [_P, _I64, _I32, _I32]),
    "cpc_partition": (_I32, [_P, _P, _P, _I32, _I64, _P, _I64, _I64, _I32, _P, _SZ, _P, _P, _P, _P]),
    "cpc_spearman_workspace_bytes": (_SZ, [_I64, _I64, _I64]),
    "cpc_spearman_fit": (_I32, [_P, _P, _P, _I64, _P, _I64, _P, _I64, _P, ctypes.POINTER(Options), _P, _SZ, _P, _P,
                                _P]),
    "cpc_kendall_workspace_bytes": (_SZ, [_I64, _I64, _I64]),
    "cpc_kendall_fit": (_I32, [_P, _P, _P, _I64, _P, _I64, _P, _I64, _P, ctypes.POINTER(Options), _P, _SZ, _P, _P,
                               _P]),
    "cpc_gaussk_workspace_bytes": (_SZ, [_I64, _I32, _I64, _I64]),
    "cpc_gaussk_fit": (_I32, [_P, _P, _I64, _I32, _P, _I64, _P, _I64, ctypes.POINTER(Options), _P, _SZ, _P, _P, _P]),
    "cpc_phase_times": (_I32, [_P, ctypes.POINTER(ctypes.c_float)]),
    "cpc_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "cpc_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libcpc.so. Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_1609_05530_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code: int) -> None:
    if code != 0:
        L = lib()
        raise CpcError(code, f"{L.cpc_strerror(code).decode()}: {L.cpc_last_error().decode()}")
