"""ctypes binding of liblpdec.so: argument marshalling only (every step runs in the HIP
library). The names follow include/lpdec.h."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblpdec.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, EBUSY, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
FLAG_IPM_CAP, FLAG_NONFINITE, FLAG_MALP_CAP, FLAG_INCONSISTENT, FLAG_COST_DECREASE, FLAG_ALP_CAPACITY, \
    FLAG_CUT_CYCLE = -1, -2, -3, -4, -5, -6, -7

OPT = {name: k for k, name in enumerate([
    "MALP_MODE", "PRECISION", "TAU_VIOL", "TAU_ACT", "TAU_INT", "IPM_EPS", "SIGMA", "ETA",
    "PCG_TOL", "PCG_MAXIT", "REF_TOL", "REF_MAX", "IPM_MAX", "MALP_MAX", "BLOCK", "PRECOND", "XI_TOL", "IPM_STALL", "DIRECT_FALLBACK", "MTS_REUSE", "WARM_START", "SERVER_STREAMS", "IPM_WARM", "SERVER_MODE", "DISPATCH_ORDER", "TAU_COST"])}


class Stats(C.Structure):
    _fields_ = [("malp_iters", C.c_int32), ("ipm_iters", C.c_int32), ("pcg_iters", C.c_int32),
                ("p_max", C.c_int32), ("ref_rounds", C.c_int32), ("mts_rounds", C.c_int32),
                ("max_levels", C.c_int32), ("status", C.c_int32), ("escalations", C.c_int32),
                ("direct_solves", C.c_int32), ("pcg_rows", C.c_int64),
                ("ipm_cols", C.c_int64), ("ticks_mts", C.c_int64), ("ticks_solve", C.c_int64),
                ("ticks_total", C.c_int64), ("ticks_pcg", C.c_int64),
                ("ticks_dense", C.c_int64), ("dense_cube", C.c_int64)]


STATS_FIELDS = [f[0] for f in Stats._fields_]

_P = C.c_void_p
_I = C.c_int32
_D = C.c_double

# name -> (restype, argtypes)
_SIGS = {
    "lpdec_ctx_create": (_I, [C.c_int, C.POINTER(_P)]),
    "lpdec_ctx_destroy": (_I, [_P]),
    "lpdec_last_error": (C.c_char_p, [_P]),
    "lpdec_set_option": (_I, [_P, _I, _D]),
    "lpdec_get_option": (_I, [_P, _I, C.POINTER(_D)]),
    "lpdec_code_create": (_I, [_P, _I, _I, _P, _P, C.POINTER(_P)]),
    "lpdec_code_destroy": (_I, [_P]),
    "lpdec_decode": (_I, [_P, _P, _P, _P, C.POINTER(_I), C.POINTER(_D), C.POINTER(Stats), _P]),
    "lpdec_decode_batch": (_I, [_P, _P, _I, _P, _I, _P, _P, _P, _P, _P, _P]),
    "lpdec_alp_decode_batch": (_I, [_P, _P, _I, _P, _P, _P, _P, _P, _P]),
    "lpdec_decode_batch_noalloc": (_I, [_P, _P, _I, _P, _I, _P, _P, _P, _P, _P, _P]),
    "lpdec_decode_batch_trace": (_I, [_P, _P, _I, _P, _I, _P, _P, _P, _P, _P, _P, _I]),
    "lpdec_cut_search_batch": (_I, [_P, _P, _I, _P, _P, _P, _P]),
    "lpdec_mts_batch": (_I, [_P, _P, _I, _P, _P, _P, _P, _P, _P]),
    "lpdec_normal_matvec_batch": (_I, [_P, _P, _I, _P, _P, _P, _P, _P, _I]),
    "lpdec_newton_solve_batch": (_I, [_P, _P, _I, _P, _P, _P, _P, _P, _P, _P, _I]),
    "lpdec_ipm_batch": (_I, [_P, _P, _I, _P, _P, _P, _P, _P, _P, _P, _I]),
    "lpdec_server_create": (_I, [_P, C.c_size_t, _I, C.POINTER(_P)]),
    "lpdec_server_submit": (_I, [_P, _P, _P, C.POINTER(C.c_uint64)]),
    "lpdec_server_poll": (_I, [_P, C.c_uint64, _P, C.POINTER(_I), C.POINTER(_D), C.POINTER(_D)]),
    "lpdec_server_drain": (_I, [_P]),
    "lpdec_server_destroy": (_I, [_P]),
}

EXPORTED = sorted(_SIGS)

_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Loads the HIP library. Raises if it has not been built: there is no fallback.

    torch is imported first so that its HIP runtime (soname libamdhip64.so.7) is the one in
    the process: the library then binds to it instead of loading a second runtime, and device
    pointers and streams from torch are valid in the library."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with `python -m paper_0902_0657_amd.build` "
                              "(the decoder has no CPU fallback)")
        lib = C.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
