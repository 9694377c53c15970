"""ctypes view of libisdf.so (the C ABI declared in include/isdf.h).

Loading imports torch first, so that the process maps a single HIP runtime
(torch's), which the library then shares (same soname).  There is no
fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libisdf.so")

# status codes
OK, E_ARG, E_WORKSPACE, E_HIP, E_UNSUPPORTED, E_SCRATCH = 0, -1, -2, -3, -4, -5
E_NOT_PD, E_NONFINITE, W_EMPTY_CLUSTER, E_BAD_IDX = 1, 2, 3, 4
C128, C64 = 0, 1
PRECS = {"fp64": 0, "fp32": 1, "bf16x6": 2, "fp16x3": 3}
WEIGHTS = {"ssm": 0, "psm": 1, "sm": 2, "scm": 3, "sqm": 4}
KM_WEIGHT_GIVEN = 1
FIT_FACTOR = 1
BWD_FIRST, BWD_LAST = 1, 2


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double * 3)]


class KmeansInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("converged", C.c_int32),
                ("empty_update", C.c_int32), ("empty_final", C.c_int32), ("ties", C.c_int32),
                ("near_ties", C.c_int32), ("changed", C.c_int32), ("objective", C.c_double),
                ("pairs_evaluated", C.c_int64), ("bound_tests", C.c_int64)]


class QrcpInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("rank", C.c_int32), ("near_ties", C.c_int32),
                ("reserved", C.c_int32), ("r00", C.c_double)]


class FitInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("pivot", C.c_int32), ("bad_idx", C.c_int32),
                ("reserved", C.c_int32), ("pivot_min", C.c_double), ("pivot_max", C.c_double),
                ("loss", C.c_double)]


_P = C.c_void_p
_I32, _I64, _U32, _D, _SZ = C.c_int32, C.c_int64, C.c_uint32, C.c_double, C.c_size_t
_G = C.POINTER(Grid)

SIGNATURES = {
    "isdf_version": (C.c_char_p, []),
    "isdf_strerror": (C.c_char_p, [C.c_int]),
    "isdf_kmeans_workspace": (_SZ, [_G, _I32, _I32]),
    "isdf_kmeans": (C.c_int, [_G, C.c_int, _P, _I64, _I32, _P, _I64, _I32, _I32, _U32, _I32, _P, _I32, _D,
                              _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "isdf_kmeans_noalloc": (C.c_int, [_G, C.c_int, _P, _I64, _I32, _P, _I64, _I32, _I32, _U32, _I32, _P, _I32, _D,
                                      _P, _P, _P, _P, _P, _P, _P]),
    "isdf_fit_minv_elems": (_SZ, [_I32, _I32]),
    "isdf_fit_workspace": (_SZ, [_G, _I32, _I32, _I32, _I32, C.c_int, _I64]),
    "isdf_fit_backward_workspace": (_SZ, [_G, _I32, _I32, _I32, _I32, C.c_int, _I64]),
    "isdf_fit": (C.c_int, [_G, C.c_int, _P, _I64, _I32, _P, _I64, _I32, _P, _I32, C.c_int, _P, _U32, _I64,
                           _I64, _P, _I64, _I64, _P, _P, _SZ, _P]),
    "isdf_zc_workspace": (_SZ, [_I32, _I32, _I32, _I32, C.c_int, _I64]),
    "isdf_zc": (C.c_int, [_G, C.c_int, _P, _I64, _I32, _P, _I64, _I32, _P, _I32, C.c_int, _I64, _I64, _P, _I64,
                          _P, _SZ, _P]),
    "isdf_zc_ab": (C.c_int, [_G, C.c_int, _P, _I64, _I32, _P, _I64, _I32, _P, _I32, C.c_int, _I64, _I64, _P, _I64,
                             _P, _P, _P, _SZ, _P]),
    "isdf_apply_minv": (C.c_int, [_I32, _I32, _P, _P, _I64, _I64, C.c_int, _P, _I64, _P]),
    "isdf_fit_backward": (C.c_int, [_G, C.c_int, _P, _I64, _I32, _P, _I64, _I32, _P, _I32, C.c_int, _P,
                                    _P, _I64, _P, _P, _I64, _P, _I64, _P, _I64, _P, _P, _SZ, _P]),
    "isdf_fit_backward_gram_workspace": (_SZ, [_G, _I32, _I32, _I32, _I32, C.c_int, _I64]),
    "isdf_fit_backward_gram": (C.c_int, [_G, C.c_int, _P, _I64, _I32, _P, _I64, _I32, _P, _I32, C.c_int, _P,
                                         _P, _I64, _P, _P, _I64, _P, _I64, _P, _I64, _P, _P, _P, _P, _P, _SZ, _P]),
    "isdf_fit_backward_rows": (C.c_int, [_G, C.c_int, _P, _I64, _I32, _P, _I64, _I32, _P, _I32, C.c_int, _P,
                                         _P, _I64, _P, _P, _I64, _P, _I64, _P, _I64, _I64, _I64, _P, _P, _P, _U32,
                                         _P, _P, _SZ, _P]),
    "isdf_fit_residual_workspace": (_SZ, [_G, _I32, _I32, _I32, _I32, C.c_int, _I64]),
    "isdf_fit_residual": (C.c_int, [_G, C.c_int, _P, _I64, _I32, _P, _I64, _I32, _P, _I32, C.c_int, _P, _I64, _P,
                                    _P, _P, _SZ, _P]),
    "isdf_poisson_workspace": (_SZ, [_G, _I32, _I32]),
    "isdf_poisson": (C.c_int, [_G, C.c_int, _P, _I64, _I32, _I32, _P, _I64, _P, _SZ, _P]),
    "isdf_exchange_workspace": (_SZ, [_G, _I32, _I32, _I32, _I64]),
    "isdf_exchange": (C.c_int, [_G, C.c_int, _P, _I64, _I32, _P, _I64, _I32, _P, _I32, _P, _I64, _I32, _P, _I64,
                                _I64, _P, _SZ, _P]),
    "isdf_qrcp_workspace": (_SZ, [_G, _I32, _I32]),
    "isdf_qrcp": (C.c_int, [_G, C.c_int, _P, _I64, _I32, _P, _I64, _I32, _I32, _D, _D, _P, _P, _P, _P, _P, _SZ,
                            _P]),
    "isdf_qrcp_sketch_workspace": (_SZ, [_G, _I32, _I32, _I32, _I32]),
    "isdf_qrcp_sketch": (C.c_int, [_G, C.c_int, _P, _I64, _I32, _P, _I64, _I32, _P, _P, _I32, _I32, _D, _D, _P, _P,
                                   _P, _P, _P, _SZ, _P]),
    "isdf_cluster_residual_workspace": (_SZ, []),
    "isdf_cluster_residual": (C.c_int, [_G, C.c_int, _P, _I64, _I32, _P, _I64, _I32, _P, _P, _I32, _P, _P, _SZ,
                                        _P]),
}

_lib = None


def load() -> C.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2208_07731_amd.build`")
    import torch  # noqa: F401  (maps torch's HIP runtime before ours resolves it)
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().isdf_strerror(int(code)).decode()


def make_grid(n, h=(1.0, 1.0, 1.0)) -> Grid:
    if isinstance(n, int):
        n = (n, n, n)
    g = Grid()
    for a in range(3):
        g.n[a] = int(n[a])
        g.h[a] = float(h[a])
    return g
