"""ctypes binding of libtucker_als.so (argument marshalling only).

Every step of the computation runs in the library's HIP kernels; PyTorch only
supplies device memory and the current stream.  There is no fallback: if the
library is not built, loading raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtucker_als.so")

TK_F64, TK_F32, TK_BF16 = 0, 1, 2
TK_RESID_AUTO, TK_RESID_TRACE, TK_RESID_EXPLICIT = 0, 1, 2
TK_COMPUTE_AS_STORAGE = 0
TK_MAX_ORDER = 8

STATUS = {
    0: "TK_OK", 1: "TK_NOT_CONVERGED", 2: "TK_SKIPPED", -1: "TK_ERR_INVALID_ARG",
    -2: "TK_ERR_UNSUPPORTED_DTYPE", -3: "TK_ERR_WORKSPACE_TOO_SMALL",
    -4: "TK_ERR_RANK_DEFICIENT", -5: "TK_ERR_NONFINITE", -6: "TK_ERR_HIP",
}

# Every symbol declared in include/tucker_als.h.
EXPORTS = [
    "als_sthosvd", "als_thosvd", "als_workspace_bytes", "ttm",
    "tucker_reconstruct", "tucker_reconstruct_workspace_bytes",
    "contract_allbut", "contract_allbut_workspace_bytes", "als_init_step",
    "als_sweep_step", "als_sweep_kernel", "qr_f64", "als_sthosvd_batched",
    "als_sthosvd_batched_workspace_bytes", "hooi_refine", "hooi_workspace_bytes",
    "st_order_auto", "tk_status_string", "als_sthosvd_noalloc", "als_sthosvd_noalloc_max_bytes",
]


class tk_als_opts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_size_t),
        ("tol", ctypes.c_double),
        ("max_iters", ctypes.c_int32),
        ("resid_mode", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("order", ctypes.POINTER(ctypes.c_int32)),
        ("singular_vectors", ctypes.c_int32),
        ("compute", ctypes.c_int32),
        ("init_U", ctypes.POINTER(ctypes.c_void_p)),
    ]


class tk_als_info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32 * TK_MAX_ORDER),
        ("converged", ctypes.c_int32 * TK_MAX_ORDER),
        ("resid", ctypes.c_double * TK_MAX_ORDER),
        ("norm_a", ctypes.c_double),
        ("sweeps", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("mode_status", ctypes.c_int32 * TK_MAX_ORDER),
        ("resid_form", ctypes.c_int32 * TK_MAX_ORDER),
    ]


class tk_hooi_info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("relerr_init", ctypes.c_double),
        ("relerr", ctypes.c_double),
        ("norm_a", ctypes.c_double),
        ("sweeps", ctypes.c_int32),
        ("status", ctypes.c_int32),
    ]


class TuckerALSError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = int(code)
        super().__init__(f"{where}: {STATUS.get(self.code, self.code)}")


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
_SZ = ctypes.c_size_t
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PI32 = ctypes.POINTER(ctypes.c_int32)
_PD = ctypes.POINTER(ctypes.c_double)


def _declare(lib):
    drv = [_P, _I32, _I32, _PI64, _PI32, ctypes.POINTER(tk_als_opts),
           ctypes.POINTER(_P), _P, _P, _SZ, ctypes.POINTER(tk_als_info), _P]
    lib.als_sthosvd.argtypes = drv
    lib.als_thosvd.argtypes = drv
    lib.als_sthosvd.restype = lib.als_thosvd.restype = _I32
    lib.als_sthosvd_noalloc.argtypes = [_P, _I32, _I32, _PI64, _PI32,
                                        ctypes.POINTER(tk_als_opts), ctypes.POINTER(_P), _P,
                                        ctypes.POINTER(tk_als_info), _P]
    lib.als_sthosvd_noalloc.restype = _I32
    lib.als_sthosvd_noalloc_max_bytes.argtypes = []
    lib.als_sthosvd_noalloc_max_bytes.restype = _SZ
    lib.als_workspace_bytes.argtypes = [_I32, _I32, _I32, _PI64, _PI32]
    lib.als_workspace_bytes.restype = _SZ
    lib.ttm.argtypes = [_P, _I32, _I32, _PI64, _I32, _P, _I32, _I64, _I32, _P, _I32, _P]
    lib.ttm.restype = _I32
    lib.tucker_reconstruct.argtypes = [_P, _I32, _I32, _PI32, _PI64, ctypes.POINTER(_P),
                                       _P, _P, _SZ, _P]
    lib.tucker_reconstruct.restype = _I32
    lib.tucker_reconstruct_workspace_bytes.argtypes = [_I32, _I32, _PI32, _PI64]
    lib.tucker_reconstruct_workspace_bytes.restype = _SZ
    lib.contract_allbut.argtypes = [_P, _P, _I32, _I32, _PI64, _I32, _I64, _P, _P, _SZ, _P]
    lib.contract_allbut.restype = _I32
    lib.contract_allbut_workspace_bytes.argtypes = [_I32, _I32, _PI64, _I32, _I64]
    lib.contract_allbut_workspace_bytes.restype = _SZ
    lib.als_init_step.argtypes = [_P, _I32, _I32, _PI64, _I32, _I32, _U64, _P, _P, _PD,
                                  _P, _SZ, _P]
    lib.als_init_step.restype = _I32
    lib.als_sweep_step.argtypes = [_P, _I32, _I32, _PI64, _I32, _I32, _P, _P,
                                   ctypes.c_double, _I32, _PD, _P, _SZ, _P]
    lib.als_sweep_step.restype = _I32
    lib.als_sweep_kernel.argtypes = [_P, _I32, _I32, _PI64, _I32, _I32, _P, _P, _P, _I32, _P,
                                     _SZ, _P]
    lib.als_sweep_kernel.restype = _I32
    lib.qr_f64.argtypes = [_P, _I64, _I32, _P, _P, _P, _SZ, _P]
    lib.qr_f64.restype = _I32
    lib.als_sthosvd_batched.argtypes = [_P, _I32, _I32, _PI64, _PI32, _PI64,
                                        ctypes.POINTER(tk_als_opts), _P, _PI64, _P, _PI64,
                                        _PI32, _PI32, _P, _SZ, _P]
    lib.als_sthosvd_batched.restype = _I32
    lib.als_sthosvd_batched_workspace_bytes.argtypes = [_I32, _PI64, _PI32]
    lib.als_sthosvd_batched_workspace_bytes.restype = _SZ
    lib.hooi_refine.argtypes = [_P, _I32, _I32, _PI64, _PI32, ctypes.POINTER(tk_als_opts),
                                ctypes.c_double, _I32, ctypes.POINTER(_P), _P, _P, _SZ,
                                ctypes.POINTER(tk_hooi_info), _P]
    lib.hooi_refine.restype = _I32
    lib.hooi_workspace_bytes.argtypes = [_I32, _I32, _PI64, _PI32]
    lib.hooi_workspace_bytes.restype = _SZ
    lib.st_order_auto.argtypes = [_I32, _PI64, _PI32, _PI32]
    lib.st_order_auto.restype = _I32
    lib.tk_status_string.argtypes = [_I32]
    lib.tk_status_string.restype = ctypes.c_char_p


def load_library(path: str | None = None):
    """Load libtucker_als.so (raises if it has not been built).  The
    environment variable TUCKER_ALS_LIBRARY names another build of the same
    library (the sanitizer build, for instance)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or os.environ.get("TUCKER_ALS_LIBRARY") or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(
            f"{p} is missing: build it with `python -m paper_2004_02583_amd.build` "
            "(the HIP library is required; there is no fallback path)")
    lib = ctypes.CDLL(p)
    _declare(lib)
    _lib = lib
    return lib


def lib():
    return load_library()


def i64arr(vals):
    a = (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])
    return a


def i32arr(vals):
    return (ctypes.c_int32 * len(vals))(*[int(v) for v in vals])


def ptrarr(ptrs):
    return (ctypes.c_void_p * len(ptrs))(*[ctypes.c_void_p(int(p)) for p in ptrs])


def check(code: int, where: str, allow=(0,)):
    if code not in allow:
        raise TuckerALSError(code, where)
    return code
