"""ctypes binding of libshssa.so: argument marshalling only.

Every call lands in the C ABI declared in include/shssa.h; nothing here
computes any part of the method.  Loading fails loudly when the library has
not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libshssa.so")

SSA_OK, SSA_EINVAL, SSA_EEMPTY, SSA_ERANK, SSA_ENOMEM, SSA_ENOCONV, SSA_EDEVICE, SSA_EBUSY, SSA_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
SSA_FP64, SSA_FP32, SSA_FP32_BASIS32 = 0, 1, 2


class Request(C.Structure):
    _fields_ = [("x", C.c_void_p), ("nx", C.c_int), ("ny", C.c_int), ("mask", C.c_void_p),
                ("wmask", C.c_void_p), ("lx", C.c_int), ("ly", C.c_int), ("r", C.c_int),
                ("precision", C.c_int), ("seed", C.c_ulonglong)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int), ("restarts", C.c_int), ("basis", C.c_int), ("converged", C.c_int),
                ("side", C.c_int), ("batch", C.c_int), ("svd_sweeps", C.c_int), ("max_resid", C.c_double), ("ms_setup", C.c_double),
                ("ms_lanczos", C.c_double), ("ms_finish", C.c_double), ("device_bytes", C.c_size_t),
                ("fft_rows", C.c_int), ("fft_cols", C.c_int)]


class Times(C.Structure):
    _fields_ = [("queue_ms", C.c_double), ("total_ms", C.c_double)]


_lib = None

_SIGS = {
    "ssa_ctx_create": (C.c_int, [C.c_int, C.c_size_t, C.c_char_p, C.POINTER(C.c_void_p)]),
    "ssa_ctx_destroy": (None, [C.c_void_p]),
    "ssa_ctx_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ssa_ctx_sync": (C.c_int, [C.c_void_p]),
    "ssa_ctx_set_slots": (C.c_int, [C.c_void_p, C.c_int]),
    "ssa_ctx_profile": (C.c_int, [C.c_void_p, C.c_char_p]),
    "ssa_ctx_profile_every": (C.c_int, [C.c_void_p, C.c_int]),
    "ssa_ctx_profile_read": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_long),
                                       C.POINTER(C.c_double)]),
    "ssa_ctx_profile_read_kind": (C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_long),
                                            C.POINTER(C.c_double)]),
    "ssa_ctx_profile_launches": (C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_long)]),
    "ssa_decompose": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                C.c_int, C.c_int, C.c_int, C.POINTER(C.c_void_p)]),
    "ssa_decompose_multi": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.c_void_p, C.c_int, C.c_int,
                                      C.c_int, C.c_int, C.POINTER(C.c_void_p)]),
    "ssa_decompose_batch": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(Request), C.POINTER(C.c_void_p),
                                      C.POINTER(C.c_int)]),
    "ssa_decompose_batch_dev": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(Request), C.POINTER(C.c_void_p),
                                          C.POINTER(C.c_int)]),
    "ssa_get_dims": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                               C.POINTER(C.c_int), C.POINTER(C.c_long), C.POINTER(C.c_long),
                               C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "ssa_get_sigma": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ssa_get_vectors": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ssa_get_vectors_lex": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ssa_get_weights": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ssa_reconstruct": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "ssa_wcor": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "ssa_orthogonality": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "ssa_rforecast": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_int)]),
    "ssa_extend": (C.c_int, [C.c_void_p, C.c_int]),
    "ssa_esprit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "ssa_esprit_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "ssa_esprit_tls": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "ssa_esprit2d": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ssa_decompose_mosaic": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                       C.c_int, C.c_void_p, C.c_void_p]),
    "ssa_decompose_m2d": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                                    C.c_int, C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "ssa_decompose_eigen": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                      C.c_int, C.c_int, C.POINTER(C.c_void_p)]),
    "ssa_vforecast": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_int)]),
    "ssa_rforecast_row": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_int)]),
    "ssa_vforecast_row": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_int)]),
    "ssa_reconstruct_batch_dev": (C.c_int, [C.c_int, C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p, C.c_int,
                                            C.POINTER(C.c_void_p)]),
    "ssa_get_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    "ssa_submit": (C.c_int, [C.c_void_p, C.POINTER(Request), C.c_void_p, C.c_void_p, C.c_int,
                             C.POINTER(C.c_uint64)]),
    "ssa_submit_multi": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.c_void_p, C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_uint64)]),
    "ssa_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int)]),
    "ssa_wait": (C.c_int, [C.c_void_p, C.c_uint64]),
    "ssa_take": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_void_p), C.c_void_p, C.POINTER(Times)]),
    "ssa_free": (None, [C.c_void_p]),
    "ssa_strerror": (C.c_char_p, [C.c_int]),
    "ssa_last_error": (C.c_char_p, []),
}


def lib():
    """Load libshssa.so (raises if it has not been built).

    PyTorch is imported first when it is installed: its wheel carries its own
    HIP runtime under the same soname, and the library must bind to that one
    so that torch's streams and device buffers are valid in its calls."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIBPATH):
            raise RuntimeError("libshssa.so is not built: run __graft_entry__.build() "
                               "or python paper_1309_5050_amd/build.py")
        L = C.CDLL(LIBPATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class SsaError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        L = lib()
        msg = L.ssa_strerror(code).decode()
        detail = L.ssa_last_error().decode()
        super().__init__(f"{what}: {msg} ({detail})" if what else f"{msg} ({detail})")
        self.code = code


def check(code: int, what: str = "") -> int:
    if code != SSA_OK:
        raise SsaError(code, what)
    return code
