"""ctypes declarations of libspm (include/spm.h).  Loading fails loudly when the
shared library has not been built."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspm.so")

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double
_INT = ctypes.c_int

# name -> argtypes (every function returns int status except the two string getters)
SIGNATURES = {
    "spm_tree_build": [_P, _I64, _I32, _I32, _I32, _P],
    "spm_tree_destroy": [_P],
    "spm_tree_info": [_P, _P, _P, _P],
    "spm_tree_arrays": [_P, _P, _P, _P, _P, _P],
    "spm_tree_block_pattern": [_P, _D, _P, _P, _P],
    "spm_compress_pattern_upload": [_I64, _P, _P, _I32, _P, _P, _P],
    "spm_block_pattern_upload": [_I64, _I32, _P, _P, _P, _P, _P],
    "spm_block_pattern_plan": [_I64, _I32, _P, _P, _P, _P, _P],
    "spm_compress_pattern_plan": [_I64, _P, _P, _I32, _P, _P, _P],
    "spm_pattern_upload": [_P, _P],
    "spm_pattern_workspace_bytes": [_P, _P],
    "spm_pattern_upload_workspace": [_P, _P, ctypes.c_size_t, _P],
    "spm_pattern_classes": [_P, _P, _P, _P, _P, _P, _P, _P],
    "spm_pattern_destroy": [_P],
    "spm_pattern_info": [_P, _P, _P, _P, _P],
    "spm_pattern_tiles": [_P, _P, _P, _P],
    "spm_pattern_download_csr": [_P, _P, _P],
    "spm_values_from_csr": [_P, _P, _P, _P],
    "spm_values_to_csr": [_P, _P, _P, _P],
    "spm_kernel_compress": [_P, _P, _I32, _D, _D, _I32, _P, _P],
    "spm_masked_gemm": [_P, _INT, _P, _INT, _P, _INT, _P, _P],
    "spm_masked_gemm_workspace": [_P, _INT, _INT, _INT, _P],
    "spm_masked_gemm_ws": [_P, _INT, _P, _INT, _P, _INT, _P, _P, ctypes.c_size_t, _P],
    "spm_masked_gemm_noalloc_max_bytes": [_P],
    "spm_masked_gemm_noalloc": [_P, _INT, _P, _INT, _P, _INT, _P, _P],
    "spm_masked_gemm_backward": [_P, _INT, _P, _P, _P, _P, _P, _P],
    "spm_masked_gemm_backward_workspace": [_P, _INT, _P],
    "spm_masked_gemm_backward_ws": [_P, _INT, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P],
    "spm_axpy": [_P, _INT, _D, _P, _D, _P, _P],
    "spm_convert": [_P, _INT, _P, _INT, _P, _P],
    "spm_sqdist": [_P, _INT, _P, _P, _P, _P],
    "spm_sqdist_eye": [_P, _INT, _D, _P, _P, _P],
    "spm_dot": [_P, _P, _P, _P, _P],
    "spm_quadform": [_P, _P, _P, _P, _P],
    "spm_fill_outer": [_P, _D, _P, _P, _P],
    "spm_spmm": [_P, _P, _P, _I32, _P, _P],
    "spm_fst": [_P, _P, _I32, _P, _I32, _P],
    "spm_contour_rule": [_D, _D, _I32, _P, _P],
    "spm_contour_invsqrt_scratch": [_P, _I32, _P],
    "spm_contour_invsqrt": [_P, _P, _D, _D, _I32, _I32, _P, _P, _P, ctypes.c_size_t, _P],
    "spm_ns_sqrt_scratch": [_P, _P],
    "spm_ns_sqrt": [_P, _P, _P, _P, _I32, _P, _P, ctypes.c_size_t, _P],
    "spm_expm_taylor_scratch": [_P, _P],
    "spm_expm_taylor": [_P, _P, _P, _I32, _P, ctypes.c_size_t, _P],
    "spm_newton_schulz_scratch": [_P, _INT, _P],
    "spm_newton_schulz": [_P, _P, _P, _I32, _I32, _INT, _D, _P, _P, _P, ctypes.c_size_t, _P],
}

_lib = None


class SpmError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func}: status {status} ({msg})")
        self.status = status


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libspm.so not built: expected {LIB_PATH} (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.spm_status_string.argtypes = [ctypes.c_int]
    lib.spm_status_string.restype = ctypes.c_char_p
    lib.spm_last_error.argtypes = []
    lib.spm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def call(name: str, *args) -> int:
    lib = load()
    st = getattr(lib, name)(*args)
    if st != 0:
        raise SpmError(st, name, lib.spm_last_error().decode())
    return st
