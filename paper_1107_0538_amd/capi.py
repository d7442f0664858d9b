"""ctypes binding of libjpcg.so: argument marshalling only.

Every computation happens in the HIP library.  This module never imports the
oracle and has no CPU fallback: if the library is not built, load() raises.
"""
from __future__ import annotations

import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libjpcg.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "jpcg.h")
PROBE_HEADER = os.path.join(os.path.dirname(PKG), "include", "jpcg_probe.h")

CG_CONVERGED, CG_MAXIT, CG_BREAKDOWN = 0, 1, 2
CG_EINVAL, CG_EDIAG, CG_ENOMEM, CG_EHIP, CG_ETIMEOUT, CG_EUNSUPPORTED, CG_ESCRATCH = -1, -2, -3, -4, -5, -6, -7
GRAM_SCRATCH_DOUBLES, GRAM_CHUNK = 4 << 20, 2048
CG_MEM_HOST, CG_MEM_DEVICE = 0, 1
CG_PRECOND_DEFAULT, CG_PRECOND_JACOBI, CG_PRECOND_NONE = 0, 1, 2
CG_FORM_STANDARD, CG_FORM_SINGLE_REDUCTION = 0, 1
FORMS = {"standard": CG_FORM_STANDARD, "single": CG_FORM_SINGLE_REDUCTION}

_P = ctypes.c_void_p


class cg_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("mem", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("rowptr", _P), ("col", _P), ("val", _P)]


class cg_opts(ctypes.Structure):
    _fields_ = [("precond", ctypes.c_int32), ("fp32_copy", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("nnz_per_lane", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("history", ctypes.c_int32), ("block_size", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("form", ctypes.c_int32), ("col_bits", ctypes.c_int32), ("reserved", ctypes.c_int32 * 6)]


class cg_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("replacements", ctypes.c_int32),
                ("outer", ctypes.c_int32), ("relres_recur", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class cg_config(ctypes.Structure):
    _fields_ = [("nnz_per_lane", ctypes.c_int32), ("block_size", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("tiles", ctypes.c_int32), ("chunk", ctypes.c_int32), ("form", ctypes.c_int32),
                ("tune_cached", ctypes.c_int32), ("col_bits", ctypes.c_int32),
                ("spmv_nnz_per_lane", ctypes.c_int32), ("spmv_block_size", ctypes.c_int32),
                ("spmv_grid", ctypes.c_int32), ("spmv_us", ctypes.c_double), ("iter_us", ctypes.c_double),
                ("spmm_blocks_per_cu", ctypes.c_int32), ("spmm_pad", ctypes.c_int32), ("spmm_us", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes)
SIGNATURES = {
    "cg_opts_default": (None, [ctypes.POINTER(cg_opts)]),
    "cg_create": (ctypes.c_int, [ctypes.POINTER(cg_csr), ctypes.POINTER(cg_opts), _P, ctypes.POINTER(_P)]),
    "cg_solve": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(cg_info)]),
    "cg_solve_mixed": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_int32, ctypes.POINTER(cg_info)]),
    "cg_solve_mixed_matrix": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                             ctypes.POINTER(cg_info)]),
    "spmv": (ctypes.c_int, [_P, _P, _P]),
    "jpcg_stream_triad": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_int64, ctypes.c_int32, _P]),
    "spmm": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32]),
    "cg_solve_multi": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                      ctypes.POINTER(cg_info)]),
    "cg_solve_multi_mixed": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                            ctypes.c_double, ctypes.c_int32, ctypes.POINTER(cg_info)]),
    "cg_solve_block": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                      ctypes.POINTER(cg_info)]),
    "cg_batch_create": (ctypes.c_int, [ctypes.c_int32, _P, ctypes.POINTER(cg_opts), _P, ctypes.POINTER(_P)]),
    "cg_batch_solve": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(cg_info)]),
    "cg_batch_offset": (ctypes.c_int64, [_P, ctypes.c_int32]),
    "cg_batch_teams": (ctypes.c_int, [_P, _P]),
    "cg_batch_last_error": (ctypes.c_char_p, [_P]),
    "cg_batch_destroy": (None, [_P]),
    "dense_gram": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, _P, ctypes.c_int32,
                                  ctypes.c_int64, _P, _P]),
    "dense_gram_noalloc": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, _P, ctypes.c_int32,
                                          ctypes.c_int64, _P, _P]),
    "dense_gemm": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, _P, ctypes.c_int32, _P,
                                  ctypes.c_int64, _P]),
    "pod_decode": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, _P, ctypes.c_int32, _P, _P,
                                  _P, _P]),
    "q1_apply": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, _P, _P, _P, _P]),
    "q1_assemble": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, _P, _P, _P, _P, _P]),
    "mlp_create": (ctypes.c_int, [ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "mlp_param_count": (ctypes.c_int64, [_P]),
    "mlp_set_params": (ctypes.c_int, [_P, _P]),
    "mlp_get_params": (ctypes.c_int, [_P, _P]),
    "mlp_forward": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P]),
    "mlp_gradients": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_double)]),
    "mlp_train_step": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, ctypes.POINTER(ctypes.c_double)]),
    "mlp_destroy": (None, [_P]),
    "cg_get_history": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "cg_get_config": (ctypes.c_int, [_P, ctypes.POINTER(cg_config)]),
    "cg_destroy": (None, [_P]),
    "cg_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "cg_last_error": (ctypes.c_char_p, [_P]),
}

_lib = None


def load():
    """Load the built HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_1107_0538_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_functions(path: str = HEADER) -> list[str]:
    """Names of the functions declared in the public header."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) - {"if", "sizeof", "defined"})


class CGError(RuntimeError):
    def __init__(self, code: int, detail: str = ""):
        self.code = code
        msg = load().cg_strerror(code).decode()
        super().__init__(f"{msg} ({code})" + (f": {detail}" if detail else ""))


def check(code: int, ctx=None) -> int:
    if code < 0:
        detail = load().cg_last_error(ctx).decode() if ctx else ""
        if code == CG_EINVAL:
            raise ValueError(CGError(code, detail))
        raise CGError(code, detail)
    return code
