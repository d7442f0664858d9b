"""Oracle for the GPU solver -- TEST INFRASTRUCTURE ONLY.

Plain CPU implementations of what the GPU path computes, written from the
paper and from textbook definitions.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the GPU library and its
Python binding never do, and this package never imports them.

- `pcg`, `pcg_mixed_matrix`, `spmv`, `residual`, `dot`: FP64 C code in pcg_oracle.c, loaded
  through ctypes (built with gcc, -O2 -ffp-contract=off).  A second build of
  the same source with -fopenmp (`pcg(..., parallel=True)`) exists only to
  time the oracle on all host cores; its dot products sum in another order.
- `mlp`: an FP64 numpy multilayer perceptron (forward, backward, Adam).
- `pod`: proper orthogonal decomposition by the method of snapshots.
- `block_cg`: block PCG for several right-hand sides (O'Leary's method in
  the breakdown-free form, search blocks orthonormalised by shifted
  Cholesky QR), numpy FP64 around the C oracle's product.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pcg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")

CONVERGED, MAXIT, BREAKDOWN = 0, 1, 2
EINVAL, EDIAG, ENOMEM = -1, -2, -3
STATUS_NAMES = {0: "CONVERGED", 1: "MAXIT", 2: "BREAKDOWN", -1: "EINVAL", -2: "EDIAG", -3: "ENOMEM"}


class OracleInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("status", ctypes.c_int),
        ("replacements", ctypes.c_int),
        ("pad", ctypes.c_int),
        ("relres_recur", ctypes.c_double),
        ("relres_true", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


def build(out: str = LIB) -> str:
    """Compile the oracle with gcc: -O2, no fused multiply-add, no fast-math."""
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           SRC, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build_omp(out: str = LIB_OMP) -> str:
    """The same source with OpenMP, for timing the oracle on every host core."""
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           SRC, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_libs = {}
_lib = None  # the plain build (tests swap it for mutated copies)


def _bind(L):
    P = ctypes.c_void_p
    L.oracle_spmv.argtypes = [ctypes.c_int, P, P, P, P, P]
    L.oracle_spmv.restype = ctypes.c_int
    L.oracle_dot.argtypes = [ctypes.c_int, P, P, ctypes.c_int]
    L.oracle_dot.restype = ctypes.c_double
    L.oracle_residual.argtypes = [ctypes.c_int, P, P, P, P, P, P]
    L.oracle_residual.restype = ctypes.c_double
    L.oracle_pcg.argtypes = [ctypes.c_int, P, P, P, P, P, ctypes.c_double, ctypes.c_int,
                             ctypes.c_int, ctypes.c_int, ctypes.POINTER(OracleInfo), P, P]
    L.oracle_pcg.restype = ctypes.c_int
    L.oracle_pcg_sr.argtypes = L.oracle_pcg.argtypes
    L.oracle_pcg_sr.restype = ctypes.c_int
    L.oracle_pcg_m32.argtypes = [ctypes.c_int, P, P, P, P, P, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_double, ctypes.POINTER(OracleInfo)]
    L.oracle_pcg_m32.restype = ctypes.c_int
    L.oracle_threads.argtypes = []
    L.oracle_threads.restype = ctypes.c_int
    return L


def lib(parallel: bool = False):
    """Load the oracle library (the OpenMP build with parallel=True),
    building it first if nothing is built."""
    global _lib
    if parallel:
        if "omp" not in _libs:
            if not os.path.exists(LIB_OMP):
                build_omp()
            _libs["omp"] = _bind(ctypes.CDLL(LIB_OMP))
        return _libs["omp"]
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = _bind(ctypes.CDLL(LIB))
    return _lib


def threads(parallel: bool = False) -> int:
    """Threads a solve of that build uses (1 for the plain build)."""
    return lib(parallel).oracle_threads()


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr_arrays(a):
    rowptr = np.ascontiguousarray(a.rowptr, dtype=np.int32)
    col = np.ascontiguousarray(a.col, dtype=np.int32)
    val = np.ascontiguousarray(a.val, dtype=np.float64)
    return rowptr, col, val


def spmv(a, x) -> np.ndarray:
    """y = A x in FP64, rows summed in stored order."""
    rowptr, col, val = _csr_arrays(a)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(a.n)
    rc = lib().oracle_spmv(a.n, _p(rowptr), _p(col), _p(val), _p(x), _p(y))
    if rc != 0:
        raise ValueError("oracle_spmv: bad arguments")
    return y


def dot(x, y, mode: int = 0) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    return lib().oracle_dot(x.size, _p(x), _p(y), mode)


def residual(a, b, x) -> tuple[np.ndarray, float]:
    """(r = b - A x, ||r||_2)."""
    rowptr, col, val = _csr_arrays(a)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    r = np.empty(a.n)
    nr = lib().oracle_residual(a.n, _p(rowptr), _p(col), _p(val), _p(b), _p(x), _p(r))
    return r, nr


def relres(a, b, x) -> float:
    """||b - A x|| / ||b|| in FP64."""
    _, nr = residual(a, b, x)
    nb = float(np.sqrt(dot(b, b)))
    return nr / nb if nb > 0 else nr


def pcg(a, b, x0=None, tol: float = 1e-10, maxit: int = 0, precond: str = "jacobi",
        sum_mode: int = 0, history: bool = False, trace: bool = False, form: str = "standard",
        parallel: bool = False):
    """Run the oracle solve.  Returns (x, info dict[, hist][, trace]).

    form: "standard" (two reductions per iteration) or "single" (the
    single-reduction Chronopoulos-Gear form of the same iteration).
    parallel: run the OpenMP build (timing only).
    """
    rowptr, col, val = _csr_arrays(a)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(a.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    mi = a.n if maxit <= 0 else maxit
    hist = np.full(mi + 1, np.nan) if history else None
    tr = np.full((mi + 1, 4, a.n), np.nan) if trace else None
    info = OracleInfo()
    pc = {"none": 0, "jacobi": 1}[precond]
    L = lib(parallel)
    fn = {"standard": L.oracle_pcg, "single": L.oracle_pcg_sr}[form]
    fn(a.n, _p(rowptr), _p(col), _p(val), _p(b), _p(x), tol, mi, pc, sum_mode,
       ctypes.byref(info), _p(hist) if history else None, _p(tr) if trace else None)
    d = info.as_dict()
    out = [x, d]
    if history:
        out.append(hist[: d["iters"] + 1])
    if trace:
        out.append(tr[: d["iters"] + 1])
    return tuple(out)


def pcg_mixed_matrix(a, b, x0=None, tol: float = 1e-10, maxit: int = 0, precond: str = "jacobi",
                     drop: float = 1e-2, parallel: bool = False):
    """The FP64 solve whose loop products use the FP32-rounded values in the
    row-sum-preserving evaluation, confirming on the FP64 true residual each
    time the residual has fallen by `drop` since the last replacement
    (oracle_pcg_m32).  Returns (x, info dict)."""
    rowptr, col, val = _csr_arrays(a)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(a.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    info = OracleInfo()
    lib(parallel).oracle_pcg_m32(a.n, _p(rowptr), _p(col), _p(val), _p(b), _p(x), tol, a.n if maxit <= 0 else maxit,
                                 {"none": 0, "jacobi": 1}[precond], float(drop), ctypes.byref(info))
    return x, info.as_dict()
