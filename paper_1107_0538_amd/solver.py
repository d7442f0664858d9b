"""Python face of the C-ABI: torch supplies device memory and the stream.

Names follow the C calls (cg_create / cg_solve / spmv).  Nothing here
computes: each method validates and marshals its arguments, then calls the
HIP library.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import capi


def _torch():
    import torch

    return torch


def _as_device_vec(t, n, name, dtype=None):
    torch = _torch()
    dtype = dtype or torch.float64
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP torch tensor")
    if t.dtype != dtype or t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor with {n} entries")
    return t


def make_csr(a) -> tuple[capi.cg_csr, list]:
    """cg_csr for a matrix given as an object with n/rowptr/col/val (numpy or torch)."""
    torch = _torch()
    keep = []
    if isinstance(a.rowptr, torch.Tensor) and a.rowptr.is_cuda:
        if a.rowptr.numel() != int(a.n) + 1 or a.val.numel() != a.col.numel():
            raise ValueError("rowptr must have n + 1 entries and val as many as col")
        rowptr = a.rowptr.to(torch.int32).contiguous()
        col = a.col.to(torch.int32).contiguous()
        val = a.val.to(torch.float64).contiguous()
        keep += [rowptr, col, val]
        csr = capi.cg_csr(int(a.n), capi.CG_MEM_DEVICE, int(col.numel()), rowptr.data_ptr(),
                          col.data_ptr(), val.data_ptr())
    else:
        rowptr = np.ascontiguousarray(a.rowptr, dtype=np.int32)
        col = np.ascontiguousarray(a.col, dtype=np.int32)
        val = np.ascontiguousarray(a.val, dtype=np.float64)
        keep += [rowptr, col, val]
        if val.size != col.size:
            raise ValueError("val must have as many entries as col")
        if rowptr.size != int(a.n) + 1:
            raise ValueError("rowptr must have n + 1 entries")
        csr = capi.cg_csr(int(a.n), capi.CG_MEM_HOST, int(col.size), rowptr.ctypes.data, col.ctypes.data,
                          val.ctypes.data)
    return csr, keep


def make_opts(precond="jacobi", fp32_copy=False, autotune=False, nnz_per_lane=0, blocks_per_cu=0,
              history=False, block_size=0, chunk=0, form="standard", col_bits=0) -> capi.cg_opts:
    o = capi.cg_opts()
    capi.load().cg_opts_default(ctypes.byref(o))
    o.precond = {"jacobi": capi.CG_PRECOND_JACOBI, "none": capi.CG_PRECOND_NONE}[precond]
    o.fp32_copy = int(bool(fp32_copy))
    o.autotune = int(bool(autotune))
    o.nnz_per_lane = int(nnz_per_lane)
    o.blocks_per_cu = int(blocks_per_cu)
    o.history = int(bool(history))
    o.block_size = int(block_size)
    o.chunk = int(chunk)
    o.form = capi.FORMS[form]
    o.col_bits = int(col_bits)
    return o


class Solver:
    """A cg_ctx: one SPD CSR matrix resident on the GPU."""

    def __init__(self, a, precond="jacobi", fp32_copy=False, autotune=False, nnz_per_lane=0,
                 blocks_per_cu=0, history=False, block_size=0, chunk=0, form="standard", col_bits=0,
                 stream=None):
        torch = _torch()
        self._lib = capi.load()
        self.n = int(a.n)
        self.nnz = int(a.rowptr[-1])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        csr, _keep = make_csr(a)
        opts = make_opts(precond, fp32_copy, autotune, nnz_per_lane, blocks_per_cu, history, block_size, chunk,
                         form, col_bits)
        ctx = ctypes.c_void_p()
        rc = self._lib.cg_create(ctypes.byref(csr), ctypes.byref(opts), ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(ctx))
        capi.check(rc)
        self.ctx = ctx
        self.history_enabled = bool(history)

    def close(self):
        if getattr(self, "ctx", None):
            self._lib.cg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- the three calls of the path ------------------------------------------------
    def cg_solve(self, b, x, tol=1e-10, maxit=0) -> dict:
        """In-place solve: x holds x0 on entry, the solution on exit."""
        _as_device_vec(b, self.n, "b")
        _as_device_vec(x, self.n, "x")
        info = capi.cg_info()
        rc = self._lib.cg_solve(self.ctx, b.data_ptr(), x.data_ptr(), float(tol), int(maxit), ctypes.byref(info))
        capi.check(rc, self.ctx)
        return info.as_dict()

    def solve(self, b, x0=None, tol=1e-10, maxit=0):
        torch = _torch()
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        info = self.cg_solve(b, x, tol, maxit)
        return x, info

    def cg_solve_mixed(self, b, x, tol=1e-10, maxit_outer=0, tol_inner=0.0, maxit_inner=0) -> dict:
        """In-place mixed-precision solve (FP32 inner CG, FP64 refinement)."""
        _as_device_vec(b, self.n, "b")
        _as_device_vec(x, self.n, "x")
        info = capi.cg_info()
        rc = self._lib.cg_solve_mixed(self.ctx, b.data_ptr(), x.data_ptr(), float(tol), int(maxit_outer),
                                      float(tol_inner), int(maxit_inner), ctypes.byref(info))
        capi.check(rc, self.ctx)
        return info.as_dict()

    def solve_mixed(self, b, x0=None, tol=1e-10, maxit_outer=0, tol_inner=0.0, maxit_inner=0):
        torch = _torch()
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        info = self.cg_solve_mixed(b, x, tol, maxit_outer, tol_inner, maxit_inner)
        return x, info

    def cg_solve_mixed_matrix(self, b, x, tol=1e-10, maxit=0, drop=0.0) -> dict:
        """FP64 iteration whose products stream FP32 values (needs fp32_copy); x holds x0 and the solution."""
        _as_device_vec(b, self.n, "b")
        _as_device_vec(x, self.n, "x")
        info = capi.cg_info()
        rc = self._lib.cg_solve_mixed_matrix(self.ctx, b.data_ptr(), x.data_ptr(), float(tol), int(maxit),
                                             float(drop), ctypes.byref(info))
        capi.check(rc, self.ctx)
        return info.as_dict()

    def solve_mixed_matrix(self, b, x0=None, tol=1e-10, maxit=0, drop=0.0):
        torch = _torch()
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        info = self.cg_solve_mixed_matrix(b, x, tol, maxit, drop)
        return x, info

    def spmv(self, x, y=None):
        torch = _torch()
        _as_device_vec(x, self.n, "x")
        if y is None:
            y = torch.empty_like(x)
        _as_device_vec(y, self.n, "y")
        capi.check(self._lib.spmv(self.ctx, x.data_ptr(), y.data_ptr()), self.ctx)
        return y

    # -- multi-RHS ------------------------------------------------------------------
    def _as_block(self, t, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or t.dim() != 2 \
                or t.shape[0] != self.n or not (1 <= t.shape[1] <= 64) or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape (n, s), 1 <= s <= 64")
        return t

    def spmm(self, X, Y=None):
        torch = _torch()
        self._as_block(X, "X")
        if Y is None:
            Y = torch.empty_like(X)
        self._as_block(Y, "Y")
        capi.check(self._lib.spmm(self.ctx, X.data_ptr(), Y.data_ptr(), X.shape[1]), self.ctx)
        return Y

    def cg_solve_multi(self, B, X, tol=1e-10, maxit=0) -> list:
        self._as_block(B, "B")
        self._as_block(X, "X")
        s = B.shape[1]
        infos = (capi.cg_info * s)()
        rc = self._lib.cg_solve_multi(self.ctx, B.data_ptr(), X.data_ptr(), s, float(tol), int(maxit), infos)
        capi.check(rc, self.ctx)
        return [infos[j].as_dict() for j in range(s)]

    def solve_multi(self, B, X0=None, tol=1e-10, maxit=0):
        torch = _torch()
        X = torch.zeros_like(B) if X0 is None else X0.clone()
        infos = self.cg_solve_multi(B, X, tol, maxit)
        return X, infos

    def cg_solve_block(self, B, X, tol=1e-10, maxit=0) -> list:
        """Block CG over the n x s block B (one shared Krylov space); X holds X0 and the solution."""
        self._as_block(B, "B")
        self._as_block(X, "X")
        s = B.shape[1]
        infos = (capi.cg_info * s)()
        rc = self._lib.cg_solve_block(self.ctx, B.data_ptr(), X.data_ptr(), s, float(tol), int(maxit), infos)
        capi.check(rc, self.ctx)
        return [infos[j].as_dict() for j in range(s)]

    def solve_block(self, B, X0=None, tol=1e-10, maxit=0):
        torch = _torch()
        X = torch.zeros_like(B) if X0 is None else X0.clone()
        infos = self.cg_solve_block(B, X, tol, maxit)
        return X, infos

    def cg_solve_multi_mixed(self, B, X, tol=1e-10, maxit_outer=0, tol_inner=0.0, maxit_inner=0) -> list:
        self._as_block(B, "B")
        self._as_block(X, "X")
        s = B.shape[1]
        infos = (capi.cg_info * s)()
        rc = self._lib.cg_solve_multi_mixed(self.ctx, B.data_ptr(), X.data_ptr(), s, float(tol), int(maxit_outer),
                                            float(tol_inner), int(maxit_inner), infos)
        capi.check(rc, self.ctx)
        return [infos[j].as_dict() for j in range(s)]

    def solve_multi_mixed(self, B, X0=None, tol=1e-10, maxit_outer=0, tol_inner=0.0, maxit_inner=0):
        torch = _torch()
        X = torch.zeros_like(B) if X0 is None else X0.clone()
        infos = self.cg_solve_multi_mixed(B, X, tol, maxit_outer, tol_inner, maxit_inner)
        return X, infos

    # -- introspection -------------------------------------------------------------
    def history(self) -> np.ndarray:
        cap = self.n + 1
        buf = np.empty(cap)
        m = capi.check(self._lib.cg_get_history(self.ctx, buf.ctypes.data, cap), self.ctx)
        return buf[:m].copy()

    def config(self) -> dict:
        c = capi.cg_config()
        capi.check(self._lib.cg_get_config(self.ctx, ctypes.byref(c)), self.ctx)
        return c.as_dict()


class Batch:
    """A cg_batch: many independent SPD CSR systems solved in one launch."""

    def __init__(self, systems, precond="jacobi", nnz_per_lane=0, blocks_per_cu=0, autotune=False, col_bits=0,
                 stream=None):
        torch = _torch()
        self._lib = capi.load()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.nsys = len(systems)
        arr = (capi.cg_csr * self.nsys)()
        self._keep = []
        for i, a in enumerate(systems):
            csr, keep = make_csr(a)
            if csr.mem != capi.CG_MEM_HOST:
                raise ValueError("batched systems must be host (numpy) CSR matrices")
            arr[i] = csr
            self._keep.append(keep)
        opts = make_opts(precond, autotune=autotune, nnz_per_lane=nnz_per_lane, blocks_per_cu=blocks_per_cu,
                         col_bits=col_bits)
        h = ctypes.c_void_p()
        rc = self._lib.cg_batch_create(self.nsys, arr, ctypes.byref(opts), ctypes.c_void_p(self.stream.cuda_stream),
                                       ctypes.byref(h))
        self._keep = None
        capi.check(rc)
        self.h = h
        self.offsets = [int(self._lib.cg_batch_offset(h, s)) for s in range(self.nsys + 1)]
        self.n_total = self.offsets[-1]

    def teams(self):
        t = (ctypes.c_int32 * self.nsys)()
        grid = self._lib.cg_batch_teams(self.h, t)
        return list(t), grid

    def cg_solve(self, b_cat, x_cat, tol=1e-10, maxit=0):
        _as_device_vec(b_cat, self.n_total, "b_cat")
        _as_device_vec(x_cat, self.n_total, "x_cat")
        infos = (capi.cg_info * self.nsys)()
        rc = self._lib.cg_batch_solve(self.h, b_cat.data_ptr(), x_cat.data_ptr(), float(tol), int(maxit), infos)
        if rc < 0:
            raise capi.CGError(rc, self._lib.cg_batch_last_error(self.h).decode())
        return [infos[s].as_dict() for s in range(self.nsys)]

    def solve(self, b_cat, x0=None, tol=1e-10, maxit=0):
        torch = _torch()
        x = torch.zeros_like(b_cat) if x0 is None else x0.clone()
        infos = self.cg_solve(b_cat, x, tol, maxit)
        return x, infos

    def close(self):
        if getattr(self, "h", None):
            self._lib.cg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -- structured Q1 operator from element coefficients (no CSR on the host) -----------------
def _q1_check(n_edge, sigma):
    torch = _torch()
    if n_edge < 2:
        raise ValueError("n_edge must be at least 2")
    if not isinstance(sigma, torch.Tensor) or not sigma.is_cuda or sigma.dtype != torch.float64 \
            or sigma.numel() != (n_edge - 1) ** 3 or not sigma.is_contiguous():
        raise ValueError("sigma must be a contiguous float64 CUDA tensor of (n_edge - 1)^3 element coefficients")


def q1_apply(n_edge, sigma, x, y=None, c=1e-3, stream=None):
    """y = A x for the Q1 operator of the element coefficients sigma, without forming A."""
    torch = _torch()
    _q1_check(n_edge, sigma)
    _as_device_vec(x, n_edge ** 3, "x")
    if y is None:
        y = torch.empty_like(x)
    _as_device_vec(y, n_edge ** 3, "y")
    st = stream if stream is not None else torch.cuda.current_stream()
    capi.check(capi.load().q1_apply(int(n_edge), float(c), sigma.data_ptr(), x.data_ptr(), y.data_ptr(),
                                    ctypes.c_void_p(st.cuda_stream)))
    return y


class DeviceCSR:
    """A CSR matrix in device memory (torch tensors), accepted by Solver."""

    def __init__(self, n, rowptr, col, val):
        self.n, self.rowptr, self.col, self.val = n, rowptr, col, val

    @property
    def nnz(self):
        return int(self.col.numel())


def q1_assemble(n_edge, sigma, c=1e-3, stream=None) -> DeviceCSR:
    """The Q1 operator of the element coefficients sigma, assembled in CSR on the device."""
    torch = _torch()
    _q1_check(n_edge, sigma)
    n = n_edge ** 3
    nnz = (3 * n_edge - 2) ** 3
    dev = sigma.device
    rowptr = torch.empty(n + 1, dtype=torch.int32, device=dev)
    col = torch.empty(nnz, dtype=torch.int32, device=dev)
    val = torch.empty(nnz, dtype=torch.float64, device=dev)
    st = stream if stream is not None else torch.cuda.current_stream()
    capi.check(capi.load().q1_assemble(int(n_edge), float(c), sigma.data_ptr(), rowptr.data_ptr(), col.data_ptr(),
                                       val.data_ptr(), ctypes.c_void_p(st.cuda_stream)))
    return DeviceCSR(n, rowptr, col, val)
