"""Learned warm start: POD basis of past solutions + a small MLP that maps
source parameters to POD coefficients, so that CG starts from x0 = Phi c_hat.

Python binds the HIP calls (dense_gram, dense_gemm, pod_decode, mlp_*); the
dense products, the network's forward/backward/Adam and every CG solve run in
the library.  The host does the small set-up arithmetic only: the eigen-
decomposition of the m x m snapshot Gram matrix (m = 500), the per-mode
standardisation statistics of 2000 x 64 coefficients, and the input map
theta -> 2 theta - 1 of the network's 24 inputs per sample (the output
de-standardisation is applied in FP64 by the decode kernel).
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import capi


def _torch():
    import torch

    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_dev(t, dtype, name, ndim=2):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or t.dim() != ndim:
        raise ValueError(f"{name} must be a {ndim}-D {dtype} CUDA tensor")
    if t.stride(-1) != 1:
        raise ValueError(f"{name} must have unit stride in its last dimension")
    return t


# -- dense products ------------------------------------------------------------------------------
def dense_gram(A, B=None, stream=None):
    """C = A' B for device FP64 row-major blocks A (n x ka), B (n x kb); deterministic."""
    torch = _torch()
    B = A if B is None else B
    _check_dev(A, torch.float64, "A")
    _check_dev(B, torch.float64, "B")
    if A.shape[0] != B.shape[0]:
        raise ValueError("A and B must have the same number of rows")
    C = torch.empty((A.shape[1], B.shape[1]), dtype=torch.float64, device=A.device)
    capi.check(capi.load().dense_gram(A.data_ptr(), A.shape[0], A.shape[1], A.stride(0), B.data_ptr(),
                                      B.shape[1], B.stride(0), C.data_ptr(), _stream_ptr(stream)))
    return C


def dense_gemm(A, W, stream=None):
    """C = A W for a device FP64 block A (n x k) and a small row-major W (k x m)."""
    torch = _torch()
    _check_dev(A, torch.float64, "A")
    _check_dev(W, torch.float64, "W")
    W = W.contiguous()
    if W.shape[0] != A.shape[1]:
        raise ValueError("W must have as many rows as A has columns")
    C = torch.empty((A.shape[0], W.shape[1]), dtype=torch.float64, device=A.device)
    capi.check(capi.load().dense_gemm(A.data_ptr(), A.shape[0], A.shape[1], A.stride(0), W.data_ptr(), W.shape[1],
                                      C.data_ptr(), W.shape[1], _stream_ptr(stream)))
    return C


def pod_decode(Phi, coef, out=None, scale=None, shift=None, stream=None):
    """X (n x nb) = Phi c' with c = scale * coef + shift (per mode, FP64) for FP32 coef (nb x k)."""
    torch = _torch()
    _check_dev(Phi, torch.float64, "Phi")
    _check_dev(coef, torch.float32, "coef")
    coef = coef.contiguous()
    n, k = Phi.shape
    nb = coef.shape[0]
    if coef.shape[1] != k:
        raise ValueError("coef must have as many columns as Phi")
    if out is None:
        out = torch.empty((n, nb), dtype=torch.float64, device=Phi.device)
    if out.dtype != torch.float64 or out.numel() != n * nb or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor with n * nb entries")
    ptrs = []
    for v in (scale, shift):
        if v is None:
            ptrs.append(None)
        else:
            _check_dev(v, torch.float64, "scale/shift", ndim=1)
            if v.numel() != k:
                raise ValueError("scale and shift must have k entries")
            ptrs.append(v.data_ptr())
    capi.check(capi.load().pod_decode(Phi.data_ptr(), n, k, Phi.stride(0), coef.data_ptr(), nb, ptrs[0], ptrs[1],
                                      out.data_ptr(), _stream_ptr(stream)))
    return out


# -- the network ---------------------------------------------------------------------------------
def he_uniform(dims, seed=0):
    """Flat FP32 parameters (per layer W row-major, then b) with He-style uniform weights."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in zip(dims[:-1], dims[1:]):
        bound = np.sqrt(6.0 / fan_in) / 2.0
        parts.append(rng.uniform(-bound, bound, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def layer_views(flat, dims):
    """(W, b) views into a flat parameter vector."""
    out, o = [], 0
    for fan_in, fan_out in zip(dims[:-1], dims[1:]):
        W = flat[o:o + fan_in * fan_out].reshape(fan_out, fan_in)
        o += fan_in * fan_out
        b = flat[o:o + fan_out]
        o += fan_out
        out.append((W, b))
    return out


class MLP:
    """An mlp_net: SiLU hidden layers, linear output, MSE loss, Adam; FP32 or BF16."""

    PRECISIONS = {"fp32": 0, "bf16": 1}

    def __init__(self, dims, precision="bf16", max_batch=2048, stream=None):
        torch = _torch()
        self._lib = capi.load()
        self.dims = [int(d) for d in dims]
        self.precision = precision
        self.max_batch = int(max_batch)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        arr = (ctypes.c_int32 * len(self.dims))(*self.dims)
        h = ctypes.c_void_p()
        capi.check(self._lib.mlp_create(len(self.dims) - 1, arr, self.PRECISIONS[precision], self.max_batch,
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.nparam = int(self._lib.mlp_param_count(h))

    def close(self):
        if getattr(self, "h", None):
            self._lib.mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        if flat.size != self.nparam:
            raise ValueError(f"expected {self.nparam} parameters")
        capi.check(self._lib.mlp_set_params(self.h, flat.ctypes.data))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.nparam, np.float32)
        capi.check(self._lib.mlp_get_params(self.h, out.ctypes.data))
        return out

    def _batch(self, X, width, name):
        torch = _torch()
        if not isinstance(X, torch.Tensor) or not X.is_cuda or X.dtype != torch.float32 or X.dim() != 2 \
                or X.shape[1] != width or not X.is_contiguous() or not (1 <= X.shape[0] <= self.max_batch):
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor (batch <= {self.max_batch}, {width})")
        return X

    def forward(self, X, Y=None):
        torch = _torch()
        self._batch(X, self.dims[0], "X")
        if Y is None:
            Y = torch.empty((X.shape[0], self.dims[-1]), dtype=torch.float32, device=X.device)
        self._batch(Y, self.dims[-1], "Y")
        capi.check(self._lib.mlp_forward(self.h, X.data_ptr(), X.shape[0], Y.data_ptr()))
        return Y

    def gradients(self, X, T):
        self._batch(X, self.dims[0], "X")
        self._batch(T, self.dims[-1], "T")
        g = np.empty(self.nparam, np.float32)
        loss = ctypes.c_double()
        capi.check(self._lib.mlp_gradients(self.h, X.data_ptr(), T.data_ptr(), X.shape[0], g.ctypes.data,
                                           ctypes.byref(loss)))
        return g, loss.value

    def train_step(self, X, T, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, want_loss=False):
        self._batch(X, self.dims[0], "X")
        self._batch(T, self.dims[-1], "T")
        loss = ctypes.c_double()
        capi.check(self._lib.mlp_train_step(self.h, X.data_ptr(), T.data_ptr(), X.shape[0], float(lr), float(beta1),
                                            float(beta2), float(eps), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None


# -- the pipeline --------------------------------------------------------------------------------
class LearnedWarmStart:
    """Snapshots -> POD basis -> MLP(theta) -> coefficients -> x0 = Phi c.

    solver: a Solver on the system matrix; family: an object with rhs(idx)
    ((len, N) host array) and theta() ((count, d) host array).  Index ranges:
    [0, n_pod) build the basis and train, [n_pod, n_train) train only,
    [n_train, count) are held out.
    """

    def __init__(self, solver, family, n_pod=500, n_train=1500, modes=64, hidden=(256, 256), precision="bf16",
                 seed=0):
        self.solver = solver
        self.family = family
        self.n_pod, self.n_train, self.k = int(n_pod), int(n_train), int(modes)
        if not (self.k <= self.n_pod <= self.n_train <= family.count):
            raise ValueError("need modes <= n_pod <= n_train <= count")
        self.hidden = tuple(int(h) for h in hidden)
        self.precision = precision
        self.seed = seed
        self.theta = np.ascontiguousarray(family.theta(), dtype=np.float64)
        self.timings = {}
        self.Phi = None
        self.net = None

    # snapshots: solve each training right-hand side with the multi-RHS solver
    def snapshots(self, idx, tol=1e-10, block=64, maxit=0, log=None):
        """Device (N x len(idx)) block of solutions, and the per-solve infos."""
        torch = _torch()
        dev = torch.device("cuda", torch.cuda.current_device())
        idx = np.asarray(idx)
        S = torch.empty((self.solver.n, len(idx)), dtype=torch.float64, device=dev)
        infos = []
        for j0 in range(0, len(idx), block):
            sel = idx[j0:j0 + block]
            B = torch.as_tensor(np.ascontiguousarray(self.family.rhs(sel).T), device=dev)
            X, inf = self.solver.solve_multi(B, tol=tol, maxit=maxit)
            if log:
                log(f"snapshots {j0 + len(sel)}/{len(idx)}: max iterations {max(i['iters'] for i in inf)}")
            bad = [j0 + j for j, i in enumerate(inf) if i["status"] != capi.CG_CONVERGED]
            if bad:
                raise RuntimeError(f"snapshot solves did not converge for columns {bad[:8]}")
            S[:, j0:j0 + len(sel)].copy_(X)
            infos += inf
        return S, infos

    def build_basis(self, S):
        """Phi (N x k) from the first n_pod snapshot columns (method of snapshots)."""
        torch = _torch()
        Sp = S[:, :self.n_pod]
        G = dense_gram(Sp).cpu().numpy()
        lam, V = np.linalg.eigh(0.5 * (G + G.T))
        order = np.argsort(lam)[::-1][:self.k]
        lam, V = lam[order], V[:, order]
        if lam[-1] <= 0:
            raise ValueError("snapshot Gram matrix has fewer than k positive eigenvalues")
        self.energy = lam
        Wm = torch.as_tensor(np.ascontiguousarray(V / np.sqrt(lam)), device=S.device)
        self.Phi = dense_gemm(Sp, Wm)
        return self.Phi

    def coefficients(self, S):
        """(columns of S) x k matrix of POD coefficients Phi' S, on the host."""
        return dense_gram(self.Phi, S).cpu().numpy().T.copy()

    def fit(self, epochs=300, batch=256, lr=1e-3, log_every=0, tol=1e-10, maxit=0, log=None):
        """Generate the snapshots (CG to tol), build the basis and train the network."""
        torch = _torch()
        dev = torch.device("cuda", torch.cuda.current_device())
        t0 = time.perf_counter()
        S, infos = self.snapshots(np.arange(self.n_train), tol=tol, maxit=maxit, log=log)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        self.build_basis(S)
        C = self.coefficients(S)
        del S
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        # standardise targets per mode and map inputs to [-1, 1]
        self.mu = C.mean(0)
        self.sigma = C.std(0) + 1e-300
        T = ((C - self.mu) / self.sigma).astype(np.float32)
        Xin = self.inputs(self.theta[:self.n_train])
        dims = [Xin.shape[1], *self.hidden, self.k]
        self.net = MLP(dims, self.precision, max_batch=max(batch, 1))
        self.net.set_params(he_uniform(dims, self.seed))
        rng = np.random.default_rng(self.seed + 1)
        nb = self.n_train // batch
        self.loss_curve = []
        for ep in range(epochs):
            perm = rng.permutation(self.n_train)[:nb * batch]
            Xd = torch.as_tensor(Xin[perm], device=dev)
            Td = torch.as_tensor(T[perm], device=dev)
            last = ep == epochs - 1 or (log_every and ep % log_every == 0)
            for i in range(nb):
                want = last and i == nb - 1
                loss = self.net.train_step(Xd[i * batch:(i + 1) * batch], Td[i * batch:(i + 1) * batch], lr=lr,
                                           want_loss=want)
                if want:
                    self.loss_curve.append((ep, loss))
                    if log:
                        log(f"epoch {ep}: loss {loss:.3e}")
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        self._finish()
        self.timings = {"snapshots_s": t1 - t0, "pod_s": t2 - t1, "train_s": t3 - t2,
                        "snapshot_iters_mean": float(np.mean([i["iters"] for i in infos]))}
        return self

    def _finish(self):
        """The output de-standardisation is applied in FP64 by the decode."""
        torch = _torch()
        self.scale = torch.as_tensor(self.sigma, dtype=torch.float64, device=self.Phi.device)
        self.shift = torch.as_tensor(self.mu, dtype=torch.float64, device=self.Phi.device)

    @staticmethod
    def inputs(theta_rows):
        """Network inputs: theta -> 2 theta - 1 in FP32, exactly as in training (in BF16 mode the
        forward pass rounds these to BF16, as the training steps did)."""
        return (2.0 * np.asarray(theta_rows, dtype=np.float64) - 1.0).astype(np.float32)

    def predict(self, theta_rows):
        """Standardised FP32 coefficients (len x k) on the device for host theta rows."""
        torch = _torch()
        X = torch.as_tensor(np.ascontiguousarray(self.inputs(theta_rows)), device=self.Phi.device)
        return self.net.forward(X)

    def x0(self, theta_rows, out=None):
        """Device start vector(s) (N x len) = Phi MLP(theta)."""
        return pod_decode(self.Phi, self.predict(theta_rows), out, self.scale, self.shift)
