"""Proper orthogonal decomposition oracle -- TEST INFRASTRUCTURE ONLY.

Method of snapshots (Sirovich, 1987): for snapshots S (N x m, one solution
per column), the Gram matrix C = S'S has eigenpairs (lambda_i, v_i) and the
POD modes are phi_i = S v_i / sqrt(lambda_i), orthonormal, ordered by
decreasing lambda_i (the captured energy).  Uncentred: the mean stays in the
modes.  Plain numpy FP64; shares nothing with the GPU library.
"""
from __future__ import annotations

import numpy as np


def gram(S):
    """C = S' S."""
    S = np.asarray(S, dtype=np.float64)
    return S.T @ S


def modes(S, k):
    """(Phi (N x k), lambda (all eigenvalues, descending))."""
    C = gram(S)
    lam, V = np.linalg.eigh(C)
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order]
    Phi = S @ V[:, :k] / np.sqrt(lam[:k])
    return Phi, lam


def project(Phi, X):
    """Coefficients C = Phi' X."""
    return Phi.T @ X


def decode(Phi, C):
    """X = Phi C."""
    return Phi @ C
