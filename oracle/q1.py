"""Q1 hexahedral operator oracle -- TEST INFRASTRUCTURE ONLY.

The paper's system comes from a finite-element model (Section IV); the
stand-in workload discretises -div(sigma grad u) + c u on the unit cube with
trilinear (Q1) hexahedra, n nodes per edge, spacing h = 1/(n-1), one
coefficient sigma_e per element.  This module applies that operator element
by element, as a finite-element code does without assembling: for every
element, gather its 8 nodal values, multiply by the 8 x 8 element matrix
sigma_e K_e + c M_e, and add the result into its 8 nodes.

The element matrices are built from the 1-D linear element on [0, h]:
    k1 = [[1, -1], [-1, 1]] / h,   m1 = h [[2, 1], [1, 2]] / 6,
    K_e = k1 (x) m1 (x) m1 + m1 (x) k1 (x) m1 + m1 (x) m1 (x) k1,
    M_e = m1 (x) m1 (x) m1,
with local node (bz, by, bx) in {0, 1}^3 at index 4 bz + 2 by + bx.  Plain
numpy FP64, vectorised over elements; shares nothing with the GPU library
(and nothing with the workload generator's entry tables either).
"""
from __future__ import annotations

import numpy as np


def element_matrices(h: float):
    """(K_e, M_e), each 8 x 8, for a cube of side h."""
    k1 = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    m1 = h * np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
    K = np.kron(np.kron(k1, m1), m1) + np.kron(np.kron(m1, k1), m1) + np.kron(np.kron(m1, m1), k1)
    M = np.kron(np.kron(m1, m1), m1)
    return K, M


def _element_nodes(n: int) -> np.ndarray:
    """((n-1)^3, 8) node ids of every element, local order 4 bz + 2 by + bx."""
    e = np.arange(n - 1)
    ez, ey, ex = np.meshgrid(e, e, e, indexing="ij")
    base = (ex + n * ey + n * n * ez).reshape(-1)
    local = np.array([bx + n * by + n * n * bz for bz in (0, 1) for by in (0, 1) for bx in (0, 1)])
    return base[:, None] + local[None, :]


def apply(n: int, sigma, c: float, x) -> np.ndarray:
    """y = A x for A = sum_e (sigma_e K_e + c M_e), summed element by element.

    sigma: (n-1, n-1, n-1) indexed [ez, ey, ex]; x: (n^3,) or (n^3, s).
    """
    h = 1.0 / (n - 1)
    K, M = element_matrices(h)
    nodes = _element_nodes(n)
    x = np.asarray(x, dtype=np.float64)
    X = x.reshape(x.shape[0], -1)                   # (N, s)
    sig = np.asarray(sigma, dtype=np.float64).reshape(-1)
    Xe = X[nodes]                                   # (E, 8, s): each element's nodal values
    Ye = sig[:, None, None] * np.einsum("ab,ebs->eas", K, Xe) + c * np.einsum("ab,ebs->eas", M, Xe)
    Y = np.zeros_like(X)
    np.add.at(Y, nodes.reshape(-1), Ye.reshape(-1, X.shape[1]))   # add into the element's nodes
    return Y.reshape(x.shape)


def diagonal(n: int, sigma, c: float) -> np.ndarray:
    """The diagonal of A, element by element."""
    h = 1.0 / (n - 1)
    K, M = element_matrices(h)
    nodes = _element_nodes(n)
    sig = np.asarray(sigma, dtype=np.float64).reshape(-1)
    d = np.zeros(n ** 3)
    np.add.at(d, nodes.reshape(-1), (sig[:, None] * np.diag(K)[None, :] + c * np.diag(M)[None, :]).reshape(-1))
    return d


def abs_row_bound(n: int, sigma, c: float, x) -> np.ndarray:
    """sum_e sum_b |sigma_e K_e[a, b] + c M_e[a, b]| |x_b| at every node: an upper
    bound of sum_j |a_ij x_j| (the scale of row i's rounding), element by element."""
    h = 1.0 / (n - 1)
    K, M = element_matrices(h)
    nodes = _element_nodes(n)
    ax = np.abs(np.asarray(x, dtype=np.float64))
    sig = np.asarray(sigma, dtype=np.float64).reshape(-1)
    Ae = np.abs(sig[:, None, None] * K[None] + c * M[None])       # (E, 8, 8)
    ye = np.einsum("eab,eb->ea", Ae, ax[nodes])
    y = np.zeros(n ** 3)
    np.add.at(y, nodes.reshape(-1), ye.reshape(-1))
    return y
