"""Block conjugate-gradient oracle for several right-hand sides -- TEST INFRASTRUCTURE ONLY.

Solves A X = B for an SPD matrix A (CSR) and s right-hand sides at once with
O'Leary's block conjugate-gradient method (Linear Algebra Appl. 29, 1980),
the paper's conjugate-gradient iteration (Section IV) applied to a block of
vectors: one block product A P per iteration, s x s matrices in place of the
scalars alpha and beta, and a Krylov space that grows by up to s directions
per iteration.  Plain numpy FP64; the sparse product is the C oracle's
sequential row sum, one column at a time.  Shares nothing with the GPU
library.

Rank deficiency: as the columns converge the search block becomes nearly
linearly dependent and P'AP singular.  The breakdown-free form of Ji and Li
(BIT Numer. Math. 57, 2017) avoids this by orthonormalising every new search
block with rank revelation, so that dependent directions are dropped:

    R = B - A X;  Z = M^-1 R;  P = orth(Z)
    loop:  Q = A P
           alpha = (P'Q)^-1 (P'R);   X += P alpha;   R -= Q alpha
           stop when every column passes ||r_j|| <= tol ||b_j||, confirmed on
           the true residuals B - A X (if a column fails, R is replaced by the
           true residuals and the block restarts from P = orth(M^-1 R))
           Z = M^-1 R
           beta = -(P'Q)^-1 (Q'Z);   P = orth(Z + P beta)

orth(W) is the shifted Cholesky QR of Fukaya, Kannan, Nakatsukasa, Zhang and
Yamamoto (SIAM J. Sci. Comput. 42, 2020): CholeskyQR with a shift of
11 (N s + s (s + 1)) u ||W||^2 on the Gram matrix, then CholeskyQR twice
more, which gives an orthonormal basis for condition numbers up to ~1/u
(these blocks reach 1e9, beyond plain or repeated CholeskyQR).  Here the
columns are scaled to unit norm first (so the decisions do not depend on the
columns' scales), and the second and third factorisations drop every column
whose pivot is <= tau: a direction whose remaining pivot is that small after the
first, shifted pass is dependent on the ones already taken.  Each pass forms
its block explicitly (W_k = W_{k-1} T_k, T_k the inverse transposed factor),
as the method requires.  Kept columns stay in place and dropped ones become
zero columns; the live columns of P form the basis.

Iterations count block products A P in the loop (as in the single-vector
oracle).  Statuses: CONVERGED, MAXIT, BREAKDOWN (P'Q not positive definite,
or a non-finite value).
"""
from __future__ import annotations

import numpy as np

from . import BREAKDOWN, CONVERGED, MAXIT, spmv

UNIT_ROUNDOFF = 2.0 ** -53
TAU = 1e-14


def spmm(a, X):
    """A X, each column the oracle's sequential CSR product."""
    X = np.asarray(X, dtype=np.float64)
    return np.stack([spmv(a, np.ascontiguousarray(X[:, j])) for j in range(X.shape[1])], axis=1)


def cholesky_drop(G, tau):
    """Cholesky factorisation of a symmetric PSD matrix G (s x s) that drops
    dependent columns.

    Columns are taken in order; column k's pivot is its remaining diagonal
    entry after the kept columns before it (the squared distance of column k
    from their span, for a Gram matrix).  A pivot <= tau drops column k:
    its column of L is zero and it takes no part in later updates.  Returns
    (L, keep): L lower triangular with G[keep][:, keep] = L_kk L_kk', where
    L_kk is L restricted to the kept rows and columns.
    """
    s = G.shape[0]
    A = np.array(G, dtype=np.float64, copy=True)
    L = np.zeros((s, s))
    keep = np.zeros(s, dtype=bool)
    for k in range(s):
        d = A[k, k]
        if not (d > tau):
            continue
        keep[k] = True
        L[k, k] = np.sqrt(d)
        L[k + 1:, k] = A[k + 1:, k] / L[k, k]
        A[k + 1:, k + 1:] -= np.outer(L[k + 1:, k], L[k + 1:, k])
    return L, keep


def _inverse_factor(L, keep):
    """T (s x s) = L_kk^-T placed at the kept rows and columns, zero elsewhere:
    W T holds W[:, keep] L_kk^-T in the kept columns and zero in the others."""
    s = L.shape[0]
    T = np.zeros((s, s))
    idx = np.flatnonzero(keep)
    if idx.size:
        T[np.ix_(idx, idx)] = np.linalg.solve(L[np.ix_(idx, idx)], np.eye(idx.size)).T
    return T


def orth(W, tau=TAU):
    """(P, keep): an orthonormal basis of the numerical column span of W (N x s),
    in the kept columns of P (the others are zero).

    Three CholeskyQR passes, each W_k = W_{k-1} T_k with T_k from the
    Cholesky factor of the Gram matrix of W_{k-1}; the first on the
    column-scaled W with the shift, the other two dropping columns at tau.
    """
    W = np.asarray(W, dtype=np.float64)
    n, s = W.shape
    d = np.einsum("ij,ij->j", W, W)
    D = np.where(d > 0.0, 1.0 / np.sqrt(np.where(d > 0.0, d, 1.0)), 0.0)
    W0 = W * D
    G = W0.T @ W0
    shift = 11.0 * (n * s + s * (s + 1)) * UNIT_ROUNDOFF * np.trace(G)
    L, keep = cholesky_drop(G + shift * np.eye(s), 0.0)
    Wk = W0 @ _inverse_factor(L, keep)
    for _ in range(2):
        L, keep = cholesky_drop(Wk.T @ Wk, tau)
        Wk = Wk @ _inverse_factor(L, keep)
    return Wk, keep


def _spd_solve(gamma, live, rhs):
    """gamma[live][:, live]^-1 rhs[live] at the live rows, zero rows elsewhere
    (Cholesky); None if that block is not positive definite."""
    out = np.zeros_like(rhs)
    idx = np.flatnonzero(live)
    if idx.size == 0:
        return out
    G = gamma[np.ix_(idx, idx)]
    try:
        C = np.linalg.cholesky(0.5 * (G + G.T))
    except np.linalg.LinAlgError:
        return None
    out[idx] = np.linalg.solve(C.T, np.linalg.solve(C, rhs[idx]))
    return out


def block_pcg(a, B, X0=None, tol=1e-10, maxit=0, precond="jacobi", tau=TAU, history=False):
    """Breakdown-free block Jacobi-PCG.  Returns (X, info[, hist]).

    info: iters (block products in the loop), status, replacements (restarts
    from the true residual), relres_true (per column, of the returned X),
    ranks (search-block rank per iteration).  hist[k] = max_j ||r_j|| / ||b_j||
    of the recurrence after k iterations.
    """
    B = np.asarray(B, dtype=np.float64)
    n, s = B.shape
    X = np.zeros_like(B) if X0 is None else np.array(X0, dtype=np.float64, copy=True)
    dinv = np.ones(n)
    if precond == "jacobi":
        rows = np.repeat(np.arange(n), np.diff(a.rowptr))
        on_diag = np.asarray(a.col) == rows
        d = np.bincount(rows[on_diag], weights=np.asarray(a.val)[on_diag], minlength=n)
        present = np.bincount(rows[on_diag], minlength=n) > 0
        if not np.all(present & (d > 0.0)):
            raise ValueError("Jacobi needs every diagonal entry present and positive")
        dinv = 1.0 / d
    maxit = n if maxit <= 0 else maxit
    nb = np.linalg.norm(B, axis=0)
    zero = nb == 0.0
    X[:, zero] = 0.0
    thr = tol * nb

    def passed(R):
        return bool(np.all(np.linalg.norm(R, axis=0) <= thr))

    def finish(status, k, repl, ranks, hist):
        rt = np.linalg.norm(B - spmm(a, X), axis=0)
        info = {"iters": k, "status": status, "replacements": repl, "ranks": ranks,
                "relres_true": np.where(zero, 0.0, rt / np.where(zero, 1.0, nb))}
        return (X, info, np.array(hist)) if history else (X, info)

    R = B - spmm(a, X)
    hist = [float(np.max(np.linalg.norm(R, axis=0)[~zero] / nb[~zero])) if np.any(~zero) else 0.0]
    if passed(R):
        return finish(CONVERGED, 0, 0, [], hist)
    if not np.all(np.isfinite(R)):
        return finish(BREAKDOWN, 0, 0, [], hist)
    Z = dinv[:, None] * R
    P, live = orth(Z, tau)
    ranks = [int(live.sum())]
    k = repl = 0
    status = MAXIT
    while k < maxit:
        Q = spmm(a, P)
        PQ = P.T @ Q
        alpha = _spd_solve(PQ, live, P.T @ R)
        if alpha is None or not np.all(np.isfinite(alpha)):
            status = BREAKDOWN
            break
        X += P @ alpha
        R -= Q @ alpha
        k += 1
        hist.append(float(np.max(np.linalg.norm(R, axis=0)[~zero] / nb[~zero])))
        if not np.all(np.isfinite(R)):
            status = BREAKDOWN
            break
        if passed(R):
            Rt = B - spmm(a, X)
            if passed(Rt):
                status = CONVERGED
                break
            R = Rt
            repl += 1
            Z = dinv[:, None] * R
            P, live = orth(Z, tau)
            ranks.append(int(live.sum()))
            continue
        Z = dinv[:, None] * R
        beta = _spd_solve(PQ, live, Q.T @ Z)
        if beta is None:
            status = BREAKDOWN
            break
        beta = -beta
        P, live = orth(Z + P @ beta, tau)
        ranks.append(int(live.sum()))
        if not live.any():
            status = BREAKDOWN
            break
    return finish(status, k, repl, ranks, hist)
