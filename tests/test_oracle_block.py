"""Pins for the block conjugate-gradient oracle (O'Leary's block CG in the
breakdown-free form, search blocks orthonormalised by shifted Cholesky QR),
against things other than itself:
  - one right-hand side: the block iteration is the single-vector PCG
    iteration (the oracle's C code) up to rounding, iterate by iterate;
  - dense Cholesky solves of small systems (LAPACK via scipy);
  - finite termination: the block Krylov space grows by s directions per
    iteration, so an N x N system is solved in about N / s iterations;
  - block conjugacy P_i' A P_j = 0 and residual orthogonality R_k' P_j = 0;
  - rank deficiency: duplicate, zero and dependent right-hand sides;
  - the building blocks: pivoted Cholesky against the matrix it factors, and
    orth() against the singular values and span of an input of known
    conditioning.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import oracle.block_cg as bc
import workloads as W


def dense_csr(d):
    n = d.shape[0]
    rowptr, col, val = [0], [], []
    for i in range(n):
        nz = np.nonzero(d[i])[0]
        col.extend(nz.tolist())
        val.extend(d[i, nz].tolist())
        rowptr.append(len(col))
    return W.CSR(n, np.array(rowptr, np.int32), np.array(col, np.int32), np.array(val, np.float64))


def spd(n, cond, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.geomspace(1.0, cond, n)
    return (Q * lam) @ Q.T


def test_cholesky_drop_factors_the_kept_columns():
    rng = np.random.default_rng(0)
    for s, rank in [(6, 6), (9, 4), (64, 64), (64, 17)]:
        F = rng.standard_normal((s, rank)) * np.geomspace(1.0, 1e-3, rank)
        G = F @ F.T
        L, keep = bc.cholesky_drop(G, 1e-12 * np.max(np.diag(G)))
        assert int(keep.sum()) == rank
        idx = np.flatnonzero(keep)
        Lk = L[np.ix_(idx, idx)]
        assert np.max(np.abs(Lk @ Lk.T - G[np.ix_(idx, idx)])) <= 1e-12 * np.max(np.abs(G))
        assert np.allclose(L, np.tril(L))
        assert not L[:, ~keep].any()
        # Columns are taken greedily in order: the first `rank` columns of a
        # random rank-`rank` Gram matrix are independent, the rest dependent.
        assert np.array_equal(idx, np.arange(rank))
    # A zero column and a repeated column are dropped where they occur.
    F = rng.standard_normal((5, 8))
    Wm = np.concatenate([F[:, :2], np.zeros((5, 1)), F[:, :1], F[:, 2:4]], axis=1)
    L, keep = bc.cholesky_drop(Wm.T @ Wm, 1e-12)
    assert keep.tolist() == [True, True, False, False, True, True]
    # The matrix of a full-rank Gram factorisation is the textbook Cholesky factor.
    G = F.T @ F + np.eye(8)
    L, keep = bc.cholesky_drop(G, 0.0)
    assert keep.all() and np.allclose(L, np.linalg.cholesky(G), rtol=1e-13, atol=1e-13)


def test_orth_ill_conditioned_and_rank_deficient():
    rng = np.random.default_rng(1)
    n, s = 3000, 16
    U, _ = np.linalg.qr(rng.standard_normal((n, s)))
    V, _ = np.linalg.qr(rng.standard_normal((s, s)))
    for cond in (1e2, 1e9, 1e12):
        Wm = (U * np.geomspace(1.0, 1.0 / cond, s)) @ V.T * 7.0
        P, keep = bc.orth(Wm)
        assert keep.all()
        assert np.max(np.abs(P.T @ P - np.eye(s))) <= 1e-12
        # Same span: W is reproduced from its coefficients in P.
        assert np.linalg.norm(Wm - P @ (P.T @ Wm)) <= 1e-10 * np.linalg.norm(Wm)
    # Rank 5: 11 columns are combinations of the first 5; one zero column.
    F = rng.standard_normal((n, 5))
    Wm = np.concatenate([F, F @ rng.standard_normal((5, 10)), np.zeros((n, 1))], axis=1)
    P, keep = bc.orth(Wm)
    assert keep.tolist() == [True] * 5 + [False] * 11
    assert np.max(np.abs(P[:, keep].T @ P[:, keep] - np.eye(5))) <= 1e-12
    assert not P[:, ~keep].any()
    assert np.linalg.norm(Wm - P @ (P.T @ Wm)) <= 1e-10 * np.linalg.norm(Wm)
    # Column scales do not change the decision: an independent direction held
    # only by a column 1e-18 times smaller than the others is kept.
    P2, keep2 = bc.orth(Wm * np.geomspace(1e-8, 1e8, Wm.shape[1]))
    assert int(keep2.sum()) == 5
    g = rng.standard_normal((n, 1))
    P3, keep3 = bc.orth(np.concatenate([F * 1e8, g * 1e-10], axis=1))
    assert keep3.all()
    assert np.linalg.norm(g - P3 @ (P3.T @ g)) <= 1e-10 * np.linalg.norm(g)


@pytest.mark.parametrize("precond", ["jacobi", "none"])
def test_one_column_is_the_single_vector_iteration(precond):
    a, b = W.problem(8, 3)
    for k in (1, 2, 5, 12):
        xb, ib = bc.block_pcg(a, b[:, None], tol=1e-10, maxit=k, precond=precond)
        xs, is_ = oracle.pcg(a, b, tol=1e-10, maxit=k, precond=precond)
        assert ib["iters"] == is_["iters"] == k
        assert np.linalg.norm(xb[:, 0] - xs) <= 1e-9 * np.linalg.norm(xs)
    xb, ib = bc.block_pcg(a, b[:, None], tol=1e-10, precond=precond)
    xs, is_ = oracle.pcg(a, b, tol=1e-10, precond=precond)
    assert ib["status"] == is_["status"] == oracle.CONVERGED
    assert abs(ib["iters"] - is_["iters"]) <= 2


@pytest.mark.parametrize("n,s,cond", [(12, 3, 1e3), (40, 5, 1e4), (30, 8, 1e2)])
def test_matches_cholesky(n, s, cond):
    d = spd(n, cond, n + s)
    a = dense_csr(d)
    B = np.random.default_rng(n).standard_normal((n, s))
    X, info = bc.block_pcg(a, B, tol=1e-10, precond="none")
    assert info["status"] == oracle.CONVERGED
    Xc = sla.cho_solve(sla.cho_factor(d), B)
    for j in range(s):
        assert np.linalg.norm(X[:, j] - Xc[:, j]) <= cond * 1e-10 * np.linalg.norm(Xc[:, j]) * 10
    assert np.all(info["relres_true"] <= 1e-10)


def test_finite_termination():
    # 48 x 48 with 8 right-hand sides: 6 blocks span R^48.
    n, s = 48, 8
    a = dense_csr(spd(n, 10.0, 2))
    B = np.random.default_rng(3).standard_normal((n, s))
    X, info = bc.block_pcg(a, B, tol=1e-12, precond="none")
    assert info["status"] == oracle.CONVERGED
    assert info["iters"] <= n // s + 1
    # One right-hand side needs about n iterations of the same matrix.
    _, i1 = oracle.pcg(a, B[:, 0], tol=1e-12, precond="none")
    assert i1["iters"] > 2 * info["iters"]


def test_block_conjugacy_and_residual_orthogonality():
    # Traced by running k iterations for k = 1..5 (the iterates of a k-step
    # run are those of the longer run): consecutive search blocks are
    # A-conjugate and each residual is orthogonal to the previous blocks.
    n, s = 60, 4
    d = spd(n, 50.0, 4)
    a = dense_csr(d)
    B = np.random.default_rng(5).standard_normal((n, s))
    Xs = [np.zeros((n, s))] + [bc.block_pcg(a, B, tol=1e-14, maxit=k, precond="none")[0] for k in range(1, 6)]
    dirs = [Xs[k + 1] - Xs[k] for k in range(5)]  # P_k alpha_k: spans the k-th search block
    for i in range(5):
        for j in range(i):
            assert np.linalg.norm(dirs[i].T @ d @ dirs[j]) <= 1e-8 * np.linalg.norm(dirs[i]) * np.linalg.norm(
                d @ dirs[j])
    for k in range(1, 6):
        Rk = B - d @ Xs[k]
        for j in range(k):
            assert np.linalg.norm(Rk.T @ dirs[j]) <= 1e-8 * np.linalg.norm(Rk) * np.linalg.norm(dirs[j])


def test_fewer_block_iterations_than_single_on_the_fem_system():
    a, _ = W.problem(12, 0)
    B = W.multi_rhs(a.n, 8)
    X, info = bc.block_pcg(a, B, tol=1e-10)
    assert info["status"] == oracle.CONVERGED
    singles = [oracle.pcg(a, B[:, j], tol=1e-10)[1]["iters"] for j in range(8)]
    assert info["iters"] < min(singles)
    assert np.all(info["relres_true"] <= 1e-10)
    for j in range(8):
        xo, _ = oracle.pcg(a, B[:, j], tol=1e-10)
        assert np.linalg.norm(X[:, j] - xo) <= 1e-8 * np.linalg.norm(xo)


def test_rank_deficient_right_hand_sides():
    a, _ = W.problem(10, 1)
    rng = np.random.default_rng(6)
    F = W.multi_rhs(a.n, 3, seed=7)
    B = np.concatenate([F, F[:, :1], np.zeros((a.n, 1)), F @ rng.standard_normal((3, 3))], axis=1)
    X, info = bc.block_pcg(a, B, tol=1e-10)
    assert info["status"] == oracle.CONVERGED
    assert np.all(info["relres_true"] <= 1e-10)
    # The block has rank 3 in exact arithmetic; rounding noise in the
    # converging residuals adds directions only near convergence, and never
    # more than the 6 non-zero columns.
    assert info["ranks"][:20] == [3] * 20 and max(info["ranks"]) <= 6
    assert not X[:, 4].any()
    assert np.linalg.norm(X[:, 3] - X[:, 0]) <= 1e-8 * np.linalg.norm(X[:, 0])


def test_degenerate_inputs():
    a, b = W.problem(6, 2)
    B = np.stack([b, -b, 2 * b], axis=1)
    X, info = bc.block_pcg(a, np.zeros_like(B))
    assert info["status"] == oracle.CONVERGED and info["iters"] == 0 and not X.any()
    Xs, _ = bc.block_pcg(a, B, tol=1e-12)
    _, info = bc.block_pcg(a, B, X0=Xs, tol=1e-10)
    assert info["status"] == oracle.CONVERGED and info["iters"] == 0
    Bn = B.copy()
    Bn[3, 1] = np.nan
    _, info = bc.block_pcg(a, Bn)
    assert info["status"] == oracle.BREAKDOWN
    d = a.to_dense()
    d[0, 0] = -d[0, 0]
    _, info = bc.block_pcg(dense_csr(d), B, precond="none")
    assert info["status"] == oracle.BREAKDOWN
    _, info = bc.block_pcg(a, B, tol=1e-10, maxit=2)
    assert info["status"] == oracle.MAXIT and info["iters"] == 2
