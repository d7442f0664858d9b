"""Pins for the FP64 conjugate-gradient oracle, against things other than itself.

The method is the conjugate-gradient iteration for SPD systems (Section IV,
after Golub and Van Loan) with tolerance 1e-10 (Table I caption).  Each pin
below comes from the mathematics of CG or from a library routine solving the
same special case:
  - dense Cholesky solves of the same systems (LAPACK via scipy);
  - residual orthogonality r_i' M^-1 r_j = 0 and A-conjugacy p_i' A p_j = 0;
  - monotone decrease of the A-norm error and the Chebyshev bound;
  - finite termination: k distinct eigenvalues => at most k iterations;
  - degenerate inputs: b = 0, x0 = x*, maxit = 1, indefinite A, NaN input.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import workloads as W


def dense_csr(a_dense):
    n = a_dense.shape[0]
    rowptr, col, val = [0], [], []
    for i in range(n):
        nz = np.nonzero(a_dense[i])[0]
        col.extend(nz.tolist())
        val.extend(a_dense[i, nz].tolist())
        rowptr.append(len(col))
    return W.CSR(n, np.array(rowptr, np.int32), np.array(col, np.int32), np.array(val, np.float64))


def test_spmv_brute_force():
    rng = np.random.default_rng(0)
    for n in (1, 5, 17):
        d = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.4)
        a = dense_csr(d)
        x = rng.standard_normal(n)
        y = oracle.spmv(a, x)
        assert np.max(np.abs(y - d @ x)) <= 1e-14 * max(1.0, np.max(np.abs(d) @ np.abs(x)))
    a, _ = W.problem(6, 2)
    x = rng.standard_normal(a.n)
    y = oracle.spmv(a, x)
    ref = a.to_dense() @ x
    bound = 1e-14 * (np.abs(a.to_dense()) @ np.abs(x))
    assert np.all(np.abs(y - ref) <= bound)


FORMS = ["standard", "single"]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("n,seed,pc", [(4, 0, "jacobi"), (6, 1, "jacobi"), (7, 2, "none"), (8, 3, "jacobi")])
def test_cg_matches_cholesky(n, seed, pc, form):
    a, b = W.problem(n, seed)
    d = a.to_dense()
    xc = sla.cho_solve(sla.cho_factor(d), b)
    x, info = oracle.pcg(a, b, tol=1e-10, precond=pc, form=form)
    assert info["status"] == oracle.CONVERGED
    assert info["relres_true"] <= 1e-10
    kappa = np.linalg.cond(d)
    # Perturbation bound ||x - x*|| / ||x*|| <= kappa ||b - A x|| / ||b||, plus Cholesky's own error.
    err = np.linalg.norm(x - xc) / np.linalg.norm(xc)
    assert err <= kappa * info["relres_true"] * 1.01 + kappa * 1e-15
    # And CG really is that close in practice: x agrees with Cholesky far below the bound.
    assert err <= 1e-6


@pytest.mark.parametrize("form", FORMS)
def test_cg_well_conditioned_to_roundoff(form):
    rng = np.random.default_rng(4)
    n = 40
    g = rng.standard_normal((n, n))
    d = g @ g.T / n + 3 * np.eye(n)
    b = rng.standard_normal(n)
    x, info = oracle.pcg(dense_csr(d), b, tol=1e-14, precond="jacobi", form=form)
    xc = sla.cho_solve(sla.cho_factor(d), b)
    assert info["status"] == oracle.CONVERGED and info["iters"] <= n
    assert np.linalg.norm(x - xc) / np.linalg.norm(xc) <= 1e-12


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("pc", ["jacobi", "none"])
def test_invariants(pc, form):
    # Orthogonality r_i' z_j = 0, conjugacy p_i' A p_j = 0, monotone A-norm error, Chebyshev bound.
    a, b = W.problem(5, 7)
    d = a.to_dense()
    xs = sla.cho_solve(sla.cho_factor(d), b)
    x, info, tr = oracle.pcg(a, b, tol=1e-10, precond=pc, trace=True, form=form)
    k = info["iters"]
    assert info["status"] == oracle.CONVERGED and k >= 10
    X, R, Z, P = tr[:, 0], tr[:, 1], tr[:, 2], tr[:, 3]
    m = min(k, 12)  # exact orthogonality holds for the first steps before rounding erodes it
    for i in range(m):
        for j in range(i):
            rz = R[i] @ Z[j] / (np.linalg.norm(R[i]) * np.linalg.norm(Z[j]))
            pap = P[i] @ d @ P[j] / np.sqrt((P[i] @ d @ P[i]) * (P[j] @ d @ P[j]))
            assert abs(rz) < 1e-8, (i, j, rz)
            assert abs(pap) < 1e-8, (i, j, pap)
    # Recurrence residual equals the true residual early on.
    for i in range(m):
        assert np.linalg.norm(R[i] - (b - d @ X[i])) <= 1e-12 * np.linalg.norm(b)
    e = X - xs
    anorm = np.sqrt(np.einsum("ki,ij,kj->k", e, d, e))
    assert np.all(np.diff(anorm) <= 1e-12 * anorm[0])
    # ||e_k||_A <= 2 ((sqrt(kappa)-1)/(sqrt(kappa)+1))^k ||e_0||_A with kappa of M^-1 A.
    dinv = 1 / np.sqrt(np.diag(d)) if pc == "jacobi" else np.ones(a.n)
    ev = np.linalg.eigvalsh(dinv[:, None] * d * dinv[None, :])
    kap = ev[-1] / ev[0]
    rate = (np.sqrt(kap) - 1) / (np.sqrt(kap) + 1)
    ks = np.arange(len(anorm))
    assert np.all(anorm <= 2 * rate ** ks * anorm[0] * (1 + 1e-9) + 1e-14 * anorm[0])


@pytest.mark.parametrize("form", FORMS)
def test_distinct_eigenvalues_finite_termination(form):
    rng = np.random.default_rng(1)
    n = 30
    u = rng.standard_normal(n)
    d = np.eye(n) + np.outer(u, u)  # eigenvalues {1, 1 + |u|^2}
    x, info = oracle.pcg(dense_csr(d), rng.standard_normal(n), tol=1e-12, precond="none", form=form)
    assert info["status"] == oracle.CONVERGED and info["iters"] == 2
    d3 = np.diag(np.repeat([1.0, 4.0, 9.0], 10))
    x, info = oracle.pcg(dense_csr(d3), rng.standard_normal(n), tol=1e-12, precond="none", form=form)
    assert info["iters"] == 3
    # A diagonal matrix under Jacobi is the identity after preconditioning: one step.
    dd = np.diag(rng.uniform(1, 100, n))
    b = rng.standard_normal(n)
    x, info = oracle.pcg(dense_csr(dd), b, tol=1e-14, precond="jacobi", form=form)
    assert info["iters"] == 1 and np.allclose(x, b / np.diag(dd), rtol=1e-15)


def test_termination_within_n():
    a, b = W.problem(3, 9)
    x, info = oracle.pcg(a, b, tol=1e-12)
    assert info["status"] == oracle.CONVERGED and info["iters"] <= a.n


@pytest.mark.parametrize("form", FORMS)
def test_degenerate_cases(form):
    a, b = W.problem(5, 3)
    x, info = oracle.pcg(a, np.zeros(a.n), x0=np.ones(a.n), form=form)
    assert info["status"] == oracle.CONVERGED and info["iters"] == 0 and not x.any()
    xs = sla.cho_solve(sla.cho_factor(a.to_dense()), b)
    x, info = oracle.pcg(a, b, x0=xs, form=form)
    assert info["status"] == oracle.CONVERGED and info["iters"] == 0
    x, info = oracle.pcg(a, b, maxit=1, form=form)
    assert info["status"] == oracle.MAXIT and info["iters"] == 1
    bn = b.copy()
    bn[3] = np.nan
    x, info = oracle.pcg(a, bn, form=form)
    assert info["status"] == oracle.BREAKDOWN
    # Indefinite: flip one diagonal block sign.
    ind = dense_csr(np.diag([1.0, 2.0, -3.0, 4.0]))
    x, info = oracle.pcg(ind, np.ones(4), precond="none", form=form)
    assert info["status"] == oracle.BREAKDOWN
    # Jacobi needs a positive diagonal.
    bad = dense_csr(np.array([[0.0, 1.0], [1.0, 2.0]]))
    x, info = oracle.pcg(bad, np.ones(2), precond="jacobi", form=form)
    assert info["status"] == oracle.EDIAG


def test_history_matches_true_residual_at_exit():
    a, b = W.problem(8, 0)
    x, info, hist, tr = oracle.pcg(a, b, history=True, trace=True)
    assert len(hist) == info["iters"] + 1
    # Early on, the recurrence residual norm equals the true residual norm of the iterate.
    d, nb = a.to_dense(), np.linalg.norm(b)
    for k in range(8):
        assert abs(hist[k] - np.linalg.norm(b - d @ tr[k, 0]) / nb) <= 1e-12 * hist[0]
    assert hist[-1] <= 1e-10 < hist[-2]
    assert abs(oracle.relres(a, b, x) - info["relres_true"]) <= 1e-3 * info["relres_true"]


def test_self_consistency_pairwise_16():
    # Two rounding orders of the same method: the GPU parity target (+-2 iterations,
    # solution rel. error 1e-8) must be attainable between them.
    a, b = W.problem(16, 0)
    x0, i0 = oracle.pcg(a, b, sum_mode=0)
    x1, i1 = oracle.pcg(a, b, sum_mode=1)
    assert abs(i0["iters"] - i1["iters"]) <= 2
    assert np.linalg.norm(x0 - x1) / np.linalg.norm(x0) <= 1e-8
    # The same on the part of x beyond its constant mode (1'b / c per entry
    # dominates ||x||): the bar the GPU solves are held to is attainable.
    xm0, xm1 = x0 - x0.mean(), x1 - x1.mean()
    assert np.linalg.norm(xm0 - xm1) / np.linalg.norm(xm0) <= 1e-8


def test_single_reduction_form_tracks_standard_iterates():
    # Same Krylov iterates in exact arithmetic: early iterates agree to rounding level,
    # and on the FEM system the counts agree within +-2 and the solutions within 1e-8.
    a, b = W.problem(6, 4)
    _, i0, t0 = oracle.pcg(a, b, trace=True)
    _, i1, t1 = oracle.pcg(a, b, trace=True, form="single")
    for k in range(10):
        for slot in (0, 1, 3):  # x, r, p
            ref = np.linalg.norm(t0[k, slot])
            assert np.linalg.norm(t1[k, slot] - t0[k, slot]) <= 1e-9 * ref, (k, slot)
    a, b = W.problem(16, 0)
    x0, i0 = oracle.pcg(a, b)
    x1, i1 = oracle.pcg(a, b, form="single")
    assert abs(i0["iters"] - i1["iters"]) <= 2 and i1["relres_true"] <= 1e-10
    assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) <= 1e-8


@pytest.mark.parametrize("fam_n,first,count", [(14, 0, 8), (16, 0, 40)])
def test_single_reduction_form_across_replacements(fam_n, first, count):
    # Systems whose solves need residual replacements at 1e-10.  The single-
    # reduction form takes sigma = p's (never a scalar recurrence, which turns
    # negative on 15 of the first 40 of these 16^3 right-hand sides) and
    # recomputes w = A u and s = A p after a replacement, so it keeps
    # tracking the standard form: same status, within +-2 iterations, the
    # same solution to 1e-8 with and without its constant mode.
    a, _ = W.problem(fam_n, 0)
    fam = W.amplitude_family(n=fam_n, count=first + count)
    reps = 0
    for b in fam.rhs(np.arange(first, first + count)):
        x0, i0 = oracle.pcg(a, b)
        x1, i1 = oracle.pcg(a, b, form="single")
        reps += i1["replacements"]
        assert i0["status"] == i1["status"] == oracle.CONVERGED
        assert abs(i0["iters"] - i1["iters"]) <= 2
        assert i1["relres_true"] <= 1e-10
        assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) <= 1e-8
        xm0, xm1 = x0 - x0.mean(), x1 - x1.mean()
        assert np.linalg.norm(xm1 - xm0) / np.linalg.norm(xm0) <= 1e-8
    assert reps >= count // 2


def _residual_reversed_rows(a, b, x):
    """b - A x with every row summed from its last stored entry to its first."""
    prod = a.val * x[a.col]
    lens = np.diff(a.rowptr)
    acc = np.zeros(a.n)
    for k in range(int(lens.max())):
        has = lens > k
        acc[has] += prod[a.rowptr[1:][has] - 1 - k]
    return b - acc


@pytest.mark.slow
def test_learned_family_attainable_accuracy():
    # Why the learned family is solved to 1e-8: b = M f of narrow smooth
    # sources is small against A x, whose constant mode is 1'b / c with
    # c = 1e-3.  The FP64 true residual b - A x of such x is then determined
    # only to about u || |A| |x| || (the rounding of the row sums), which is
    # of the order of 1e-10 ||b|| itself: two summation orders of the same
    # residual already differ by more than a tenth of 1e-10 ||b||, and the
    # oracle, with residual replacement, stays above 1e-10 for three times the
    # iterations that 1e-8 takes.
    a, _ = W.problem(51, 0)
    fam = W.source_family(n=51, count=2)
    rows = np.repeat(np.arange(a.n), np.diff(a.rowptr))
    u = 2.0 ** -53
    for s in range(2):
        b = fam.rhs(s)[0]
        nb = np.linalg.norm(b)
        x8, i8 = oracle.pcg(a, b, tol=1e-8)
        assert i8["status"] == oracle.CONVERGED and i8["iters"] < 400
        r1, _ = oracle.residual(a, b, x8)
        r2 = _residual_reversed_rows(a, b, x8)
        assert np.linalg.norm(r1 - r2) / nb >= 1e-11
        abs_ax = np.bincount(rows, weights=np.abs(a.val) * np.abs(x8[a.col]), minlength=a.n)
        assert u * np.linalg.norm(abs_ax) / nb >= 5e-11
        x, info = oracle.pcg(a, b, tol=1e-10, maxit=3 * i8["iters"])
        assert info["status"] == oracle.MAXIT and info["replacements"] >= 2
        assert info["relres_true"] > 1e-10


def test_mixed_matrix_form_tracks_fp64():
    # The FP32-matrix form is the FP64 iteration on a perturbed operator
    # (values rounded to single precision, row sums kept in double) with
    # reliable updates on the FP64 residual: it must meet the tolerance on
    # the FP64 residual in about the FP64 oracle's iterations, within 1e-8 of
    # its solution once the constant mode is removed.
    from conftest import mean_removed_relerr

    for n, seed in ((12, 0), (16, 0), (16, 3)):
        a, b = W.problem(n, seed)
        x, i = oracle.pcg(a, b, tol=1e-10)
        for drop in (1e-1, 1e-2, 1e-3):
            xm, im = oracle.pcg_mixed_matrix(a, b, tol=1e-10, drop=drop)
            assert im["status"] == oracle.CONVERGED and im["relres_true"] <= 1e-10
            assert abs(im["iters"] - i["iters"]) <= 2
            # The constant mode (A 1 is only the small mass term) is barely
            # determined by a 1e-10 residual, so the distance to the FP64
            # solution is judged with that mode removed.
            assert mean_removed_relerr(xm, x) <= 1e-8
            # one replacement per factor drop of residual reduction (10 decades to 1e-10)
            assert im["replacements"] >= int(10 / -np.log10(drop)) - 1
        # Without the updates the recurrence stalls above the tolerance (the
        # FP32 values move the fixed point away from A^-1 b).
        _, i0 = oracle.pcg_mixed_matrix(a, b, tol=1e-10, drop=0.0, maxit=4 * i["iters"])
        assert i0["status"] == oracle.MAXIT


def test_mixed_matrix_form_exact_values():
    # Values already in single precision (dyadic entries): the only difference
    # from the plain product is the row-sum-preserving evaluation, so the
    # iterates equal the plain oracle's to rounding.
    rng = np.random.default_rng(4)
    n = 30
    B = rng.integers(-4, 5, (n, n)).astype(float)
    d = B @ B.T / 8.0 + np.eye(n) * 4.0
    rowptr = np.arange(0, n * n + 1, n, dtype=np.int32)
    a = W.CSR(n, rowptr, np.tile(np.arange(n, dtype=np.int32), n), d.reshape(-1))
    assert np.array_equal(a.val.astype(np.float32).astype(np.float64), a.val)
    b = rng.standard_normal(n)
    for k in (1, 3, 8):
        x, _ = oracle.pcg(a, b, maxit=k, tol=1e-14)
        xm, _ = oracle.pcg_mixed_matrix(a, b, maxit=k, tol=1e-14, drop=0.0)
        assert np.linalg.norm(xm - x) <= 1e-12 * np.linalg.norm(x)
