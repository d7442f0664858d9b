"""Pins for the synthetic Q1-hex systems (input generation, not the solver).

The paper fixes N = 132651 and NNZ = 3442951 (Section IV and the caption of
Table I); the rest is fixed by the textbook trilinear element.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W


def _m1(n):
    # 1-D linear element on [0, 1], written out independently of the generator.
    h = 1.0 / (n - 1)
    m = np.diag(np.full(n, 2 * h / 3))
    m[0, 0] = m[-1, -1] = h / 3
    m += np.diag(np.full(n - 1, h / 6), 1) + np.diag(np.full(n - 1, h / 6), -1)
    return m


def _k1(n):
    h = 1.0 / (n - 1)
    k = np.diag(np.full(n, 2 / h))
    k[0, 0] = k[-1, -1] = 1 / h
    k += np.diag(np.full(n - 1, -1 / h), 1) + np.diag(np.full(n - 1, -1 / h), -1)
    return k


def test_paper_size_exact():
    # Section IV: N=132651, NNZ=3442951 -- reproduced exactly at 51^3.
    a, _ = W.problem(51, 0)
    assert a.n == 132651 and a.nnz == 3442951
    assert W.pattern_size(16) == (4096, 97336)
    assert W.pattern_size(128) == (2097152, 55742968)


@pytest.mark.parametrize("n", [3, 7, 16])
def test_row_histogram_and_sorted_columns(n):
    a, _ = W.problem(n, 0)
    cnt = np.diff(a.rowptr)
    hist = {int(k): int(v) for k, v in zip(*np.unique(cnt, return_counts=True))}
    want = {8: 8, 12: 12 * (n - 2), 18: 6 * (n - 2) ** 2, 27: (n - 2) ** 3}
    assert hist == {k: v for k, v in want.items() if v}
    for i in range(a.n):
        c = a.col[a.rowptr[i]:a.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c


def test_bitwise_symmetric():
    a, _ = W.problem(16, 0)
    s = a.to_scipy()
    d = (s - s.T).tocoo()
    assert d.nnz == 0 or np.all(d.data == 0.0)


def test_constants_in_kernel_of_stiffness():
    # K 1 = 0 for any sigma, so A 1 = c M 1 and 1'A1 = c |Omega| = c.
    n = 12
    a, _ = W.problem(n, 5)
    m = W.mass_matrix(n).to_scipy()
    one = np.ones(a.n)
    a1 = a.to_scipy() @ one
    scale = abs(a.to_scipy()) @ one
    assert np.all(np.abs(a1 - W.MASS_COEF * (m @ one)) <= 1e-13 * scale)
    assert abs(one @ a1 - W.MASS_COEF) <= 1e-12


def test_interior_stencil_constant_sigma():
    n, s, c = 9, 2.5, 1e-3
    a = W.assemble(n, np.full((n - 1,) * 3, s), c).to_dense()
    h = 1.0 / (n - 1)
    i = 4 + n * 4 + n * n * 4
    assert a[i, i] == pytest.approx(h * (8 / 3) * s + c * h ** 3 * 8 / 27, rel=1e-14)
    assert a[i, i + 1] == pytest.approx(c * h ** 3 * 2 / 27, rel=1e-14)
    assert a[i, i + 1 + n] == pytest.approx(-s * h / 6 + c * h ** 3 / 54, rel=1e-14)
    assert a[i, i + 1 + n + n * n] == pytest.approx(-s * h / 12 + c * h ** 3 / 216, rel=1e-14)
    assert a[i].sum() == pytest.approx(c * h ** 3, rel=1e-9)


def test_kronecker_form_constant_sigma():
    # A = s (K1 x M1 x M1 + M1 x K1 x M1 + M1 x M1 x K1) + c M1 x M1 x M1, an independent build.
    n, s, c = 6, 0.7, 1e-3
    a = W.assemble(n, np.full((n - 1,) * 3, s), c).to_dense()
    m, k = _m1(n), _k1(n)
    kr = lambda x, y, z: np.kron(x, np.kron(y, z))
    ref = s * (kr(k, m, m) + kr(m, k, m) + kr(m, m, k)) + c * kr(m, m, m)
    assert np.max(np.abs(a - ref)) <= 1e-15 * np.max(np.abs(ref)) * 10


def test_spd_small():
    a, _ = W.problem(5, 1)
    ev = np.linalg.eigvalsh(a.to_dense())
    assert ev[0] > 0


def test_seed_order_sigma_then_b():
    a1, b1 = W.problem(6, 11)
    rng = np.random.default_rng(11)
    rng.standard_normal(5 ** 3)
    assert np.array_equal(b1, rng.uniform(-1, 1, 6 ** 3))


def test_source_rhs_equals_mass_times_field():
    fam = W.source_family(n=9, count=3, k=4, seed=3)
    m = W.mass_matrix(9).to_scipy()
    b = fam.rhs([0, 1, 2])
    for s in range(3):
        ref = m @ fam.source_field(s)
        assert np.max(np.abs(b[s] - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert fam.theta().shape == (3, 12)


def test_batch_sizes_in_range():
    sys = W.batch_systems(count=3)
    for n, a, b in sys:
        assert 12 <= n <= 48 and a.n == n ** 3 and a.nnz == (3 * n - 2) ** 3 and b.shape == (a.n,)


def test_stored_oracle_values_128():
    # The stored 128^3 oracle solves (tests/golden/make_q1hex128.py) describe
    # this workload: sizes by the closed forms, the standard form converged.
    import json
    import os

    with open(os.path.join(os.path.dirname(__file__), "golden", "q1hex128_oracle.json")) as f:
        g = json.load(f)
    assert g["n"] == 128 ** 3 and g["nnz"] == (3 * 128 - 2) ** 3
    rows = g["rows"]
    assert len(rows) == len(set(rows)) == 1024 and rows == sorted(rows) and 0 <= rows[0] and rows[-1] < g["n"]
    st = g["forms"]["standard"]
    assert st["status"] == 0 and st["relres_true"] <= 1e-10 and 0 < st["iters"] <= g["n"]
    assert len(st["x_rows"]) == 1024 and st["x_norm"] > 0


def test_elementwise_q1_oracle_matches_the_assembled_matrix():
    # Two independent builds of the same operator: the generator's entry
    # tables (assembled CSR, multiplied by the C oracle) and the element-by-
    # element oracle with element matrices from 1-D Kronecker products.
    import oracle
    import oracle.q1 as q1

    for n in (2, 3, 6, 11):
        rng = np.random.default_rng(n)
        sig = np.exp(rng.standard_normal((n - 1,) * 3))
        a = W.assemble(n, sig, 1e-3)
        x = rng.standard_normal(n ** 3)
        y = q1.apply(n, sig, 1e-3, x)
        yo = oracle.spmv(a, x)
        rows = np.repeat(np.arange(a.n), np.diff(a.rowptr))
        absax = np.bincount(rows, weights=np.abs(a.val * x[a.col]), minlength=a.n)
        assert np.all(np.abs(y - yo) <= 1e-14 * absax)
        # The element-wise rounding scale bounds the assembled row's sum_j |a_ij x_j|.
        assert np.all(q1.abs_row_bound(n, sig, 1e-3, x) >= absax * (1 - 1e-12))
        X = rng.standard_normal((n ** 3, 3))
        y1 = q1.apply(n, sig, 1e-3, X[:, 1])
        assert np.allclose(q1.apply(n, sig, 1e-3, X)[:, 1], y1, rtol=0, atol=1e-14 * np.max(np.abs(y1)))
        d = q1.diagonal(n, sig, 1e-3)
        dd = a.to_dense().diagonal() if n <= 6 else np.array(
            [a.val[a.rowptr[i]:a.rowptr[i + 1]][a.col[a.rowptr[i]:a.rowptr[i + 1]] == i][0] for i in range(a.n)])
        assert np.allclose(d, dd, rtol=1e-14, atol=0)


def test_elementwise_q1_oracle_invariants():
    import oracle.q1 as q1

    n = 7
    rng = np.random.default_rng(3)
    sig = np.exp(rng.standard_normal((n - 1,) * 3))
    # K 1 = 0: the operator maps the constant to c M 1, and 1'A1 = c |Omega|.
    y = q1.apply(n, sig, 1e-3, np.ones(n ** 3))
    ym = q1.apply(n, np.zeros_like(sig), 1.0, np.ones(n ** 3))
    assert np.allclose(y, 1e-3 * ym, rtol=1e-12, atol=1e-18)
    assert abs(y.sum() - 1e-3) <= 1e-15
    # Symmetric: x'A y = y'A x.
    x, z = rng.standard_normal(n ** 3), rng.standard_normal(n ** 3)
    assert abs(x @ q1.apply(n, sig, 1e-3, z) - z @ q1.apply(n, sig, 1e-3, x)) <= 1e-12 * abs(x @ q1.apply(n, sig, 1e-3, z))
    # Element matrices: K_e 1 = 0, 1'M_e 1 = h^3, textbook diagonal 8/3 s... in units of h.
    K, M = q1.element_matrices(0.5)
    assert np.allclose(K @ np.ones(8), 0.0) and np.isclose(M.sum(), 0.5 ** 3)
    assert np.allclose(np.diag(K), 0.5 / 3.0) and np.allclose(np.diag(M), 0.5 ** 3 / 27.0)
