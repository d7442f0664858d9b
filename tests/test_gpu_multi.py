"""Multi-RHS form: s independent Jacobi-PCG recurrences sharing one product per iteration.

Each column is judged against its own FP64 oracle solve with the single-RHS
criteria (+-2 iterations, solution within 1e-8, true relres <= 1e-10); spmm's
column j must equal the oracle's sequential product of column j bitwise.
"""
import functools

import numpy as np
import pytest

import oracle
import workloads as W
from conftest import mean_removed_relerr, tol_recomputed

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def mat(n, seed=0):
    return W.problem(n, seed)[0]


def _t(a, dev):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), device=dev)


@pytest.mark.parametrize("n,s", [(16, 64), (16, 7), (51, 64), (3, 1)])
def test_spmm_bitwise(cuda, n, s):
    from paper_1107_0538_amd import Solver

    a = mat(n)
    X = np.random.default_rng(n + s).uniform(-1, 1, (a.n, s))
    Y = Solver(a).spmm(_t(X, cuda)).cpu().numpy()
    for j in range(s):
        assert np.array_equal(Y[:, j], oracle.spmv(a, X[:, j])), j


@pytest.mark.parametrize("s", [64, 3])
def test_spmm_bitwise_ragged_and_hub_rows(cuda, s):
    # Short rows and four hub rows of more than 1024 nonzeros (many gather
    # batches per row, the tail batch reading into the arrays' zero pad).
    from test_gpu_pcg import ragged_matrix

    from paper_1107_0538_amd import Solver

    a = ragged_matrix()
    X = np.random.default_rng(s).uniform(-1, 1, (a.n, s))
    Y = Solver(a).spmm(_t(X, cuda)).cpu().numpy()
    for j in range(s):
        assert np.array_equal(Y[:, j], oracle.spmv(a, X[:, j])), j


def test_multi_rhs_solve_on_ragged_rows(cuda):
    from test_gpu_pcg import ragged_matrix

    from paper_1107_0538_amd import Solver

    a = ragged_matrix(seed=1)
    B = np.random.default_rng(4).uniform(-1, 1, (a.n, 8))
    X, infos = Solver(a).solve_multi(_t(B, cuda))
    X = X.cpu().numpy()
    for j in range(8):
        xo, io = oracle.pcg(a, B[:, j])
        assert infos[j]["status"] == io["status"] and abs(infos[j]["iters"] - io["iters"]) <= 2
        assert np.linalg.norm(X[:, j] - xo) <= 1e-8 * np.linalg.norm(xo)


@pytest.mark.parametrize("s", [64, 5])
def test_multi_rhs_parity_16(cuda, s):
    from paper_1107_0538_amd import Solver

    a = mat(16)
    B = W.multi_rhs(a.n, s)
    X, infos = Solver(a).solve_multi(_t(B, cuda))
    X = X.cpu().numpy()
    for j in range(s):
        xo, io = oracle.pcg(a, B[:, j])
        assert infos[j]["status"] == 0 and io["status"] == 0
        assert abs(infos[j]["iters"] - io["iters"]) <= 2, (j, infos[j], io)
        assert np.linalg.norm(X[:, j] - xo) / np.linalg.norm(xo) <= 1e-8
        assert mean_removed_relerr(X[:, j], xo) <= 1e-8
        assert oracle.relres(a, B[:, j], X[:, j]) <= tol_recomputed(a.n)


def test_multi_rhs_51_sampled(cuda):
    # The multi-RHS workload: 64 right-hand sides on the 51^3 matrix.
    from paper_1107_0538_amd import Solver

    a = mat(51)
    B = W.multi_rhs(a.n, 64)
    X, infos = Solver(a).solve_multi(_t(B, cuda))
    X = X.cpu().numpy()
    for j in range(64):
        assert infos[j]["status"] == 0
        assert oracle.relres(a, B[:, j], X[:, j]) <= tol_recomputed(a.n)
    for j in (0, 17, 63):
        xo, io = oracle.pcg(a, B[:, j])
        assert abs(infos[j]["iters"] - io["iters"]) <= 2
        assert np.linalg.norm(X[:, j] - xo) / np.linalg.norm(xo) <= 1e-8
        assert mean_removed_relerr(X[:, j], xo) <= 1e-8


def test_multi_rhs_mixed_columns(cuda):
    # Zero column, a column already solved by X0, a NaN column, and normal ones.
    from paper_1107_0538_amd import Solver

    a = mat(7)
    rng = np.random.default_rng(9)
    B = rng.uniform(-1, 1, (a.n, 6))
    B[:, 1] = 0.0
    xs, _ = oracle.pcg(a, B[:, 2], tol=1e-13)
    X0 = np.zeros_like(B)
    X0[:, 1] = 1.0
    X0[:, 2] = xs
    B[3, 4] = np.nan
    X, infos = Solver(a).solve_multi(_t(B, cuda), X0=_t(X0, cuda))
    X = X.cpu().numpy()
    assert infos[1]["status"] == 0 and infos[1]["iters"] == 0 and not X[:, 1].any()
    assert infos[2]["status"] == 0 and infos[2]["iters"] == 0
    assert infos[4]["status"] == 2
    for j in (0, 3, 5):
        xo, io = oracle.pcg(a, B[:, j])
        assert infos[j]["status"] == 0 and abs(infos[j]["iters"] - io["iters"]) <= 2
        assert np.linalg.norm(X[:, j] - xo) / np.linalg.norm(xo) <= 1e-8
        assert mean_removed_relerr(X[:, j], xo) <= 1e-8


def test_multi_rhs_limit_and_replacement(cuda):
    from paper_1107_0538_amd import Solver

    a = mat(16)
    B = W.multi_rhs(a.n, 4, seed=5)
    s = Solver(a)
    X, infos = s.solve_multi(_t(B, cuda), maxit=3)
    for j in range(4):
        xo, io = oracle.pcg(a, B[:, j], maxit=3)
        assert infos[j]["status"] == io["status"] == 1 and infos[j]["iters"] == 3
        assert np.linalg.norm(X.cpu().numpy()[:, j] - xo) <= 1e-9 * np.linalg.norm(xo)
    X, infos = s.solve_multi(_t(B, cuda), tol=1e-16, maxit=400)
    for j in range(4):
        xo, io = oracle.pcg(a, B[:, j], tol=1e-16, maxit=400)
        assert infos[j]["status"] == io["status"] == 1
        assert infos[j]["replacements"] >= 1 and io["replacements"] >= 1
        assert infos[j]["relres_true"] <= 1e-10


def test_multi_rhs_replacement_resume(cuda):
    # Right-hand sides whose solves need residual replacements: a column
    # resumes after its true-residual check while the iteration count on the
    # host has run ahead, so the resumed direction must come from the device's
    # own iteration parity.
    from paper_1107_0538_amd import Solver

    a = mat(16)
    fam = W.amplitude_family(n=16, count=64)
    B = np.ascontiguousarray(fam.rhs(np.arange(64)).T)
    X, infos = Solver(a).solve_multi(_t(B, cuda))
    X = X.cpu().numpy()
    reps = 0
    for j in range(64):
        xo, io = oracle.pcg(a, B[:, j])
        reps += io["replacements"]
        assert infos[j]["status"] == io["status"] == 0, (j, infos[j], io)
        assert abs(infos[j]["iters"] - io["iters"]) <= 2, (j, infos[j], io)
        assert np.linalg.norm(X[:, j] - xo) / np.linalg.norm(xo) <= 1e-8
        assert mean_removed_relerr(X[:, j], xo) <= 1e-8
        assert oracle.relres(a, B[:, j], X[:, j]) <= tol_recomputed(a.n)
    assert reps >= 32


def test_multi_rhs_block_width_changes(cuda):
    # One context, block widths 64, 44, 64, 5 in turn: each call matches the oracle.
    from paper_1107_0538_amd import Solver

    a = mat(16)
    s = Solver(a)
    for width in (64, 44, 64, 5):
        B = W.multi_rhs(a.n, width, seed=width)
        X, infos = s.solve_multi(_t(B, cuda))
        X = X.cpu().numpy()
        for j in (0, width // 2, width - 1):
            xo, io = oracle.pcg(a, B[:, j])
            assert infos[j]["status"] == 0 and abs(infos[j]["iters"] - io["iters"]) <= 2
            assert np.linalg.norm(X[:, j] - xo) / np.linalg.norm(xo) <= 1e-8
            assert mean_removed_relerr(X[:, j], xo) <= 1e-8


@pytest.mark.parametrize("n,s", [(16, 64), (51, 8)])
def test_multi_rhs_mixed_meets_fp64_tolerance(cuda, n, s):
    # FP32 inner multi-RHS solves with FP64 refinement: every column meets the
    # FP64 test, recomputed on the CPU.
    from paper_1107_0538_amd import Solver

    a = mat(n)
    B = W.multi_rhs(a.n, s)
    sv = Solver(a, fp32_copy=True)
    X, infos = sv.solve_multi_mixed(_t(B, cuda))
    X = X.cpu().numpy()
    for j in range(s):
        assert infos[j]["status"] == 0, (j, infos[j])
        assert infos[j]["outer"] >= 1
        assert oracle.relres(a, B[:, j], X[:, j]) <= tol_recomputed(a.n)
    for j in (0, s - 1):
        xo, io = oracle.pcg(a, B[:, j])
        assert np.linalg.norm(X[:, j] - xo) / np.linalg.norm(xo) <= 1e-5


def test_multi_rhs_mixed_columns_and_limits(cuda):
    from paper_1107_0538_amd import Solver

    a = mat(7)
    rng = np.random.default_rng(4)
    B = rng.uniform(-1, 1, (a.n, 5))
    B[:, 1] = 0.0
    B[2, 3] = np.nan
    X0 = np.zeros_like(B)
    X0[:, 1] = 1.0
    sv = Solver(a, fp32_copy=True)
    X, infos = sv.solve_multi_mixed(_t(B, cuda), X0=_t(X0, cuda))
    X = X.cpu().numpy()
    assert infos[1]["status"] == 0 and not X[:, 1].any()
    assert infos[3]["status"] == 2
    for j in (0, 2, 4):
        assert infos[j]["status"] == 0 and oracle.relres(a, B[:, j], X[:, j]) <= tol_recomputed(a.n)
    Bg = W.multi_rhs(a.n, 3, seed=8)
    X, infos = sv.solve_multi_mixed(_t(Bg, cuda), maxit_outer=1, tol_inner=1e-2)
    assert all(i["status"] == 1 and i["outer"] == 1 for i in infos)
    with pytest.raises(ValueError):
        Solver(a).solve_multi_mixed(_t(Bg, cuda))


def test_autotuned_multi_column_product(cuda):
    # With autotune the first multi-column use times the product's grid; the
    # products and solves are unchanged bitwise / within the solver's bar.
    from paper_1107_0538_amd import Solver

    a = mat(16)
    s = Solver(a, autotune=True)
    X = np.random.default_rng(3).uniform(-1, 1, (a.n, 64))
    Y = s.spmm(_t(X, cuda)).cpu().numpy()
    for j in (0, 17, 63):
        assert np.array_equal(Y[:, j], oracle.spmv(a, X[:, j]))
    cfg = s.config()
    assert cfg["spmm_blocks_per_cu"] in (1, 2, 3, 4, 6, 8) and cfg["spmm_us"] > 0
    B = W.multi_rhs(a.n, 8)
    Xm, infos = s.solve_multi(_t(B, cuda))
    Xm = Xm.cpu().numpy()
    for j in range(8):
        xo, io = oracle.pcg(a, B[:, j])
        assert abs(infos[j]["iters"] - io["iters"]) <= 2
        assert np.linalg.norm(Xm[:, j] - xo) <= 1e-8 * np.linalg.norm(xo)
    Xb, binfo = s.solve_block(_t(B, cuda))
    assert binfo[0]["status"] == 0
    for j in range(8):
        assert oracle.relres(a, B[:, j], Xb.cpu().numpy()[:, j]) <= tol_recomputed(a.n)
