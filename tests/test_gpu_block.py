"""Block CG on the GPU (cg_solve_block) against the block-CG oracle.

Both run the same algorithm (O'Leary's block CG, breakdown-free form, search
blocks orthonormalised by shifted CholeskyQR), so the bar is the solver's:
the same status, block iterations within +-2, every column's true relative
residual (recomputed on the CPU) within the tolerance, and every column of X
within 1e-8 of the oracle's, normwise and with the constant mode removed.
"""
import json
import os

import numpy as np
import pytest

import oracle
import oracle.block_cg as bc
import workloads as W
from conftest import mean_removed_relerr, tol_recomputed

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "block51_oracle.json")


def _solve(a, B, cuda, tol=1e-10, maxit=0, X0=None):
    import torch

    from paper_1107_0538_amd import Solver

    s = Solver(a)
    Bd = torch.as_tensor(np.ascontiguousarray(B), device=cuda)
    X0d = None if X0 is None else torch.as_tensor(np.ascontiguousarray(X0), device=cuda)
    X, infos = s.solve_block(Bd, X0=X0d, tol=tol, maxit=maxit)
    return X.cpu().numpy(), infos


def _check_against_oracle(a, B, Xg, infos, tol=1e-10):
    Xo, io = bc.block_pcg(a, B, tol=tol)
    assert io["status"] == oracle.CONVERGED
    assert all(i["status"] == 0 for i in infos), infos[0]
    assert abs(infos[0]["iters"] - io["iters"]) <= 2, (infos[0]["iters"], io["iters"])
    bound = tol_recomputed(a.n, tol)
    for j in range(B.shape[1]):
        if not B[:, j].any():
            assert not Xg[:, j].any()
            continue
        assert oracle.relres(a, B[:, j], Xg[:, j]) <= bound, j
        nx = np.linalg.norm(Xo[:, j])
        assert np.linalg.norm(Xg[:, j] - Xo[:, j]) <= 1e-8 * nx, j
        assert mean_removed_relerr(Xg[:, j], Xo[:, j]) <= 1e-8, j
    return io


@pytest.mark.parametrize("n,s", [(16, 64), (16, 8), (13, 5), (11, 64), (9, 1)])
def test_block_solve_parity(cuda, n, s):
    a, _ = W.problem(n, 0)
    B = W.multi_rhs(a.n, s, seed=2 + n)
    Xg, infos = _solve(a, B, cuda)
    _check_against_oracle(a, B, Xg, infos)
    assert 1 <= infos[0]["outer"] <= s  # rank of the last search block


def test_block_needs_fewer_iterations_than_columns_alone(cuda):
    import torch

    from paper_1107_0538_amd import Solver

    a, _ = W.problem(16, 0)
    B = W.multi_rhs(a.n, 64)
    s = Solver(a)
    Bd = torch.as_tensor(B, device=cuda)
    _, infos = s.solve_block(Bd)
    _, multi = s.solve_multi(Bd)
    assert infos[0]["iters"] * 3 < min(i["iters"] for i in multi)


def test_rank_deficient_block(cuda):
    a, _ = W.problem(10, 1)
    rng = np.random.default_rng(6)
    F = W.multi_rhs(a.n, 3, seed=7)
    B = np.concatenate([F, F[:, :1], np.zeros((a.n, 1)), F @ rng.standard_normal((3, 3))], axis=1)
    Xg, infos = _solve(a, B, cuda)
    _check_against_oracle(a, B, Xg, infos)
    assert np.linalg.norm(Xg[:, 3] - Xg[:, 0]) <= 1e-8 * np.linalg.norm(Xg[:, 0])


def test_degenerate_block_inputs(cuda):
    import torch

    from paper_1107_0538_amd import Solver, capi

    a, b = W.problem(6, 2)
    B = np.stack([b, -b, 2 * b], axis=1)
    s = Solver(a)
    Bd = torch.as_tensor(np.zeros_like(B), device=cuda)
    X, infos = s.solve_block(Bd)
    assert infos[0]["status"] == 0 and infos[0]["iters"] == 0 and not X.any()
    # X0 = the solution: no iteration.
    Xs, _ = bc.block_pcg(a, B, tol=1e-13)
    X, infos = s.solve_block(torch.as_tensor(B, device=cuda), X0=torch.as_tensor(Xs, device=cuda))
    assert infos[0]["status"] == 0 and infos[0]["iters"] == 0
    # Iteration limit.
    X, infos = s.solve_block(torch.as_tensor(B, device=cuda), maxit=2)
    assert infos[0]["status"] == capi.CG_MAXIT and infos[0]["iters"] == 2
    # Non-finite input.
    Bn = B.copy()
    Bn[3, 1] = np.nan
    X, infos = s.solve_block(torch.as_tensor(Bn, device=cuda))
    assert infos[0]["status"] == capi.CG_BREAKDOWN
    # An indefinite matrix breaks down like the oracle.
    d = a.to_dense()
    d[0, 0] = -d[0, 0]
    rows, cols = np.nonzero(d)
    ai = W.CSR(a.n, np.searchsorted(rows, np.arange(a.n + 1)).astype(np.int32), cols.astype(np.int32), d[rows, cols])
    _, io = bc.block_pcg(ai, B, precond="none")
    si = Solver(ai, precond="none")
    X, infos = si.solve_block(torch.as_tensor(B, device=cuda))
    assert io["status"] == oracle.BREAKDOWN and infos[0]["status"] == capi.CG_BREAKDOWN


def test_block_arguments_rejected(cuda):
    import torch

    from paper_1107_0538_amd import Solver

    a, _ = W.problem(6, 0)
    s = Solver(a)
    B = torch.zeros((a.n, 4), dtype=torch.float64, device=cuda)
    with pytest.raises(ValueError):
        s.cg_solve_block(B, B)  # aliasing
    with pytest.raises(ValueError):
        s.cg_solve_block(B, torch.zeros((a.n, 65), dtype=torch.float64, device=cuda))


def test_block_full_size_against_stored_oracle(cuda):
    # 51^3 (the paper's N and NNZ) with 64 right-hand sides: the oracle's
    # solve is stored by tests/golden/make_block51.py.
    g = json.load(open(GOLDEN))
    a, _ = W.problem(51, 0)
    B = W.multi_rhs(a.n, 64)
    Xg, infos = _solve(a, B, cuda)
    assert all(i["status"] == g["status"] for i in infos)
    assert abs(infos[0]["iters"] - g["iters"]) <= 2, (infos[0]["iters"], g["iters"])
    rows = np.asarray(g["rows"])
    Xo_rows = np.asarray(g["x_rows"])
    bound = tol_recomputed(a.n)
    for j in range(64):
        assert oracle.relres(a, B[:, j], Xg[:, j]) <= bound, j
        assert abs(np.linalg.norm(Xg[:, j]) - g["x_norm"][j]) <= 1e-8 * g["x_norm"][j]
        assert np.linalg.norm(Xg[rows, j] - Xo_rows[:, j]) <= 1e-8 * np.linalg.norm(Xo_rows[:, j])
        # The sampled rows with each side's constant mode (its mean over all rows) removed.
        dg = Xg[rows, j] - Xg[:, j].mean()
        do = Xo_rows[:, j] - g["x_mean"][j]
        assert np.linalg.norm(dg - do) <= 1e-8 * np.linalg.norm(do), j
