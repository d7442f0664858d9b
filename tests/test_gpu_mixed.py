"""Mixed-precision form: FP32 inner Jacobi-PCG, FP64 outer residual, update and test.

No paper content fixes this form; it is judged by the FP64 oracle alone: the
true relative residual of the returned x, recomputed on the CPU in FP64, must
meet the tolerance, and the distance to the FP64 oracle solution is bounded.
"""
import functools

import numpy as np
import pytest

import oracle
import workloads as W
from conftest import mean_removed_relerr, tol_recomputed

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def prob(n, seed=0):
    return W.problem(n, seed)


def _t(a, dev):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), device=dev)


@pytest.mark.parametrize("n,tol_in", [(16, 1e-5), (51, 1e-5), (51, 1e-3), (7, 1e-6)])
def test_mixed_meets_fp64_tolerance(cuda, n, tol_in):
    from paper_1107_0538_amd import Solver

    a, b = prob(n)
    s = Solver(a, fp32_copy=True)
    x, info = s.solve_mixed(_t(b, cuda), tol=1e-10, tol_inner=tol_in)
    xg = x.cpu().numpy()
    assert info["status"] == 0, info
    rr = oracle.relres(a, b, xg)
    assert rr <= tol_recomputed(a.n)
    assert abs(info["relres_true"] - rr) <= 1e-3 * rr + 1e-13
    assert info["outer"] >= 1
    # Both solutions meet relres 1e-10; on this ill-conditioned system two
    # different Krylov paths stopped there may differ by up to ~kappa * 1e-10.
    # The distance is reported; the bound is only a sanity check.
    xo, io = oracle.pcg(a, b, tol=1e-10)
    err = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    print(f"mixed n={n} tol_in={tol_in}: outer {info['outer']} inner {info['iters']} "
          f"(fp64 oracle {io['iters']}), |x - x_fp64| / |x_fp64| = {err:.2e}")
    assert err <= 1e-5, err


def test_mixed_requires_fp32_copy(cuda):
    from paper_1107_0538_amd import Solver

    a, b = prob(7)
    s = Solver(a)
    with pytest.raises(ValueError):
        s.solve_mixed(_t(b, cuda))


def test_mixed_degenerate(cuda):
    import torch

    from paper_1107_0538_amd import Solver

    a, b = prob(7)
    s = Solver(a, fp32_copy=True)
    bt = _t(b, cuda)
    x, info = s.solve_mixed(torch.zeros_like(bt), x0=torch.ones_like(bt))
    assert info["status"] == 0 and not bool(x.any())
    bn = b.copy()
    bn[2] = np.nan
    x, info = s.solve_mixed(_t(bn, cuda))
    assert info["status"] == 2
    x, info = s.solve_mixed(bt, maxit_outer=1, tol_inner=1e-2)
    assert info["status"] == 1 and info["outer"] == 1
    x, info = s.solve_mixed(bt)
    assert info["status"] == 0 and oracle.relres(a, b, x.cpu().numpy()) <= tol_recomputed(a.n)


def test_mixed_single_form_context(cuda):
    # A context whose own form is single-reduction keeps a standard FP64 solver
    # for the outer residual.
    from paper_1107_0538_amd import Solver

    a, b = prob(16)
    s = Solver(a, fp32_copy=True, form="single")
    x, info = s.solve_mixed(_t(b, cuda))
    assert info["status"] == 0 and oracle.relres(a, b, x.cpu().numpy()) <= tol_recomputed(a.n)
    y, i2 = s.solve(_t(b, cuda))
    assert i2["status"] == 0


def test_mixed_128_cubed(cuda):
    # The mixed-precision workload size: N = 2,097,152, nnz = 55,742,968.
    from paper_1107_0538_amd import Solver

    a, b = W.problem(128, 0)
    s = Solver(a, fp32_copy=True)
    x, info = s.solve_mixed(_t(b, cuda), tol=1e-10)
    assert info["status"] == 0, info
    assert oracle.relres(a, b, x.cpu().numpy()) <= tol_recomputed(a.n)


def test_mixed_column_index_widths_agree(cuda):
    # The FP32 inner products read the same columns with 16- or 32-bit
    # indices: the mixed solve is bitwise the same.
    from paper_1107_0538_amd import Solver

    a, b = prob(16)
    out = []
    for bits in (0, 32):
        s = Solver(a, fp32_copy=True, col_bits=bits)
        x, info = s.solve_mixed(_t(b, cuda), tol=1e-10)
        assert info["status"] == 0
        out.append((x.cpu().numpy(), info["iters"], info["outer"]))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1:] == out[1][1:]
    assert oracle.relres(a, b, out[0][0]) <= tol_recomputed(a.n)


@pytest.mark.parametrize("n", [16, 51])
def test_mixed_matrix_form_against_its_oracle(cuda, n):
    # The FP32-matrix form (FP64 iteration, FP32 values in the products,
    # reliable updates on the FP64 residual) against the oracle of the same
    # algorithm.
    from paper_1107_0538_amd import Solver

    a, b = W.problem(n, 0)
    s = Solver(a, fp32_copy=True)
    x, info = s.solve_mixed_matrix(_t(b, cuda))
    xo, io = oracle.pcg_mixed_matrix(a, b)
    xg = x.cpu().numpy()
    assert info["status"] == io["status"] == 0
    assert abs(info["iters"] - io["iters"]) <= 2, (info, io)
    assert np.linalg.norm(xg - xo) <= 1e-8 * np.linalg.norm(xo)
    assert mean_removed_relerr(xg, xo) <= 1e-8
    assert oracle.relres(a, b, xg) <= tol_recomputed(a.n)
    # and the FP64 solution, with the constant mode (barely determined by
    # the residual) removed
    x64, i64 = oracle.pcg(a, b)
    assert mean_removed_relerr(xg, x64) <= 1e-8


def test_mixed_matrix_form_full_size(cuda):
    # 128^3: converged on the recomputed FP64 residual, in the FP64 oracle's
    # iterations +-2, and within 1e-8 of the stored FP64 solution on the
    # sampled rows with the constant mode removed.
    import json
    import os

    from paper_1107_0538_amd import Solver

    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "q1hex128_oracle.json")))
    a, b = W.problem(128, 0)
    s = Solver(a, fp32_copy=True)
    x, info = s.solve_mixed_matrix(_t(b, cuda))
    xg = x.cpu().numpy()
    f = g["forms"]["standard"]
    assert info["status"] == 0 and oracle.relres(a, b, xg) <= tol_recomputed(a.n)
    rows = np.asarray(g["rows"])
    dg = xg[rows] - xg.mean()
    do = np.asarray(f["x_rows"]) - f["x_mean"]
    assert np.linalg.norm(dg - do) <= 1e-8 * np.linalg.norm(do)
    assert abs(info["iters"] - f["iters"]) <= 2, info
