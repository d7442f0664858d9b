"""The Q1 operator built on the device from element coefficients: the
matrix-free product q1_apply and the device assembly q1_assemble.

The product is compared with the element-by-element oracle (oracle/q1.py)
row by row within 1e-12 of sum_j |a_ij x_j| (rows cancel: A 1 is only the
small mass term); the assembled matrix with the host generator's (same
pattern bitwise, entries within a few units of rounding: the two compute
h^3 and the mass weights along different paths); and the product bitwise
with the sequential product of the assembled matrix.
"""
import numpy as np
import pytest

import oracle
import oracle.q1 as oq1
import workloads as W
from conftest import mean_removed_relerr, tol_recomputed

pytestmark = pytest.mark.gpu


def _sigma(n, seed):
    return np.exp(np.random.default_rng(seed).standard_normal((n - 1,) * 3))


def _row_bound(a, x):
    rows = np.repeat(np.arange(a.n), np.diff(a.rowptr))
    return np.bincount(rows, weights=np.abs(a.val * x[a.col]), minlength=a.n)


@pytest.mark.parametrize("n", [2, 3, 5, 16, 51])
def test_q1_apply_matches_elementwise_oracle(cuda, n):
    import torch

    from paper_1107_0538_amd import q1_apply

    sig = _sigma(n, n)
    x = np.random.default_rng(n + 1).uniform(-1, 1, n ** 3)
    y = q1_apply(n, torch.as_tensor(sig, device=cuda), torch.as_tensor(x, device=cuda)).cpu().numpy()
    yo = oq1.apply(n, sig, 1e-3, x)
    a = W.assemble(n, sig)
    assert np.all(np.abs(y - yo) <= 1e-12 * _row_bound(a, x))
    assert np.linalg.norm(y - yo) <= 1e-12 * np.linalg.norm(yo)


def test_q1_apply_full_size(cuda):
    # 128^3 (N = 2,097,152): every row against the element-by-element oracle,
    # the rounding scale of each row bounded element by element.
    import torch

    from paper_1107_0538_amd import q1_apply

    n = 128
    sig = _sigma(n, 5)
    x = np.random.default_rng(6).uniform(-1, 1, n ** 3)
    y = q1_apply(n, torch.as_tensor(sig, device=cuda), torch.as_tensor(x, device=cuda)).cpu().numpy()
    yo = oq1.apply(n, sig, 1e-3, x)
    bound = oq1.abs_row_bound(n, sig, 1e-3, x)
    assert np.all(np.abs(y - yo) <= 1e-12 * bound)
    assert np.linalg.norm(y - yo) <= 1e-12 * np.linalg.norm(yo)


@pytest.mark.parametrize("n", [2, 4, 16, 51])
def test_q1_assemble_matches_generator(cuda, n):
    import torch

    from paper_1107_0538_amd import q1_assemble

    sig = _sigma(n, 10 + n)
    m = q1_assemble(n, torch.as_tensor(sig, device=cuda))
    a = W.assemble(n, sig)
    assert np.array_equal(m.rowptr.cpu().numpy(), a.rowptr)
    assert np.array_equal(m.col.cpu().numpy(), a.col)
    val = m.val.cpu().numpy()
    # Both sum at most 8 element terms per entry, in different orders and
    # groupings: a few tens of units of rounding at most.
    assert np.all(np.abs(val - a.val) <= 32 * 2.0 ** -53 * np.abs(a.val) + 1e-300)


def test_q1_apply_is_the_assembled_product_bitwise(cuda):
    import torch

    from paper_1107_0538_amd import Solver, q1_apply, q1_assemble

    n = 16
    sig = torch.as_tensor(_sigma(n, 1), device=cuda)
    x = torch.as_tensor(np.random.default_rng(2).standard_normal(n ** 3), device=cuda)
    m = q1_assemble(n, sig)
    y = q1_apply(n, sig, x).cpu().numpy()
    host = W.CSR(m.n, m.rowptr.cpu().numpy(), m.col.cpu().numpy(), m.val.cpu().numpy())
    assert np.array_equal(y, oracle.spmv(host, x.cpu().numpy()))
    # The device CSR goes straight into a solver context (no host copy).
    s = Solver(m)
    assert np.array_equal(s.spmv(x).cpu().numpy(), y)


def test_solve_on_device_assembled_system(cuda):
    import torch

    from paper_1107_0538_amd import Solver, q1_assemble

    n = 16
    sig = np.exp(np.random.default_rng(0).standard_normal((n - 1,) * 3))
    m = q1_assemble(n, torch.as_tensor(sig, device=cuda))
    host = W.CSR(m.n, m.rowptr.cpu().numpy(), m.col.cpu().numpy(), m.val.cpu().numpy())
    b = np.random.default_rng(1).uniform(-1, 1, host.n)
    x, info = Solver(m).solve(torch.as_tensor(b, device=cuda))
    xo, io = oracle.pcg(host, b)
    xg = x.cpu().numpy()
    assert info["status"] == io["status"] == 0 and abs(info["iters"] - io["iters"]) <= 2
    assert np.linalg.norm(xg - xo) <= 1e-8 * np.linalg.norm(xo)
    assert mean_removed_relerr(xg, xo) <= 1e-8
    assert oracle.relres(host, b, xg) <= tol_recomputed(host.n)


def test_q1_arguments_rejected(cuda):
    import torch

    from paper_1107_0538_amd import capi, q1_apply

    sig = torch.ones(8, dtype=torch.float64, device=cuda)
    x = torch.ones(27, dtype=torch.float64, device=cuda)
    with pytest.raises(ValueError):
        q1_apply(3, sig[:7], x)
    with pytest.raises(ValueError):
        q1_apply(1, sig, x)
    lib = capi.load()
    assert lib.q1_apply(3, 1e-3, sig.data_ptr(), x.data_ptr(), x.data_ptr(), None) == capi.CG_EINVAL
    assert lib.q1_apply(3, -1.0, sig.data_ptr(), x.data_ptr(), sig.data_ptr(), None) == capi.CG_EINVAL
    assert lib.q1_assemble(2000, 1e-3, sig.data_ptr(), x.data_ptr(), x.data_ptr(), x.data_ptr(), None) == capi.CG_EINVAL
