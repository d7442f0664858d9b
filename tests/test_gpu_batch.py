"""Batched form: independent systems of uneven size in one persistent launch.

Each system is judged against its own FP64 oracle solve with the single-system
criteria (+-2 iterations, solution within 1e-8, true relres <= 1e-10).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from conftest import mean_removed_relerr, tol_recomputed

pytestmark = pytest.mark.gpu


def _t(a, dev):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), device=dev)


def small_batch(count=12, seed=7):
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        n = int(rng.integers(2, 17))
        a, b = W.problem(n, seed * 100 + s)
        out.append((a, b))
    return out


def check_system(a, b, x, info):
    xo, io = oracle.pcg(a, b)
    assert info["status"] == 0 and io["status"] == 0
    assert abs(info["iters"] - io["iters"]) <= 2, (info, io)
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-8
    assert mean_removed_relerr(x, xo) <= 1e-8
    assert oracle.relres(a, b, x) <= tol_recomputed(a.n)


@pytest.mark.parametrize("npl,bpc", [(4, 0), (8, 0), (16, 0), (8, 1)])
def test_small_batch_parity(cuda, npl, bpc):
    from paper_1107_0538_amd import Batch

    sys = small_batch()
    bt = Batch([a for a, _ in sys], nnz_per_lane=npl, blocks_per_cu=bpc)
    b_cat = np.concatenate([b for _, b in sys])
    x, infos = bt.solve(_t(b_cat, cuda))
    x = x.cpu().numpy()
    for s, (a, b) in enumerate(sys):
        check_system(a, b, x[bt.offsets[s]:bt.offsets[s + 1]], infos[s])
    # Deterministic and repeatable through the graph.
    x2, infos2 = bt.solve(_t(b_cat, cuda))
    assert np.array_equal(x, x2.cpu().numpy())
    assert [i["iters"] for i in infos] == [i["iters"] for i in infos2]


def test_batch_isolates_bad_systems(cuda):
    from paper_1107_0538_amd import Batch

    sys = small_batch(6, seed=3)
    bs = [b.copy() for _, b in sys]
    bs[1][:] = 0.0
    bs[4][2] = np.nan
    bt = Batch([a for a, _ in sys])
    x, infos = bt.solve(_t(np.concatenate(bs), cuda))
    x = x.cpu().numpy()
    assert infos[1]["status"] == 0 and infos[1]["iters"] == 0
    assert not x[bt.offsets[1]:bt.offsets[2]].any()
    assert infos[4]["status"] == 2
    for s in (0, 2, 3, 5):
        check_system(sys[s][0], bs[s], x[bt.offsets[s]:bt.offsets[s + 1]], infos[s])


def test_batch_rejects_bad_input(cuda):
    from paper_1107_0538_amd import Batch, capi

    a, _ = W.problem(4, 0)
    bad = W.CSR(2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32), np.array([0.0, 1.0]))
    with pytest.raises(capi.CGError):
        Batch([a, bad])
    broken = W.CSR(2, np.array([0, 1, 2], np.int32), np.array([0, 5], np.int32), np.array([1.0, 1.0]))
    with pytest.raises(ValueError):
        Batch([a, broken])


def test_batch_256_uneven_systems(cuda):
    # The batched workload: 256 systems, edge n ~ U{12..48}, seeds 1000 + s.
    from paper_1107_0538_amd import Batch

    sys = W.batch_systems(256)
    bt = Batch([a for _, a, _ in sys])
    teams, grid = bt.teams()
    assert len(teams) == 256 and min(teams) >= 1 and grid == sum(teams)
    b_cat = np.concatenate([b for _, _, b in sys])
    x, infos = bt.solve(_t(b_cat, cuda))
    x = x.cpu().numpy()
    for s, (n, a, b) in enumerate(sys):
        xs = x[bt.offsets[s]:bt.offsets[s + 1]]
        assert infos[s]["status"] == 0
        assert oracle.relres(a, b, xs) <= tol_recomputed(a.n)
    sizes = np.array([n for n, _, _ in sys])
    for s in [int(np.argmin(sizes)), int(np.argmax(sizes)), 5, 100, 200]:
        n, a, b = sys[s]
        check_system(a, b, x[bt.offsets[s]:bt.offsets[s + 1]], infos[s])


def test_batch_systems_with_replacement(cuda):
    # Systems whose solves need residual replacements at tol = 1e-10.
    from paper_1107_0538_amd import Batch

    a, _ = W.problem(16, 0)
    fam = W.amplitude_family(n=16, count=6)
    bs = list(fam.rhs(np.arange(6)))
    small, _ = W.problem(5, 1)
    mats = [a] * 6 + [small]
    bs.append(np.random.default_rng(0).uniform(-1, 1, small.n))
    bt = Batch(mats)
    x, infos = bt.solve(_t(np.concatenate(bs), cuda))
    x = x.cpu().numpy()
    for s in range(7):
        check_system(mats[s], bs[s], x[bt.offsets[s]:bt.offsets[s + 1]], infos[s])


def test_batch_autotune(cuda):
    # The tile width is chosen by timing; the result must still match the oracle.
    from paper_1107_0538_amd import Batch

    sys = small_batch(8, seed=5)
    bt = Batch([a for a, _ in sys], autotune=True)
    x, infos = bt.solve(_t(np.concatenate([b for _, b in sys]), cuda))
    x = x.cpu().numpy()
    for s, (a, b) in enumerate(sys):
        check_system(a, b, x[bt.offsets[s]:bt.offsets[s + 1]], infos[s])


def test_batch_single_and_tiny_systems(cuda):
    # One system alone, and a batch mixing 1 x 1 systems with a 3-D one.
    from paper_1107_0538_amd import Batch

    a, b = W.problem(6, 2)
    bt = Batch([a])
    x, infos = bt.solve(_t(b, cuda))
    check_system(a, b, x.cpu().numpy(), infos[0])
    one = W.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.0]))
    bt = Batch([one, a, one])
    x, infos = bt.solve(_t(np.concatenate([[4.0], b, [-6.0]]), cuda))
    x = x.cpu().numpy()
    assert infos[0]["status"] == infos[2]["status"] == 0
    assert abs(x[0] - 2.0) <= 1e-15 and abs(x[-1] + 3.0) <= 1e-15
    check_system(a, b, x[1:-1], infos[1])


def test_batch_column_index_widths(cuda):
    # 16-bit column offsets give bitwise the 32-bit results; a system whose
    # columns lie too far from its tiles' first rows falls back to 32 bits.
    import scipy.sparse as sp

    from paper_1107_0538_amd import Batch

    sys = small_batch(8, seed=5)
    b_cat = np.concatenate([b for _, b in sys])
    xs = []
    for bits in (0, 32):
        bt = Batch([a for a, _ in sys], col_bits=bits)
        x, infos = bt.solve(_t(b_cat, cuda))
        xs.append((x.cpu().numpy(), [i["iters"] for i in infos]))
    assert np.array_equal(xs[0][0], xs[1][0]) and xs[0][1] == xs[1][1]
    n = 40000
    m = sp.diags([np.full(n - 1, -1.0), np.full(n, 2.5), np.full(n - 1, -1.0)], [-1, 0, 1], format="lil")
    m[0, 32768] = m[32768, 0] = -0.25
    m = m.tocsr()
    m.sort_indices()
    wide = W.CSR(n, m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.astype(np.float64))
    bw = np.random.default_rng(6).uniform(-1, 1, n)
    sys2 = sys[:3] + [(wide, bw)]
    bt = Batch([a for a, _ in sys2])
    x, infos = bt.solve(_t(np.concatenate([b for _, b in sys2]), cuda))
    x = x.cpu().numpy()
    for s, (a, b) in enumerate(sys2):
        check_system(a, b, x[bt.offsets[s]:bt.offsets[s + 1]], infos[s])
