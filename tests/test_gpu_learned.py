"""Learned warm start on the GPU: dense products, the MLP's forward, gradients
and Adam step against the FP64 oracle, and the whole pipeline.

Tolerances: FP32 network 1e-5 relative (normwise per tensor); BF16 network
2e-2 (weights and hidden activations rounded to 8 significant bits, FP32
accumulation); dense FP64 products 1e-13 relative.
"""
import numpy as np
import pytest

import oracle
import oracle.mlp as om
import oracle.pod as op
import workloads as W
from conftest import mean_removed_relerr, tol_recomputed

pytestmark = pytest.mark.gpu

DIMS = [24, 256, 256, 64]


def _t(a, dev, dtype=None):
    import torch

    t = torch.as_tensor(np.ascontiguousarray(a), device=dev)
    return t if dtype is None else t.to(dtype)


def relnorm(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("n,ka,kb", [(5000, 64, 64), (70001, 100, 37), (1, 3, 2), (2048 * 3 + 5, 130, 65)])
def test_dense_gram(cuda, n, ka, kb):
    from paper_1107_0538_amd import learned

    rng = np.random.default_rng(n + ka)
    A = rng.standard_normal((n, ka))
    B = rng.standard_normal((n, kb))
    C = learned.dense_gram(_t(A, cuda), _t(B, cuda)).cpu().numpy()
    assert relnorm(C, A.T @ B) <= 1e-13
    # Deterministic.
    C2 = learned.dense_gram(_t(A, cuda), _t(B, cuda)).cpu().numpy()
    assert np.array_equal(C, C2)


def test_dense_gram_strided(cuda):
    from paper_1107_0538_amd import learned

    rng = np.random.default_rng(1)
    S = rng.standard_normal((3000, 90))
    Sd = _t(S, cuda)
    C = learned.dense_gram(Sd[:, :40], Sd[:, 50:]).cpu().numpy()
    assert relnorm(C, S[:, :40].T @ S[:, 50:]) <= 1e-13


@pytest.mark.parametrize("n,k,m", [(10000, 500, 64), (777, 17, 3), (64, 64, 64)])
def test_dense_gemm(cuda, n, k, m):
    from paper_1107_0538_amd import learned

    rng = np.random.default_rng(n + k + m)
    A = rng.standard_normal((n, k))
    Wm = rng.standard_normal((k, m))
    C = learned.dense_gemm(_t(A, cuda), _t(Wm, cuda)).cpu().numpy()
    assert relnorm(C, A @ Wm) <= 1e-13


@pytest.mark.parametrize("nb", [1, 5])
def test_pod_decode(cuda, nb):
    from paper_1107_0538_amd import learned

    rng = np.random.default_rng(nb)
    Phi = rng.standard_normal((20001, 64))
    coef = rng.standard_normal((nb, 64)).astype(np.float32)
    scale = rng.uniform(0.5, 2.0, 64)
    shift = rng.standard_normal(64)
    X = learned.pod_decode(_t(Phi, cuda), _t(coef, cuda), scale=_t(scale, cuda), shift=_t(shift, cuda))
    ref = Phi @ (coef.astype(np.float64) * scale + shift).T
    assert relnorm(X.cpu().numpy(), ref) <= 1e-13
    X0 = learned.pod_decode(_t(Phi, cuda), _t(coef, cuda)).cpu().numpy()
    assert relnorm(X0, Phi @ coef.astype(np.float64).T) <= 1e-13


def _net_case(batch, seed=0):
    rng = np.random.default_rng(seed)
    params = om.init_params(DIMS, seed)
    params = [(W.astype(np.float32).astype(np.float64), rng.uniform(-0.1, 0.1, b.size).astype(np.float32)
               .astype(np.float64)) for W, b in params]
    X = rng.uniform(-1, 1, (batch, DIMS[0])).astype(np.float32)
    T = rng.standard_normal((batch, DIMS[-1])).astype(np.float32)
    return params, X, T


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16", 2e-2)])
@pytest.mark.parametrize("batch", [256, 77, 1])
def test_mlp_forward_and_gradients(cuda, precision, tol, batch):
    from paper_1107_0538_amd import learned

    params, X, T = _net_case(batch)
    net = learned.MLP(DIMS, precision, max_batch=512)
    net.set_params(om.flatten(params))
    assert net.nparam == 88640
    Y = net.forward(_t(X, cuda)).cpu().numpy()
    Yo, cache = om.forward(params, X.astype(np.float64))
    assert relnorm(Y, Yo) <= tol
    g, loss = net.gradients(_t(X, cuda), _t(T, cuda))
    go = om.backward(params, cache, Yo, T.astype(np.float64))
    lo = om.loss(Yo, T.astype(np.float64))
    assert abs(loss - lo) <= tol * lo
    gv = learned.layer_views(g.astype(np.float64), DIMS)
    for l, ((gW, gb), (oW, ob)) in enumerate(zip(gv, go)):
        assert relnorm(gW, oW) <= tol, (l, "W")
        assert relnorm(gb, ob) <= tol, (l, "b")


def test_mlp_adam_steps(cuda):
    from paper_1107_0538_amd import learned

    params, X, T = _net_case(128, seed=4)
    net = learned.MLP(DIMS, "fp32", max_batch=128)
    net.set_params(om.flatten(params))
    opt = om.Adam(params, lr=1e-3)
    p = params
    for step in range(3):
        before = net.get_params().astype(np.float64)
        net.train_step(_t(X, cuda), _t(T, cuda), lr=1e-3)
        after = net.get_params().astype(np.float64)
        Yo, cache = om.forward(p, X.astype(np.float64))
        go = om.backward(p, cache, Yo, T.astype(np.float64))
        p = opt.step(p, go)
        ref = om.flatten(p)
        # Compare the updates where the gradient is well above FP32 noise.
        gflat = om.flatten(go)
        big = np.abs(gflat) > 1e-3 * np.abs(gflat).max()
        d_gpu, d_ref = after - before, ref - before
        assert relnorm(d_gpu[big], d_ref[big]) <= 1e-3, step
        # Elsewhere the two trajectories may differ by at most a few steps of size lr.
        assert np.max(np.abs(after - ref)) <= 4e-3 * (step + 1)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("bf16", 5e-2)])
def test_mlp_training_tracks_oracle(cuda, precision, tol):
    # 600 Adam steps on a smooth 24 -> 64 map from the same initial weights:
    # the GPU's training loss follows the FP64 oracle's trajectory.
    from paper_1107_0538_amd import learned

    rng = np.random.default_rng(3)
    M = rng.standard_normal((24, 64)) / np.sqrt(24)
    X = rng.uniform(-1, 1, (1024, 24)).astype(np.float32)
    T = np.tanh(X.astype(np.float64) @ M).astype(np.float32)
    flat = learned.he_uniform(DIMS, 0)
    net = learned.MLP(DIMS, precision, max_batch=256)
    net.set_params(flat)
    Xd, Td = _t(X, cuda), _t(T, cuda)
    p = [(W.copy(), b.copy()) for W, b in learned.layer_views(flat.astype(np.float64), DIMS)]
    opt = om.Adam(p, lr=1e-3)
    X64, T64 = X.astype(np.float64), T.astype(np.float64)
    first = net.gradients(Xd[:256], Td[:256])[1]
    for ep in range(150):
        for i in range(4):
            sl = slice(i * 256, (i + 1) * 256)
            net.train_step(Xd[sl], Td[sl], lr=1e-3)
            Yo, cache = om.forward(p, X64[sl])
            p = opt.step(p, om.backward(p, cache, Yo, T64[sl]))
    last = net.gradients(Xd[:256], Td[:256])[1]
    last_o = om.loss(om.forward(p, X64[:256])[0], T64[:256])
    assert last < 0.05 * first, (first, last)
    assert abs(last - last_o) <= tol * last_o, (last, last_o)


def test_mlp_rejects_bad_input(cuda):
    from paper_1107_0538_amd import capi, learned

    with pytest.raises(ValueError):
        learned.MLP([24, 0, 64], "fp32")
    net = learned.MLP([4, 8, 2], "fp32", max_batch=8)
    with pytest.raises(ValueError):
        net.forward(_t(np.zeros((9, 4), np.float32), cuda))
    with pytest.raises(ValueError):
        net.set_params(np.zeros(3, np.float32))
    lib = capi.load()
    assert lib.mlp_forward(None, None, 1, None) == capi.CG_EINVAL


def test_learned_warm_start_gain(cuda):
    # On a family whose solutions lie in a 4-dimensional space the learned
    # start vector must cut CG iterations against x0 = 0 on held-out samples.
    # Bar: the paired saving (iterations from x0 = 0 minus from the learned
    # start, per held-out right-hand side) has a mean larger than three of its
    # standard errors, i.e. the gain is real, not noise of the sample.  The
    # test also measures what the start is worth: the iterations CG from
    # x0 = 0 needs to reach the start's residual (its residual history); CG
    # restarted from the start keeps only part of that, because it rebuilds
    # the Krylov space (about 19 of 92 iterations here).
    import torch
    from paper_1107_0538_amd import Solver, learned

    n = 16
    a, _ = W.problem(n, 0)
    fam = W.amplitude_family(n=n, count=400, k=4, seed=11)
    s = Solver(a, history=True)
    ws = learned.LearnedWarmStart(s, fam, n_pod=100, n_train=300, modes=4, hidden=(64, 64), precision="fp32",
                                  seed=0).fit(epochs=1500, batch=100)
    assert ws.loss_curve[-1][1] < 1e-2
    B = fam.rhs(np.arange(300, 400))
    its0, its1, worth = [], [], []
    for j, i in enumerate(range(300, 400)):
        b = _t(B[j], cuda)
        x0 = ws.x0(fam.theta()[i:i + 1]).reshape(-1)
        r_start = oracle.relres(a, B[j], x0.cpu().numpy())
        x, info = s.solve(b, x0=x0.clone())
        assert info["status"] == 0 and oracle.relres(a, B[j], x.cpu().numpy()) <= tol_recomputed(a.n)
        _, info0 = s.solve(b)
        hist = s.history()
        reach = np.flatnonzero(hist <= r_start)
        worth.append(int(reach[0]) if reach.size else len(hist) - 1)
        its0.append(info0["iters"])
        its1.append(info["iters"])
    d = np.asarray(its0, float) - np.asarray(its1, float)
    stderr = d.std(ddof=1) / np.sqrt(d.size)
    assert d.mean() > 3.0 * stderr, (np.mean(its0), np.mean(its1), np.mean(worth), stderr)
    assert 0 < d.mean() <= np.mean(worth)
    print(f"learned start: {np.mean(its0):.1f} -> {np.mean(its1):.1f} iterations; worth {np.mean(worth):.1f}")
    torch.cuda.synchronize()


def test_network_inputs_are_the_training_inputs(cuda):
    # Inference feeds the network exactly the inputs training used (2 theta - 1
    # in FP32, rounded to BF16 inside the forward pass), so a BF16 network's
    # prediction equals its forward pass on the training inputs bit for bit.
    import torch
    from paper_1107_0538_amd import Solver, learned

    n = 8
    a, _ = W.problem(n, 0)
    fam = W.source_family(n=n, count=64, k=8, seed=3)
    ws = learned.LearnedWarmStart(Solver(a), fam, n_pod=16, n_train=48, modes=8, hidden=(32, 32),
                                  precision="bf16").fit(epochs=3, batch=16)
    th = fam.theta()[48:64]
    X = torch.as_tensor((2.0 * th - 1.0).astype(np.float32), device=cuda)
    assert torch.equal(ws.predict(th), ws.net.forward(X))


def test_learned_pipeline_source_family(cuda):
    # The source-term family at a reduced size: the POD basis is orthonormal,
    # its Gram eigenvalues match the oracle's, and CG from the network's start
    # vector converges to the same tolerance.
    from paper_1107_0538_amd import Solver, learned

    n = 16
    a, _ = W.problem(n, 0)
    fam = W.source_family(n=n, count=240, k=8, seed=3)
    s = Solver(a)
    ws = learned.LearnedWarmStart(s, fam, n_pod=100, n_train=200, modes=16, hidden=(64, 64), precision="bf16")
    ws.fit(epochs=50, batch=100)
    Phi = ws.Phi.cpu().numpy()
    Xo = np.stack([oracle.pcg(a, fam.rhs(i)[0])[0] for i in range(100)], axis=1)
    _, lam_o = op.modes(Xo, 16)
    # Orthonormal up to the method of snapshots' own error: an eigenvector of
    # the Gram matrix is accurate to ~u lambda_1 / gap, and dividing by
    # sqrt(lambda_i) amplifies it, so the bound scales with lambda_1 / lambda_i.
    lam = ws.energy
    bound = 1e3 * np.finfo(float).eps * lam[0] / np.minimum.outer(lam, lam)
    assert np.all(np.abs(Phi.T @ Phi - np.eye(16)) <= bound)
    # First-order eigenvalue perturbation is bounded by ||dG|| ~ 2 ||S|| ||dS||.
    assert np.max(np.abs(ws.energy - lam_o[:16])) <= 1e-6 * lam_o[0]
    for i in (200, 239):
        b = fam.rhs(i)[0]
        x0 = ws.x0(fam.theta()[i:i + 1]).reshape(-1)
        x, info = s.solve(_t(b, cuda), x0=x0.clone())
        assert info["status"] == 0 and oracle.relres(a, b, x.cpu().numpy()) <= tol_recomputed(a.n)
