"""Pins for the MLP and POD oracles (learned warm start), against things other than themselves.

MLP: gradients against central finite differences of the loss; SiLU's
derivative against a finite difference; one Adam step against its closed form
(the first step moves every parameter by about -lr * sign(g)); a short
training run reduces the loss.  POD: orthonormal modes, eigenvalues equal to
the squared singular values from an SVD, and the projection error equal to
the discarded energy.
"""
import numpy as np
import pytest

from oracle import mlp, pod


def test_silu_derivative():
    u = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp.silu(u + h) - mlp.silu(u - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.silu_grad(u))) <= 1e-8


@pytest.mark.parametrize("dims", [[3, 5, 4], [4, 7, 6, 2]])
def test_gradients_match_finite_differences(dims):
    rng = np.random.default_rng(1)
    params = mlp.init_params(dims, seed=2)
    params = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in params]
    X = rng.standard_normal((5, dims[0]))
    T = rng.standard_normal((5, dims[-1]))
    Y, cache = mlp.forward(params, X)
    g = mlp.flatten(mlp.backward(params, cache, Y, T))
    p0 = mlp.flatten(params)
    h = 1e-6
    fd = np.empty_like(p0)
    for i in range(p0.size):
        pp, pm = p0.copy(), p0.copy()
        pp[i] += h
        pm[i] -= h
        lp = mlp.loss(mlp.forward(mlp.unflatten(pp, dims), X)[0], T)
        lm = mlp.loss(mlp.forward(mlp.unflatten(pm, dims), X)[0], T)
        fd[i] = (lp - lm) / (2 * h)
    assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g)


def test_adam_first_step_closed_form():
    params = [(np.array([[1.0, -2.0]]), np.array([0.5]))]
    grads = [(np.array([[0.3, -4.0]]), np.array([1e-3]))]
    opt = mlp.Adam(params, lr=0.01)
    new = opt.step(params, grads)
    # t = 1: m_hat = g, v_hat = g^2, step = lr * g / (|g| + eps).
    assert np.allclose(new[0][0], [[1.0 - 0.01, -2.0 + 0.01]], rtol=0, atol=1e-9)
    assert np.allclose(new[0][1], [0.5 - 0.01 * 1e-3 / (1e-3 + 1e-8)], rtol=0, atol=1e-12)


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    dims = [3, 16, 16, 2]
    params = mlp.init_params(dims, seed=4)
    X = rng.uniform(-1, 1, (64, 3))
    T = np.stack([np.sin(X[:, 0]) + X[:, 1] * X[:, 2], X[:, 0] ** 2], axis=1)
    opt = mlp.Adam(params, lr=1e-2)
    l0 = mlp.loss(mlp.forward(params, X)[0], T)
    for _ in range(300):
        Y, cache = mlp.forward(params, X)
        params = opt.step(params, mlp.backward(params, cache, Y, T))
    assert mlp.loss(mlp.forward(params, X)[0], T) <= 0.05 * l0


def test_pod_modes():
    rng = np.random.default_rng(5)
    N, m, k = 300, 40, 8
    S = rng.standard_normal((N, 6)) @ rng.standard_normal((6, m)) * 3 + 0.01 * rng.standard_normal((N, m))
    Phi, lam = pod.modes(S, k)
    # Forming S'S squares the conditioning: mode i is orthonormal to about
    # u * lambda_1 / lambda_i.
    err = np.abs(Phi.T @ Phi - np.eye(k))
    bound = 1e3 * np.finfo(float).eps * lam[0] / np.minimum.outer(lam[:k], lam[:k])
    assert np.all(err <= bound)
    assert np.max(err[:6, :6]) <= 1e-12
    sv = np.linalg.svd(S, compute_uv=False)
    assert np.allclose(lam[:m], sv ** 2, rtol=1e-8, atol=1e-10 * sv[0] ** 2)
    resid = S - Phi @ (Phi.T @ S)
    assert abs(np.sum(resid ** 2) - np.sum(lam[k:])) <= 1e-8 * np.sum(lam)


def test_pod_project_and_decode():
    # For an orthonormal basis Q (from a QR factorisation): coefficients of a
    # combination Q C are C; decoding the coefficients of a vector in the span
    # returns it; unit coefficient vectors decode to the basis vectors, and a
    # unit vector of R^N projects onto that row of the basis.
    rng = np.random.default_rng(6)
    N, k, m = 200, 7, 5
    Q, _ = np.linalg.qr(rng.standard_normal((N, k)))
    C = rng.standard_normal((k, m))
    assert pod.project(Q, Q @ C).shape == (k, m)
    assert np.max(np.abs(pod.project(Q, Q @ C) - C)) <= 1e-13
    S = Q @ rng.standard_normal((k, m))
    assert np.max(np.abs(pod.decode(Q, pod.project(Q, S)) - S)) <= 1e-13
    assert np.array_equal(pod.decode(Q, np.eye(k)), Q)
    for i in (0, 3, N - 1):
        e = np.zeros((N, 1))
        e[i] = 1.0
        assert np.array_equal(pod.project(Q, e)[:, 0], Q[i])
    # Orthogonal complement: a vector orthogonal to the span has zero coefficients.
    v0 = rng.standard_normal(N)
    v = v0 - Q @ (Q.T @ v0)
    assert np.max(np.abs(pod.project(Q, v[:, None]))) <= 1e-13 * np.linalg.norm(v0)
