"""FP64 multilayer-perceptron oracle -- TEST INFRASTRUCTURE ONLY.

The learned warm start maps source parameters theta to POD coefficients with a
fully connected network: hidden layers h = silu(W h_prev + b), a linear output
layer, mean-squared-error loss over all outputs of a batch, and Adam
(Kingma and Ba, 2015) on the parameters.  This module writes those
definitions out plainly in numpy FP64 for the GPU kernels to be checked
against; it shares nothing with the GPU library.

Conventions (shared with the GPU path's documentation):
  W_l has shape (out, in), b_l shape (out,); a batch X has shape (B, in).
  loss = sum((Y - T)^2) / (B * out).
  silu(u) = u * sigmoid(u).
  Adam: m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
        p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np


def sigmoid(u):
    return 1.0 / (1.0 + np.exp(-u))


def silu(u):
    return u * sigmoid(u)


def silu_grad(u):
    s = sigmoid(u)
    return s * (1.0 + u * (1.0 - s))


def init_params(dims, seed=0):
    """He-style uniform initialisation, FP64: list of (W, b)."""
    rng = np.random.default_rng(seed)
    params = []
    for fan_in, fan_out in zip(dims[:-1], dims[1:]):
        bound = np.sqrt(6.0 / fan_in) / 2.0
        params.append((rng.uniform(-bound, bound, (fan_out, fan_in)), np.zeros(fan_out)))
    return params


def forward(params, X):
    """Returns (Y, cache) with cache = list of (input, pre-activation) per layer."""
    h = np.asarray(X, dtype=np.float64)
    cache = []
    for l, (W, b) in enumerate(params):
        u = h @ W.T + b
        cache.append((h, u))
        h = u if l == len(params) - 1 else silu(u)
    return h, cache


def loss(Y, T):
    return float(np.sum((Y - T) ** 2) / Y.size)


def backward(params, cache, Y, T):
    """Gradients of loss with respect to every (W, b), same structure as params."""
    d = 2.0 * (Y - T) / Y.size  # dL/dY
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        h, u = cache[l]
        if l != len(params) - 1:
            d = d * silu_grad(u)
        grads[l] = (d.T @ h, d.sum(axis=0))
        d = d @ W
    return grads


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]

    def step(self, params, grads):
        self.t += 1
        out = []
        for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for i, (p, g) in enumerate(((W, gW), (b, gb))):
                m = self.b1 * self.m[l][i] + (1 - self.b1) * g
                v = self.b2 * self.v[l][i] + (1 - self.b2) * g * g
                mh = m / (1 - self.b1 ** self.t)
                vh = v / (1 - self.b2 ** self.t)
                new.append(p - self.lr * mh / (np.sqrt(vh) + self.eps))
                if i == 0:
                    mW, vW = m, v
                else:
                    self.m[l] = (mW, m)
                    self.v[l] = (vW, v)
            out.append(tuple(new))
        return out


def flatten(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def unflatten(vec, dims):
    params, o = [], 0
    for fan_in, fan_out in zip(dims[:-1], dims[1:]):
        W = vec[o:o + fan_in * fan_out].reshape(fan_out, fan_in)
        o += fan_in * fan_out
        b = vec[o:o + fan_out]
        o += fan_out
        params.append((W.copy(), b.copy()))
    return params
