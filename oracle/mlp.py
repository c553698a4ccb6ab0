"""The learned flexible preconditioner's network, FP64 (no paper passage: the
paper's FGMRES admits any nonlinear preconditioner M_j, section 4.2).

Layers: x -> h_1 = gelu(W_1 x + b_1) -> ... -> h_L = gelu(...) -> W_out h_L + b_out,
GELU in its exact erf form gelu(x) = x (1 + erf(x / sqrt 2)) / 2.
Weights W_i are [out, in]; a batch X is [B, in].  Loss = mean of squared
errors over all B * out entries.
"""
import math

import numpy as np
from scipy.special import erf


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def init(sizes, rng):
    params = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        params.append([rng.standard_normal((b, a)) / math.sqrt(a), np.zeros(b)])
    return params


def forward(params, X):
    """Returns (output, cache of pre-activations and inputs per layer)."""
    cache = []
    h = X
    for li, (W, b) in enumerate(params):
        z = h @ W.T + b
        cache.append((h, z))
        h = gelu(z) if li < len(params) - 1 else z
    return h, cache


def mse(out, Y):
    return float(np.mean((out - Y) ** 2))


def backward(params, cache, out, Y):
    """Gradients of mse(out, Y) with respect to every W_i and b_i."""
    n = out.size
    d = 2.0 * (out - Y) / n
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        h, z = cache[li]
        if li < len(params) - 1:
            d = d * gelu_grad(z)
        grads[li] = [d.T @ h, d.sum(0)]
        d = d @ W
    return grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) in place; state holds (t, m, v)."""
    if not state:
        state["t"] = 0
        state["m"] = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
        state["v"] = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
    state["t"] += 1
    t = state["t"]
    for (p, g, m, v) in zip(params, grads, state["m"], state["v"]):
        for k in range(2):
            m[k] = b1 * m[k] + (1 - b1) * g[k]
            v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
            mh = m[k] / (1 - b1 ** t)
            vh = v[k] / (1 - b2 ** t)
            p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
