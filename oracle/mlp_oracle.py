"""FP64 NumPy oracle of the warm-start MLP (TEST INFRASTRUCTURE ONLY).

Network: 5 -> 256 -> 256 -> 256 -> 4, SiLU after the three hidden layers,
mean-squared-error loss over the 4 outputs, Adam.  Inputs are the
standardised features (Mach, log10 Re, x, y, wall distance) and outputs the
standardised targets (log rho, u/U_inf, v/U_inf, log p); see
`features` / `targets`.  Used only to check the HIP kernels' forward pass,
gradients and Adam step; the product never imports it.

Weights follow y = x W^T + b with W of shape [out, in].
"""
from __future__ import annotations

import numpy as np

SIZES = (5, 256, 256, 256, 4)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(seed, sizes=SIZES):
    """He-style uniform initialisation (the HIP library draws its own)."""
    rng = np.random.default_rng(seed)
    params = []
    for i in range(len(sizes) - 1):
        bound = np.sqrt(6.0 / sizes[i])
        W = rng.uniform(-bound, bound, size=(sizes[i + 1], sizes[i]))
        b = np.zeros(sizes[i + 1])
        params.append([W, b])
    return params


def forward(params, X):
    """Returns the output and the cached pre-activations / activations."""
    acts, pre = [X], []
    h = X
    for i, (W, b) in enumerate(params):
        z = h @ W.T + b
        pre.append(z)
        h = silu(z) if i < len(params) - 1 else z
        acts.append(h)
    return h, (acts, pre)


def loss(params, X, Y):
    out, _ = forward(params, X)
    d = out - Y
    return float(np.mean(np.sum(d * d, axis=1)))


def grads(params, X, Y):
    """Gradient of mean_n sum_k (out - Y)^2 with respect to every W and b."""
    out, (acts, pre) = forward(params, X)
    n = X.shape[0]
    g = 2.0 * (out - Y) / n
    result = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        W, _ = params[i]
        if i < len(params) - 1:
            g = g * dsilu(pre[i])
        result[i] = [g.T @ acts[i], g.sum(axis=0)]
        g = g @ W
    return result


def adam_step(params, g, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected); state = dict(t=int, m=..., v=...)."""
    state["t"] += 1
    t = state["t"]
    if "m" not in state:
        state["m"] = [[np.zeros_like(p) for p in layer] for layer in params]
        state["v"] = [[np.zeros_like(p) for p in layer] for layer in params]
    for li, layer in enumerate(params):
        for pi in range(2):
            m = state["m"][li][pi] = beta1 * state["m"][li][pi] + (1 - beta1) * g[li][pi]
            v = state["v"][li][pi] = beta2 * state["v"][li][pi] + (1 - beta2) * g[li][pi] ** 2
            mh = m / (1 - beta1 ** t)
            vh = v / (1 - beta2 ** t)
            layer[pi] = layer[pi] - lr * mh / (np.sqrt(vh) + eps)
    return params
