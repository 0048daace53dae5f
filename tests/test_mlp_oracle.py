"""Pins of the MLP oracle: backward pass vs central finite differences (FP64),
and Adam's first step against its closed form."""
import numpy as np

from oracle import mlp_oracle as M


def test_backward_matches_central_differences():
    sizes = (5, 7, 6, 5, 4)
    p = M.init_params(3, sizes)
    rng = np.random.default_rng(4)
    X, Y = rng.normal(size=(9, 5)), rng.normal(size=(9, 4))
    g = M.grads(p, X, Y)
    h = 1e-6
    for li in range(len(p)):
        for pi in range(2):
            a = p[li][pi]
            idx = [tuple(rng.integers(0, s) for s in a.shape) for _ in range(6)]
            for ix in idx:
                old = a[ix]
                a[ix] = old + h
                lp = M.loss(p, X, Y)
                a[ix] = old - h
                lm = M.loss(p, X, Y)
                a[ix] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[li][pi][ix]) <= 1e-7 * max(1.0, abs(fd))


def test_adam_first_step_is_sign_step():
    p = M.init_params(0, (5, 4, 4))
    g = [[np.full_like(W, 0.3), np.full_like(b, -2.0)] for W, b in p]
    before = [[x.copy() for x in layer] for layer in p]
    M.adam_step(p, g, {"t": 0}, lr=1e-2)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> update = lr * sign(g) (up to eps)
    for layer, old in zip(p, before):
        np.testing.assert_allclose(layer[0] - old[0], -1e-2 * np.ones_like(old[0]), rtol=1e-6)
        np.testing.assert_allclose(layer[1] - old[1], 1e-2 * np.ones_like(old[1]), rtol=1e-6)


def test_silu_derivative():
    z = np.linspace(-5, 5, 41)
    fd = (M.silu(z + 1e-6) - M.silu(z - 1e-6)) / 2e-6
    np.testing.assert_allclose(M.dsilu(z), fd, rtol=1e-8, atol=1e-10)
