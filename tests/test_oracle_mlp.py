"""Pins of the oracle's probe-depth MLP (FP64): forward against an independent
numpy forward, the gradient against central finite differences of the loss,
and Adam against its first-step closed form (update = lr * g / (|g| + eps))."""
import numpy as np
import pytest


def np_forward(p, x, dims):
    i, h1, h2 = dims
    o = 0
    W1 = p[o:o + h1 * i].reshape(h1, i); o += h1 * i
    b1 = p[o:o + h1]; o += h1
    W2 = p[o:o + h2 * h1].reshape(h2, h1); o += h2 * h1
    b2 = p[o:o + h2]; o += h2
    W3 = p[o:o + h2]; o += h2
    b3 = p[o]
    a1 = np.maximum(x @ W1.T + b1, 0)
    a2 = np.maximum(a1 @ W2.T + b2, 0)
    return a2 @ W3 + b3


def rand_params(oracle, dims, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0, 0.4, size=oracle.mlp_nparams(dims))


def test_nparams(oracle):
    assert oracle.mlp_nparams() == 64 * 24 + 64 + 64 * 64 + 64 + 64 + 1 == 5825


def test_forward_matches_numpy(oracle):
    dims = (24, 64, 64)
    p = rand_params(oracle, dims, 1)
    x = np.random.default_rng(2).normal(size=(50, 24))
    assert np.allclose(oracle.mlp_forward(p, x, dims), np_forward(p, x, dims), rtol=1e-12,
                       atol=1e-12)


@pytest.mark.parametrize("dims", [(5, 7, 6), (24, 64, 64)])
def test_gradient_matches_finite_differences(oracle, dims):
    p = rand_params(oracle, dims, 3)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(9, dims[0]))
    y = rng.normal(size=9)
    loss, g = oracle.mlp_loss_grad(p, x, y, dims)
    assert loss == pytest.approx(np.mean((np_forward(p, x, dims) - y) ** 2), rel=1e-12)
    idx = np.arange(len(p)) if len(p) < 200 else rng.choice(len(p), 300, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (np.mean((np_forward(pp, x, dims) - y) ** 2) -
              np.mean((np_forward(pm, x, dims) - y) ** 2)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i


def test_adam_first_step_closed_form(oracle):
    rng = np.random.default_rng(5)
    theta = rng.normal(size=100)
    g = rng.normal(size=100)
    m = np.zeros(100)
    v = np.zeros(100)
    t0 = theta.copy()
    oracle.adam_step(theta, m, v, g, 1, lr=1e-3)
    assert np.allclose(t0 - theta, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_steps_by_lr(oracle):
    """With a constant gradient the bias-corrected ratio m/sqrt(v) is sign(g)."""
    theta = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    g = np.array([2.0, -3.0, 0.5, -0.25])
    for t in range(1, 6):
        oracle.adam_step(theta, m, v, g, t, lr=0.01, eps=0.0)
    assert np.allclose(theta, -0.05 * np.sign(g), rtol=1e-12)
