"""Pins of the CPU surrogate-network reference (oracle/mlp.py)."""
import math

import numpy as np

from oracle import mlp


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, 7))
    t = np.zeros((n, 4))
    t[:, 0] = rng.integers(0, 2, n)
    t[:, 1:] = rng.normal(scale=0.1, size=(n, 3))
    return x, t


def test_gradient_matches_central_differences():
    """The analytic backward pass equals central differences of the loss on
    50 random parameters of every layer (binary64, no bf16 rounding)."""
    p = mlp.init_params(3) + np.random.default_rng(4).normal(scale=0.01, size=mlp.num_params())
    x, t = _batch(12, 5)
    L, g = mlp.loss_and_grad(p, x, t, lam=3.0, delta=0.05, dmax=0.17)
    rng = np.random.default_rng(6)
    idx = rng.choice(p.size, 50, replace=False)
    # make sure every layer's weights and the last biases are represented
    offs = np.cumsum([0] + [a * b + b for a, b in zip(mlp.SIZES[:-1], mlp.SIZES[1:])])
    idx = np.concatenate([idx, offs[:-1] + 1, [p.size - 1]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_and_grad(pp, x, t, lam=3.0, delta=0.05, dmax=0.17)[0]
              - mlp.loss_and_grad(pm, x, t, lam=3.0, delta=0.05, dmax=0.17)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)), (i, fd, g[i])


def test_loss_closed_forms():
    p = np.zeros(mlp.num_params())          # all-zero network outputs y = 0
    x, t = _batch(8, 1)
    t[:, 1:] = 0.0
    L, g = mlp.loss_and_grad(p, x, t)
    assert abs(L - math.log(2.0)) < 1e-15       # BCE of logit 0 is ln 2 for either label
    # only the last bias of the logit receives gradient: mean(sigmoid(0) - esc)
    last_b = g[-4:]
    assert abs(last_b[0] - np.mean(0.5 - t[:, 0])) < 1e-15 and np.all(last_b[1:] == 0)


def test_silu_values():
    assert mlp.silu(0.0) == 0.0 and mlp.silu_grad(0.0) == 0.5
    z = np.array([-30.0, -1.0, 2.0, 30.0])
    np.testing.assert_allclose(mlp.silu(z), z / (1 + np.exp(-z)), rtol=1e-15)
    h = 1e-6
    np.testing.assert_allclose(mlp.silu_grad(z), (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h),
                               rtol=1e-8, atol=1e-12)


def test_bf16_rounding():
    vals = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -9, 1 + 2.0 ** -7 + 2.0 ** -8, -2.5,
                     0.0, 3.0e38])
    want = np.array([1.0, 1.0, 1 + 2.0 ** -7, 1 + 2.0 ** -6, -2.5, 0.0, 226 / 128 * 2.0 ** 127])
    got = mlp.bf16(vals)
    np.testing.assert_array_equal(got, want)
    assert got[1] == 1.0 and got[2] == 1 + 2.0 ** -7 and got[3] == 1 + 2.0 ** -6  # ties to even


def test_adam_first_step_is_signed_learning_rate():
    """At t = 1 the bias-corrected Adam step is lr * g/|g| (up to eps)."""
    rng = np.random.default_rng(2)
    p = rng.normal(size=100)
    g = rng.normal(size=100)
    new, m, v = mlp.adam_step(p, g, np.zeros(100), np.zeros(100), 1, lr=1e-3, eps=0.0)
    np.testing.assert_allclose(new, p - 1e-3 * np.sign(g), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=4e-15)   # 1 - 0.999 is not exactly 1e-3


def test_bf16_mode_stays_close_to_binary64():
    p = mlp.init_params(9)
    x, t = _batch(64, 8)
    y64 = mlp.forward(p, x)
    y16 = mlp.forward(p, x, bf16_mode=True)
    assert np.linalg.norm(y16 - y64) / np.linalg.norm(y64) < 2e-2


def test_huber_is_squared_error_inside_and_linear_outside():
    e = np.array([-0.3, -0.05, 0.0, 0.02, 0.05, 1.0])
    np.testing.assert_allclose(mlp.huber(e, np.inf), e * e)
    np.testing.assert_allclose(mlp.huber(e, 0.05), [0.0275, 0.0025, 0.0, 0.0004, 0.0025, 0.0975])
    np.testing.assert_allclose(mlp.huber_grad(e, 0.05), [-0.1, -0.1, 0.0, 0.04, 0.1, 0.1])


def test_direction_loss_skips_rows_beyond_dmax():
    """Rows whose target correction is longer than dmax contribute only their
    class term: their loss equals that of the same rows with lam = 0."""
    p = mlp.init_params(5) + np.random.default_rng(6).normal(scale=0.01, size=mlp.num_params())
    x, t = _batch(16, 7)
    t[:, 0] = 1.0
    t[:8, 1:] = 2.0                                       # |d| = 3.46 > dmax
    Lmask, gmask = mlp.loss_and_grad(p, x, t, lam=5.0, delta=0.05, dmax=1.0)
    keep = np.r_[8:16]
    Lk, gk = mlp.loss_and_grad(p, x[keep], t[keep], lam=5.0, delta=0.05)
    Ld, gd = mlp.loss_and_grad(p, x[:8], t[:8], lam=0.0)
    assert abs(Lmask - (Lk * 8 + Ld * 8) / 16) < 1e-12
    np.testing.assert_allclose(gmask, (gk * 8 + gd * 8) / 16, rtol=1e-9, atol=1e-15)
