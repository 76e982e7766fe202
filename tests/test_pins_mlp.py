"""Pins of the MLP oracle: GELU special values and identities, analytic
gradients against central finite differences, and Adam's first step."""
import numpy as np
from scipy.stats import norm

from oracle import mlp


def test_gelu_closed_forms():
    x = np.linspace(-6, 6, 241)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    # GELU(x) - GELU(-x) = x, and GELU(x) = x Phi(x) with the normal CDF
    assert np.allclose(mlp.gelu(x) - mlp.gelu(-x), x, atol=1e-14)
    assert np.allclose(mlp.gelu(x), x * norm.cdf(x), atol=1e-14)
    # derivative at 0 is 1/2; derivative by finite differences elsewhere
    assert abs(mlp.gelu_prime(np.array([0.0]))[0] - 0.5) < 1e-15
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(mlp.gelu_prime(x), fd, atol=1e-8)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init_params(rng) + 0.05 * rng.standard_normal(mlp.N_PARAM)
    X = rng.standard_normal((7, mlp.N_IN))
    T = rng.standard_normal((7, mlp.N_OUT))
    g = mlp.grad(theta, X, T)
    idx = rng.choice(mlp.N_PARAM, 120, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.N_PARAM)
        e[i] = h
        fd = (mlp.loss(theta + e, X, T) - mlp.loss(theta - e, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_linear_special_case():
    """With W1 = W2 = 0 the hidden layers are GELU(b) constants and the
    output is W3 GELU(b2) + b3 for every input."""
    theta = np.zeros(mlp.N_PARAM)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(theta)
    b2[:] = np.linspace(-1, 1, mlp.N_H)
    rng = np.random.default_rng(1)
    W3[:] = rng.standard_normal(W3.shape)
    b3[:] = rng.standard_normal(b3.shape)
    Y, _ = mlp.forward(theta, rng.standard_normal((5, mlp.N_IN)))
    ref = W3 @ mlp.gelu(b2) + b3
    assert np.allclose(Y, ref[None, :], atol=1e-14)


def test_adam_first_step_is_signed_lr():
    """At t = 1 bias correction makes the step lr * g / (|g| + eps')."""
    g = np.array([3.0, -2.0, 1e-3, 0.0])
    th, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(th[:3], -0.01 * np.sign(g[:3]), rtol=1e-5)
    assert th[3] == 0.0


def test_bf16_rounding_values():
    """Round-to-nearest-even onto the bfloat16 grid (8 significand bits):
    exact grid values stay, halfway cases go to the even neighbour."""
    b = mlp.bf16
    assert b(1.0) == 1.0 and b(-2.5) == -2.5 and b(0.0) == 0.0
    u = 2.0 ** -7                                   # bf16 spacing just above 1
    assert b(1.0 + u / 2) == 1.0                    # tie -> even (1.0)
    assert b(1.0 + 3 * u / 2) == 1.0 + 2 * u        # tie -> even (1 + 2u)
    assert b(1.0 + 0.6 * u) == 1.0 + u
    assert b(2.0 - 2.0 ** -9) == 2.0                # rounds up across the binade
    x = np.random.default_rng(0).standard_normal(1000)
    assert np.all(np.abs(b(x) - x) <= np.abs(x) * 2.0 ** -8 * (1 + 1e-12))


def test_bf16_forward_close_to_fp64():
    """The bf16 network differs from the FP64 one by rounding only: a few
    bf16 units relative to the output scale."""
    rng = np.random.default_rng(3)
    theta = mlp.init_params(rng) + 0.05 * rng.standard_normal(mlp.N_PARAM)
    X = rng.standard_normal((50, mlp.N_IN))
    Y, _ = mlp.forward(theta, X)
    Yb = mlp.forward_bf16(theta, X)
    e = np.max(np.abs(Yb - Y)) / np.max(np.abs(Y))
    assert 1e-4 < e < 5e-2
