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


# --- bf16 forward: a one-path network where every rounding site matters -----

def _bf16_ref(v):
    """Independent round-to-nearest-even onto bfloat16 (8 significand bits)
    of the single-precision value of v, by exact integer arithmetic on the
    significand (frexp): no bit tricks shared with the oracle."""
    import math
    import struct
    v = struct.unpack("f", struct.pack("f", float(v)))[0]      # the FP32 value
    if v == 0.0:
        return 0.0
    m, e = math.frexp(v)                   # v = m 2^e, 0.5 <= |m| < 1
    s = m * 256.0                          # 8 significand bits before the point
    return math.ldexp(float(round(s)), e - 8)  # round() ties to even, exact here


def _f32_ref(v):
    import struct
    return struct.unpack("f", struct.pack("f", float(v)))[0]


def _one_path_theta():
    """Only unit 0 of each layer and input 0 are connected; every weight and
    bias value lies off the bfloat16 grid (and off FP32 for the biases)."""
    th = np.zeros(mlp.N_PARAM)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(th)
    W1[0, 0] = 1.5 + 2.0 ** -9 + 2.0 ** -20
    b1[0] = 0.1
    W2[0, 0] = -0.7
    b2[0] = 0.3
    W3[0, 0] = 2.0 / 3.0
    b3[0] = 1.0 / 3.0
    return th


def _one_path_value(x0, th, skip=()):
    """Output 0 of the bf16 network written out by hand for the one-path
    network, with the rounding sites named in `skip` left out."""
    import math
    W1, b1, W2, b2, W3, b3 = mlp.unpack(th)
    rb = lambda k, v: v if k in skip else _bf16_ref(v)
    rf = lambda k, v: v if k in skip else _f32_ref(v)
    g = lambda z: 0.5 * z * (1.0 + math.erf(z / math.sqrt(2.0)))
    z1 = rb("x", x0) * rb("w1", W1[0, 0]) + rf("b1", b1[0])
    h1 = rb("h1", g(z1))
    z2 = h1 * rb("w2", W2[0, 0]) + rf("b2", b2[0])
    h2 = rb("h2", g(z2))
    return rb("w3", W3[0, 0]) * h2 + rf("b3", b3[0])


def test_bf16_forward_each_rounding_site():
    """The oracle's bf16 network on a one-path network equals the hand-written
    evaluation with every rounding site (input, three weights and two hidden
    activations to bf16; biases to FP32) for 64 inputs, and leaving out any
    single bf16 site, or the FP32 rounding of the output bias, changes the
    hand-written output of some input by more than 1e-4 relative: each of
    those sites is pinned.  (The FP32 rounding of the two hidden biases, ~1e-8
    relative, is absorbed by the bf16 rounding that follows it and cannot show
    in any output.)"""
    th = _one_path_theta()
    xs = np.linspace(0.55, 1.95, 64) + 3 * 2.0 ** -11
    X = np.zeros((xs.size, mlp.N_IN))
    X[:, 0] = xs
    got = mlp.forward_bf16(th, X)
    ref = np.array([_one_path_value(x0, th) for x0 in xs])
    assert np.all(np.abs(got[:, 0] - ref) <= 1e-15 * np.abs(ref)), np.abs(got[:, 0] - ref).max()
    # every other output is its FP32-rounded bias (zero here)
    assert np.all(got[:, 1:] == 0.0)
    for site in ("x", "w1", "h1", "w2", "h2", "w3"):
        alt = np.array([_one_path_value(x0, th, skip=(site,)) for x0 in xs])
        assert np.max(np.abs(alt - ref) / np.abs(ref)) > 1e-4, site
    alt = np.array([_one_path_value(x0, th, skip=("b3",)) for x0 in xs])
    assert np.min(np.abs(alt - ref)) > 0.0


def test_bf16_reference_rounding_agrees_on_grid_cases():
    """The independent rounding used above agrees with the oracle's on ties
    and random values (so the one-path pin is about the sites, not the
    rounding rule)."""
    vals = [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(2.0 - 2.0 ** -9), 3.14159, 1e-3, -7.77e5]
    vals += list(np.random.default_rng(5).standard_normal(200))
    for v in vals:
        assert mlp.bf16(v) == _bf16_ref(v), v


# --- Adam beyond the first step ---------------------------------------------

def test_adam_constant_gradient_every_step():
    """With a constant gradient the bias-corrected moments equal g and g^2 at
    every step (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2 from zero), so each of
    the steps t = 1, 2, 3 moves by lr g / (|g| + eps): this needs the moments
    carried over between steps (resetting them would change steps 2 and 3)."""
    g = np.array([3.0, -2.0, 1e-3, 0.5])
    lr, eps = 0.01, 1e-8
    th, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in (1, 2, 3):
        th_new, m, v = mlp.adam_step(th, g, m, v, t, lr)
        step = th_new - th
        assert np.allclose(step, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0.0), t
        th = th_new
    # a reset of the moments before step 2 would move by a different amount
    th2, _, _ = mlp.adam_step(th, g, np.zeros(4), np.zeros(4), 2, lr)
    assert not np.allclose(th2 - th, -lr * g / (np.abs(g) + eps), rtol=1e-3)


def test_adam_scale_and_sign_symmetry():
    """Adam's update depends on the gradient history only through m/sqrt(v):
    scaling every gradient by c > 0 leaves the trajectory unchanged (up to
    eps), negating every gradient negates the steps."""
    rng = np.random.default_rng(8)
    gs = rng.standard_normal((4, 6))

    def run(sc):
        th, m, v = np.zeros(6), np.zeros(6), np.zeros(6)
        for t, g in enumerate(gs, start=1):
            th, m, v = mlp.adam_step(th, sc * g, m, v, t, 1e-3)
        return th
    base = run(1.0)
    assert np.allclose(run(1e3), base, rtol=1e-6, atol=1e-12)
    assert np.allclose(run(-1.0), -base, rtol=1e-12, atol=0.0)
    assert not np.allclose(base, 0.0)
