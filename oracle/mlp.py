"""FP64 oracle of the learned per-cell smoother network -- test
infrastructure only.

Network: 45 inputs -> 64 -> 64 (GELU after both hidden layers) -> 40 outputs,
loss = mean over samples of the squared error summed over outputs, trained by
Adam.  Flat parameter vector (row-major [out][in] weights, then biases):
W1[64][45], b1[64], W2[64][64], b2[64], W3[40][64], b3[40].
GELU(x) = x Phi(x) with the standard normal distribution function Phi.
"""
import numpy as np
from scipy.special import erf

N_IN, N_H, N_OUT = 45, 64, 40
SIZES = [(N_H, N_IN), (N_H,), (N_H, N_H), (N_H,), (N_OUT, N_H), (N_OUT,)]
N_PARAM = sum(int(np.prod(s)) for s in SIZES)


def unpack(theta):
    out, o = [], 0
    for s in SIZES:
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_prime(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def forward(theta, X):
    """Y [n, 40] for inputs X [n, 45]; also returns the intermediates."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    Z1 = X @ W1.T + b1
    H1 = gelu(Z1)
    Z2 = H1 @ W2.T + b2
    H2 = gelu(Z2)
    Y = H2 @ W3.T + b3
    return Y, (Z1, H1, Z2, H2)


def bf16(a):
    """Round to the nearest bfloat16 value (ties to even), returned as float64:
    keep the upper 16 bits of the IEEE single-precision pattern after adding
    0x7fff plus the lowest kept bit."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(theta, X):
    """The network with bfloat16 operands: inputs, weights and the two hidden
    activations rounded to bf16, biases and accumulation in (at least) FP32.
    Returns Y [n, 40]."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    H1 = bf16(gelu(bf16(X) @ bf16(W1).T + f32(b1)))
    H2 = bf16(gelu(H1 @ bf16(W2).T + f32(b2)))
    return H2 @ bf16(W3).T + f32(b3)


def loss(theta, X, T):
    Y, _ = forward(theta, X)
    return float(np.sum((Y - T) ** 2) / X.shape[0])


def grad(theta, X, T):
    """Analytic gradient of `loss` (chain rule through the three layers)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    n = X.shape[0]
    Y, (Z1, H1, Z2, H2) = forward(theta, X)
    dY = 2.0 * (Y - T) / n
    gW3 = dY.T @ H2
    gb3 = dY.sum(axis=0)
    dZ2 = (dY @ W3) * gelu_prime(Z2)
    gW2 = dZ2.T @ H1
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * gelu_prime(Z1)
    gW1 = dZ1.T @ X
    gb1 = dZ1.sum(axis=0)
    return np.concatenate([g.reshape(-1) for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) at step t >= 1; returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(rng):
    """Seeded initialisation (uniform, fan-in scaled); biases zero."""
    parts = []
    for s in SIZES:
        if len(s) == 2:
            lim = np.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rng.uniform(-lim, lim, s).reshape(-1))
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)
