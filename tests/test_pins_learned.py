"""Pins of the learned-smoother oracle (oracle.learned) on a small cut-cell
problem: special cases that reduce it to plain block Jacobi, scale
equivariance, the slot layout of the features, and consistency between the
training pairs and the sweep (a perfect network reproduces the error)."""
import numpy as np
import pytest

from oracle import learned, mg, mlp


@pytest.fixture(scope="module")
def case():
    from xdg_inputs import features, problems
    pr = problems.c4(seed=41, n=8, p=3, nrhs=1)
    pr.b = np.asarray(pr.b).reshape(-1)
    rs, g = features.cell_features(pr)
    H = mg.hierarchy_of(pr)
    return pr, H, rs, g.astype(np.float64)


def _theta(seed, out_scale):
    rng = np.random.default_rng(seed)
    th = mlp.init_params(rng) + 0.05 * rng.standard_normal(mlp.N_PARAM)
    W3, b3 = mlp.unpack(th)[4:]
    W3 *= out_scale
    b3 *= out_scale
    return th


def test_zero_network_is_plain_vcycle(case):
    pr, H, rs, g = case
    r = np.random.default_rng(1).uniform(-1, 1, pr.b.size)
    th = _theta(1, 0.0)
    z = learned.vcycle(H, rs, g, th, r, guard=4.0)
    assert np.allclose(z, H.vcycle(r), rtol=0, atol=1e-13 * np.abs(z).max())
    x, nb = learned.first_sweep(H, rs, g, th, r, guard=4.0)
    assert nb == 0
    assert np.allclose(x, H.omega * (H.Dinv[0] @ r), rtol=1e-14, atol=0)


def test_scale_equivariance(case):
    pr, H, rs, g = case
    r = np.random.default_rng(2).uniform(-1, 1, pr.b.size)
    th = _theta(2, 0.3)
    x1, _ = learned.first_sweep(H, rs, g, th, r, guard=1e30)
    for a in (1e-6, 3.0, 1e5):
        xa, _ = learned.first_sweep(H, rs, g, th, a * r, guard=1e30)
        assert np.allclose(xa, a * x1, rtol=1e-10, atol=1e-12 * a * np.abs(x1).max())
    # and the proposal really differs from plain Jacobi
    j = H.omega * (H.Dinv[0] @ r)
    assert np.linalg.norm(x1 - j) > 1e-3 * np.linalg.norm(j)


def test_feature_slots(case):
    pr, H, rs, g = case
    r = np.random.default_rng(3).uniform(-1, 1, pr.b.size)
    F, j, s = learned.features(H, rs, g, r)
    cp = np.asarray(pr.cell_ptr)
    nrow = np.diff(cp)
    assert (nrow == 2).any() and (nrow == 1).any()
    for c in range(len(cp) - 1):
        rows = range(cp[c], cp[c + 1])
        assert np.isclose(np.linalg.norm(F[c, :40]), 1.0, atol=1e-14)
        present = {int(rs[q]) for q in rows}
        for sp in (0, 1):
            blk = F[c, 20 * sp:20 * sp + 20]
            if sp not in present:
                assert not blk.any()
        for q in rows:
            sp = int(rs[q])
            assert np.allclose(F[c, 20 * sp:20 * sp + 20] * s[c], j[20 * q:20 * q + 20],
                               rtol=1e-14, atol=1e-300)
    assert np.array_equal(F[:, 40:], g)


def test_perfect_network_reproduces_the_error(case):
    """Applying the pair targets as the network output gives x = x* - x_k on
    every cell: the pairs and the sweep agree on slots and scaling."""
    pr, H, rs, g = case
    rng = np.random.default_rng(4)
    xk, xs = rng.uniform(-1, 1, pr.b.size), rng.uniform(-1, 1, pr.b.size)
    X, T = learned.pairs(H, rs, g, pr.b, xk, xs)
    r = pr.b - H.A[0] @ xk
    F, j, s = learned.features(H, rs, g, r)
    assert np.array_equal(X, F)
    cp = np.asarray(pr.cell_ptr)
    x = np.empty_like(j)
    for c in range(len(cp) - 1):
        for q in range(cp[c], cp[c + 1]):
            sp = int(rs[q])
            x[20 * q:20 * q + 20] = j[20 * q:20 * q + 20] + s[c] * T[c, 20 * sp:20 * sp + 20]
    assert np.allclose(x, xs - xk, rtol=1e-12, atol=1e-12)


def test_guard_keeps_plain_step(case):
    pr, H, rs, g = case
    r = np.random.default_rng(5).uniform(-1, 1, pr.b.size)
    th = _theta(5, 1e4)
    x, nb = learned.first_sweep(H, rs, g, th, r, guard=4.0)
    assert nb == len(pr.cell_ptr) - 1
    assert np.array_equal(x, H.omega * (H.Dinv[0] @ r))
    th[0] = np.nan
    x, nb = learned.first_sweep(H, rs, g, th, r, guard=1e30)
    assert nb == len(pr.cell_ptr) - 1 and np.all(np.isfinite(x))


def test_clipped_pairs_keep_direction(case):
    pr, H, rs, g = case
    rng = np.random.default_rng(6)
    xk, xs = rng.uniform(-1, 1, pr.b.size), rng.uniform(-1, 1, pr.b.size)
    X, T = learned.pairs(H, rs, g, pr.b, xk, xs)
    cl = float(np.median(np.linalg.norm(T, axis=1)))
    Xc, Tc = learned.pairs(H, rs, g, pr.b, xk, xs, clip=cl)
    assert np.array_equal(X, Xc)
    n, nc = np.linalg.norm(T, axis=1), np.linalg.norm(Tc, axis=1)
    assert (n > cl).any() and (n <= cl).any()
    assert np.all(nc <= cl * (1 + 1e-14))
    small = n <= cl
    assert np.array_equal(Tc[small], T[small])
    big = ~small
    cos = np.sum(T[big] * Tc[big], axis=1) / (n[big] * nc[big])
    assert np.allclose(cos, 1.0, atol=1e-14)
