"""Pins of the SIP assembly on agglomerated cut cells (Section 2.2 Eq. DefSIP /
SIPrhs, Section 2.3): exact reproduction of solutions inside the XDG space,
convergence order p+1, symmetry and positivity, and the closed form of the
p=0 operator."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from xdg_inputs.assembly import l2_error
from xdg_inputs.levelset import Quadric
from xdg_inputs.problems import build


def _matrix(pr):
    L = pr.n_rows * pr.np
    return sp.bsr_matrix((pr.val, pr.col_idx, pr.row_ptr), shape=(L, L)).tocsc()


def _manufactured(phi, qpoly, grad_q, mu):
    """u_s = phi q / mu_s: continuous across I (phi = 0 there), mu grad u = grad(phi q)
    continuous, f = -lap(phi q) in both phases (q at most linear)."""
    def u(X, s):
        return phi(X) * qpoly(X) / mu[s]

    def f(X, s):
        return -(phi.hessian_trace() * qpoly(X) + 2.0 * np.sum(phi.grad(X) * grad_q(X), axis=1))

    def g(X, s):
        return u(X, s)
    return u, f, g


CASES = [
    # D, n, p, level set, q(x) coefficients (const, linear), mu, tolerance
    (2, 8, 2, Quadric.plane([0.6, 0.8], 0.13), (1.0, [0.5, -0.3]), (1.0, 10.0), 1e-12),
    (2, 8, 2, Quadric.sphere([0.05, -0.02], 0.6), (1.3, [0.0, 0.0]), (1.0, 10.0), 1e-12),
    (2, 6, 3, Quadric.sphere([0.05, -0.02], 0.6), (0.7, [0.2, 0.4]), (1.0, 1000.0), 1e-12),
    (3, 4, 2, Quadric.plane([0.6, 0.64, 0.48], 0.1), (1.0, [0.5, -0.3, 0.2]), (1.0, 1000.0), 1e-12),
    (3, 4, 3, Quadric.sphere([0.05, -0.02, 0.03], 0.6), (1.0, [0.5, -0.3, 0.2]), (1.0, 1000.0),
     1e-11),
]


@pytest.mark.parametrize("D,n,p,phi,qc,mu,tol", CASES)
def test_polynomial_reproduction(D, n, p, phi, qc, mu, tol):
    """A solution inside the XDG space is reproduced by the discrete solve."""
    c0, c1 = qc[0], np.array(qc[1])
    qpoly = lambda X: c0 + X @ c1
    grad_q = lambda X: np.broadcast_to(c1, X.shape)
    u, f, g = _manufactured(phi, qpoly, grad_q, mu)
    pr = build("repro", D, n, p, phi, mu, rhs="load", f=f, g_dir=g, q_cut=16)
    x = spl.spsolve(_matrix(pr), pr.b)
    err = l2_error(pr.geom, pr.levels[0], x, u, p + 3)
    ref = l2_error(pr.geom, pr.levels[0], 0 * x, u, p + 3)
    assert err <= tol * max(ref, 1.0), (err, ref)


def _rates(errs):
    return [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


@pytest.mark.parametrize("p", [1, 2])
def test_convergence_order_uncut(p):
    """Uncut grid, mu = 1, u = sin(pi x) sin(pi y): L2 order p+1."""
    u = lambda X, s: np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1])
    f = lambda X, s: 2 * np.pi ** 2 * u(X, s)
    phi = Quadric.sphere([0.0, 0.0], 10.0)          # everything is species A
    errs = []
    # total-degree P_1 on squares with a penalty locks pre-asymptotically,
    # so p = 1 is measured on finer grids
    for n in ((16, 32, 64) if p == 1 else (8, 16, 32)):
        pr = build("conv", 2, n, p, phi, (1.0, 1.0), rhs="load", f=f,
                   g_dir=lambda X, s: np.zeros(len(X)), q_std=p + 4)
        x = spl.spsolve(_matrix(pr), pr.b)
        errs.append(l2_error(pr.geom, pr.levels[0], x, u, p + 4))
    r = _rates(errs)
    assert r[-1] > p + 1 - 0.25, (errs, r)


@pytest.mark.parametrize("p", [1, 2])
def test_convergence_order_xdg(p):
    """Circle, mu 1 | 10, u_s = phi cos(x) e^{y} / mu_s: L2 order p+1
    (the h^{k+1} rate of XDG stated in Section 5)."""
    phi = Quadric.sphere([0.03, -0.02], 0.6)
    mu = (1.0, 10.0)
    w = lambda X: np.cos(X[:, 0]) * np.exp(X[:, 1])

    def u(X, s):
        return phi(X) * w(X) / mu[s]

    def f(X, s):
        # -lap(phi w) = -(lap(phi) w + 2 grad phi . grad w + phi lap w), lap w = 0
        gw = np.stack([-np.sin(X[:, 0]) * np.exp(X[:, 1]), w(X)], axis=1)
        return -(phi.hessian_trace() * w(X) + 2 * np.sum(phi.grad(X) * gw, axis=1))
    errs = []
    for n in ((16, 32, 64) if p == 1 else (8, 16, 32)):
        pr = build("convx", 2, n, p, phi, mu, rhs="load", f=f, g_dir=u, q_std=p + 4, q_cut=10)
        x = spl.spsolve(_matrix(pr), pr.b)
        errs.append(l2_error(pr.geom, pr.levels[0], x, u, p + 4))
    r = _rates(errs)
    assert r[-1] > p + 1 - 0.3, (errs, r)


@pytest.mark.parametrize("D,n,p,mu", [(2, 8, 2, (1.0, 10.0)), (3, 4, 2, (1.0, 1000.0)),
                                      (3, 4, 3, (1.0, 1000.0))])
def test_symmetric_positive_definite(D, n, p, mu):
    """M is symmetric to rounding and positive definite (Section 4)."""
    phi = Quadric.sphere(np.array([0.04, -0.03, 0.05][:D]), 0.6)
    pr = build("spd", D, n, p, phi, mu, rhs="random", rng=np.random.default_rng(1))
    A = _matrix(pr).toarray()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    ev = np.linalg.eigvalsh(A)
    assert ev[0] > 0.0
    np.linalg.cholesky(A)


def test_p0_graph_laplacian():
    """p = 0 on an uncut grid: only the penalty term survives, so M is
    (eta mu / h) times the grid graph Laplacian plus one diagonal unit per
    boundary face, eta = C_eta (p+1)(p+D)/D * 2D/h."""
    D, n = 2, 5
    h = 2.0 / n
    pr = build("p0", D, n, 0, Quadric.sphere([0.0, 0.0], 10.0), (3.0, 3.0), rhs="random",
               rng=np.random.default_rng(0))
    A = _matrix(pr).toarray()
    eta = pr.c_eta * 1 * D / D * 2 * D / h
    L = np.zeros((n * n, n * n))
    for j in range(n * n):
        ix, iy = j % n, j // n
        for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            kx, ky = ix + dx, iy + dy
            L[j, j] += 1.0
            if 0 <= kx < n and 0 <= ky < n:
                L[j, ky * n + kx] -= 1.0
    # rows are ordered by representative cell = lexicographic cell index
    assert np.allclose(A, eta * 3.0 / h * L, rtol=1e-13, atol=1e-12)
