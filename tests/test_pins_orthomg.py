"""Pins of the orthonormalisation-multigrid oracle (oracle.orthomg): the
invariants the residual minimisation guarantees (W orthonormal, W = M Z,
r = b - M x, non-increasing residual norm), its coefficients against a
least-squares solve of the library, and the solver against a dense direct
solve."""
import numpy as np
import pytest

from oracle import mg, orthomg


@pytest.fixture(scope="module")
def case():
    from xdg_inputs import problems
    pr = problems.c2(seed=3, n=8, hier=[("p", 1), ("h", 1)])
    H = mg.hierarchy_of(pr)
    return pr, H


def test_rm_invariants_and_least_squares(case):
    pr, H = case
    M = H.A[0]
    rng = np.random.default_rng(0)
    b = rng.uniform(-1, 1, M.shape[0])
    x0 = rng.uniform(-1, 1, M.shape[0])
    st = orthomg._Store(x0, b - M @ x0)
    raw = []
    prev = np.linalg.norm(st.r0)
    for k in range(5):
        z = rng.standard_normal(M.shape[0])
        raw.append(z.copy())
        x, r = orthomg.rm(M, st, z)
        W, Z = np.column_stack(st.W), np.column_stack(st.Z)
        assert np.abs(W.T @ W - np.eye(k + 1)).max() <= 1e-12
        assert np.linalg.norm(M @ Z - W) <= 1e-12 * np.linalg.norm(W)
        assert np.linalg.norm(b - M @ x - r) <= 1e-12 * np.linalg.norm(st.r0)
        assert np.linalg.norm(r) <= prev * (1 + 1e-14)
        prev = np.linalg.norm(r)
        # x minimises |b - M x| over x0 + span(raw directions): same point as lstsq
        Zr = np.column_stack(raw)
        a, *_ = np.linalg.lstsq((M @ Zr), st.r0, rcond=None)
        xl = x0 + Zr @ a
        assert np.linalg.norm(x - xl) <= 1e-9 * np.linalg.norm(xl)


def test_exact_direction_gives_exact_solution(case):
    pr, H = case
    M = H.A[0]
    b = np.random.default_rng(1).uniform(-1, 1, M.shape[0])
    st = orthomg._Store(np.zeros_like(b), b)
    import scipy.sparse.linalg as spla
    xs = spla.spsolve(M.tocsc(), b)
    x, r = orthomg.rm(M, st, 3.0 * xs)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_solver_matches_direct_solve():
    from xdg_inputs import problems
    pr = problems.c1()                       # 2D p=2 16^2, three levels, 1,680 unknowns
    H = mg.hierarchy_of(pr)
    M = H.A[0]
    b = np.asarray(pr.b).reshape(-1)
    x, hist, k = orthomg.solve(H, b, rtol=1e-11, restart=12)
    assert hist[-1] <= 1e-11 and k < 200
    xs = np.linalg.solve(M.toarray(), b)
    kappa = np.linalg.cond(M.toarray())
    assert np.linalg.norm(x - xs) <= max(1e-9, 10 * kappa * 1e-11) * np.linalg.norm(xs)


def test_residual_never_increases_within_a_restart(case):
    """Within one store (between restarts) the residual norm is the least over
    a growing subspace, so it cannot increase; across a restart it starts from
    the same x and cannot increase either."""
    pr, H = case
    b = np.asarray(pr.b).reshape(-1)
    _, hist, _ = orthomg.solve(H, b, rtol=1e-10, restart=9)
    assert all(h1 <= h0 * (1 + 1e-12) for h0, h1 in zip(hist, hist[1:]))


def test_coarsest_level_is_the_direct_solve(case):
    pr, H = case
    rc = np.random.default_rng(2).uniform(-1, 1, H.A[-1].shape[0])
    assert np.allclose(orthomg.solve_level(H, H.nlev - 1, rc), H.coarse_solve(rc), rtol=0,
                       atol=0)
