"""Pins of the plain-loop C++17/OpenMP oracle (oracle/mg_omp.cpp): the CPU
baseline of the benchmark is only meaningful if it computes the same solve.

Against the numpy/scipy oracle (oracle.mg) on small grids: level matrices
(Galerkin products) to 1e-13, one V-cycle and two smoother sweeps to 1e-12,
PCG with the same iteration count and iterates within 1e-12; against a dense
direct solve on a tiny grid (the stand-in for the paper's direct solvers)."""
import numpy as np
import pytest

from oracle import mg, mg_omp


@pytest.fixture(scope="module")
def cases():
    if not __import__("os").path.exists(mg_omp.LIB):
        mg_omp.build()
    from xdg_inputs import problems
    out = {"c1": problems.c1(),
           "c2n8": problems.c2(seed=3, n=8, hier=[("p", 1), ("h", 1)])}
    return {k: (pr, mg.hierarchy_of(pr), mg_omp.OmpHierarchy(pr)) for k, pr in out.items()}


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", ["c1", "c2n8"])
def test_levels_and_operators(cases, name):
    pr, H, O = cases[name]
    assert O.nlev == H.nlev
    rng = np.random.default_rng(3)
    for l in range(H.nlev):
        G = O.level_csr(l)
        assert abs(G - H.A[l]).max() <= 1e-13 * abs(H.A[l]).max(), l
        x = rng.uniform(-1, 1, H.A[l].shape[0])
        assert _rel(O.spmv(l, x), H.A[l] @ x) <= 1e-14
    for l in range(H.nlev - 1):
        b = rng.uniform(-1, 1, H.A[l].shape[0])
        x0 = rng.uniform(-1, 1, H.A[l].shape[0])
        assert _rel(O.smooth(l, b, x0, 2), mg.jacobi(H.A[l], H.Dinv[l], b, x0, 0.7, 2)) <= 1e-12
    r = rng.uniform(-1, 1, H.A[0].shape[0])
    assert _rel(O.vcycle(r), H.vcycle(r)) <= 1e-12


@pytest.mark.parametrize("name", ["c1", "c2n8"])
def test_pcg_matches_numpy_oracle(cases, name):
    pr, H, O = cases[name]
    b = np.asarray(pr.b).reshape(-1)
    xo, ho, ito = mg.pcg(H.A[0], b, H.vcycle, rtol=1e-10, maxit=600)
    xc, hc, itc = O.pcg(b, rtol=1e-10, maxit=600)
    assert itc == ito
    assert np.max(np.abs(np.array(hc) / np.array(ho) - 1.0)) <= 1e-6
    assert _rel(xc, xo) <= 1e-12


def test_coarse_sweeps_match_numpy_oracle(cases):
    """Three sweeps on the levels below the finest (the benchmark's cycle):
    the C++ oracle's V-cycle and PCG equal the numpy oracle's."""
    pr, _, _ = cases["c2n8"]
    H = mg.hierarchy_of(pr, omega=0.9, nu=1, nu_coarse=3)
    O = mg_omp.OmpHierarchy(pr, omega=0.9, nu=1, nu_coarse=3)
    r = np.random.default_rng(7).uniform(-1, 1, H.A[0].shape[0])
    assert _rel(O.vcycle(r), H.vcycle(r)) <= 1e-12
    H1 = mg.hierarchy_of(pr, omega=0.9, nu=1)
    assert _rel(H.vcycle(r), H1.vcycle(r)) > 1e-6          # the count matters
    b = np.asarray(pr.b).reshape(-1)
    xo, ho, ito = mg.pcg(H.A[0], b, H.vcycle, rtol=1e-10, maxit=600)
    xc, hc, itc = O.pcg(b, rtol=1e-10, maxit=600)
    assert itc == ito and _rel(xc, xo) <= 1e-12
    O.close()


def test_pcg_matches_dense_direct_solve():
    from xdg_inputs.levelset import Quadric
    from xdg_inputs.problems import build
    pr = build("omp3d", 3, 4, 2, Quadric.sphere([0.02, -0.03, 0.01], 0.6), (1.0, 1000.0),
               hierarchy=[("p", 1), ("h", 1)], rhs="random", rng=np.random.default_rng(4),
               q_cut=10)
    O = mg_omp.OmpHierarchy(pr)
    A = mg.block_matrix(pr.row_ptr, pr.col_idx, pr.val).toarray()
    b = np.asarray(pr.b).reshape(-1)
    x_direct = np.linalg.solve(A, b)
    xc, hc, itc = O.pcg(b, rtol=1e-14, maxit=500)
    kappa = np.linalg.cond(A)
    assert _rel(xc, x_direct) <= max(1e-11, 10 * kappa * 2.0 ** -53)
    assert all(h1 < h0 * 10 for h0, h1 in zip(hc, hc[1:]))
