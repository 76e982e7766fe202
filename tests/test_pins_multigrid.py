"""Pins of the oracle's multigrid solve and of the transfer operators.

* orthonormal bases and nested transfers (Section 3.2: orthonormal bases make
  R^T a projector; Sum_i R_i^T R_i = I; p-transfer = [I; 0]);
* Galerkin coarse operator (Eq. XDGsysRestriction) equals the SIP form
  assembled directly on the coarse aggregated space with the fine penalties;
* V-cycle equals the closed-form error propagation S^nu (I - R B_c R^T A) S^nu
  computed with dense matrices; it is symmetric and positive definite;
* MG-PCG / FGMRES agree with a dense direct solve (the stand-in for the
  sparse direct solvers of Section 4); PCG A-norm errors decrease; FGMRES
  residuals do not increase within a restart cycle.
"""
import numpy as np
import pytest

from oracle import mg
from xdg_inputs.assembly import assemble
from xdg_inputs.levelset import Quadric
from xdg_inputs.problems import build


def _p2d(n=8, p=2, hier=None):
    hier = hier or [("p", 1), ("h", 1)]
    return build("mg2d", 2, n, p, Quadric.sphere([0.03, -0.04], 0.62), (1.0, 10.0),
                 hierarchy=hier, rhs="random", rng=np.random.default_rng(3), q_cut=12)


def _p3d(n=4, p=2):
    return build("mg3d", 3, n, p, Quadric.sphere([0.02, -0.03, 0.01], 0.6), (1.0, 1000.0),
                 hierarchy=[("p", 1), ("h", 1)], rhs="random", rng=np.random.default_rng(4),
                 q_cut=10)


def _p3d_same_degree(n=4, p=2):
    """Aggregation level at the fine degree (the paper's sequence keeps the
    degree on every level): 4^3 p2 -> 2^3 aggregates p2."""
    return build("mg3dh", 3, n, p, Quadric.sphere([0.02, -0.03, 0.01], 0.6), (1.0, 1000.0),
                 hierarchy=[("h", 1, p)], rhs="random", rng=np.random.default_rng(5),
                 q_cut=10)


@pytest.fixture(scope="module")
def pr2():
    return _p2d()


@pytest.fixture(scope="module")
def pr3h():
    return _p3d_same_degree()


@pytest.fixture(scope="module")
def pr3():
    return _p3d()


def _gram(geom, level, r, q):
    s = int(level.species[r])
    G = np.zeros((level.np, level.np))
    for j in level.pieces(r):
        P, W = geom.volume_rule(j, s, q)
        v = level.bases[r].eval(P, grad=False)
        G += (v * W[:, None]).T @ v
    return G


def test_bases_orthonormal(pr2, pr3, pr3h):
    """Mass matrix of every part is the identity, to the rounding of a
    Cholesky re-orthonormalisation (kappa(G) eps with kappa(G) up to ~1e4 on
    small cut parts inside a large bounding box)."""
    for pr in (pr2, pr3, pr3h):
        for lv in pr.levels:
            worst = max(np.abs(_gram(pr.geom, lv, r, lv.deg + 2) - np.eye(lv.np)).max()
                        for r in range(lv.n_rows))
            assert worst < 1e-10


def test_transfer_invariants(pr2, pr3, pr3h):
    for pr in (pr2, pr3, pr3h):
        for t, (fine, coarse) in enumerate(zip(pr.levels[:-1], pr.levels[1:])):
            T = pr.transfers[t]
            if T["kind"] == mg.T_PTRUNC:
                # computed by quadrature the p-transfer is [I; 0]
                for r in range(0, fine.n_rows, max(1, fine.n_rows // 40)):
                    s = int(fine.species[r])
                    M = 0.0
                    for j in fine.pieces(r):
                        P, W = pr.geom.volume_rule(j, s, fine.deg + 2)
                        a = fine.bases[r].eval(P, grad=False)
                        b = coarse.bases[r].eval(P, grad=False)
                        M = M + (a * W[:, None]).T @ b
                    E = np.zeros((fine.np, coarse.np))
                    E[:coarse.np, :coarse.np] = np.eye(coarse.np)
                    assert np.abs(M - E).max() < 1e-12
            else:
                S = np.zeros((coarse.n_rows, coarse.np, coarse.np))
                for i in range(fine.n_rows):
                    S[T["parent"][i]] += T["R"][i].T @ T["R"][i]
                assert np.abs(S - np.eye(coarse.np)).max() < 1e-12
                Rm = mg.transfer_matrix(T, fine.n_rows, fine.np).toarray()
                # R^T is a left inverse of R, R R^T an orthogonal projector
                assert np.allclose(Rm.T @ Rm, np.eye(Rm.shape[1]), atol=1e-12)


def test_galerkin_equals_coarse_assembly(pr2, pr3, pr3h):
    """R^T M R equals SIP assembled on the coarse space with the fine-level
    penalties; faces inside a coarse aggregate drop out."""
    for pr in (pr2, pr3, pr3h):
        H = mg.hierarchy_of(pr)
        for l in range(1, H.nlev):
            lv = pr.levels[l]
            rp, ci, val = assemble(pr.geom, lv, pr.mu, pr.penalty, lv.deg + 2)
            A = mg.block_matrix(rp, ci, val).toarray()
            G = H.A[l].toarray()
            assert np.abs(A - G).max() <= 1e-11 * np.abs(G).max(), l


def test_p_level_is_leading_subblock(pr2):
    H = mg.hierarchy_of(pr2)
    npc = H.np[1]
    A0 = H.A[0].toarray().reshape(pr2.n_rows, pr2.np, pr2.n_rows, pr2.np)
    lead = A0[:, :npc, :, :npc].reshape(pr2.n_rows * npc, -1)
    assert np.array_equal(lead, H.A[1].toarray())


def _vcycle_dense(H, level, sweeps):
    """B_l = (I - S^nu (I - R B_{l+1} R^T A) S^nu) A^{-1}, S = I - w D^{-1} A,
    nu = sweeps[l] (the same count before and after the coarse correction)."""
    A = H.A[level].toarray()
    if level == H.nlev - 1:
        return np.linalg.inv(A)
    I = np.eye(A.shape[0])
    S = I - H.omega * H.Dinv[level].toarray() @ A
    R = H.R[level].toarray()
    Bc = _vcycle_dense(H, level + 1, sweeps)
    Sn = np.linalg.matrix_power(S, sweeps[level])
    E = Sn @ (I - R @ Bc @ R.T @ A) @ Sn
    return (I - E) @ np.linalg.inv(A)


@pytest.mark.parametrize("nu,omega,nu_c", [(2, 0.7, 0), (1, 0.9, 0), (1, 0.9, 3)])
def test_vcycle_closed_form_and_spd(nu, omega, nu_c, pr2, pr3, pr3h):
    """(2, 0.7): the configs' smoother; (1, 0.9): one sweep on every level;
    (1, 0.9) with 3 sweeps on the levels below the finest: the benchmark's."""
    for pr in (pr2, pr3, pr3h):
        H = mg.hierarchy_of(pr, omega=omega, nu=nu, nu_coarse=nu_c)
        L = H.A[0].shape[0]
        B = np.column_stack([H.vcycle(e) for e in np.eye(L)])
        sweeps = [nu] + [nu_c if nu_c > 0 else nu] * (H.nlev - 1)
        Bd = _vcycle_dense(H, 0, sweeps)
        assert np.abs(B - Bd).max() <= 1e-9 * np.abs(Bd).max()
        assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
        assert np.linalg.eigvalsh(0.5 * (B + B.T))[0] > 0.0
        # eigenvalues of B A lie in (0, 1] when every smoother is A-convergent
        for l in range(H.nlev - 1):
            assert H.omega * H.lambda_max_DinvA(l, 300) < 2.0
        ev = np.linalg.eigvals(B @ H.A[0].toarray()).real
        assert ev.min() > 0.0 and ev.max() <= 1.0 + 1e-10


def test_block_inverses_and_coarse_solve(pr3):
    H = mg.hierarchy_of(pr3)
    for l in range(H.nlev - 1):
        A = H.A[l].toarray()
        cp, Np = H.cell_ptr[l], H.np[l]
        Dinv = H.Dinv[l].toarray()
        for c in range(len(cp) - 1):
            s = slice(cp[c] * Np, cp[c + 1] * Np)
            assert np.allclose(A[s, s] @ Dinv[s, s], np.eye(s.stop - s.start), atol=1e-10)
    Ac = H.A[-1].toarray()
    r = np.random.default_rng(0).standard_normal(Ac.shape[0])
    assert np.allclose(H.coarse_solve(r), np.linalg.solve(Ac, r), rtol=1e-10, atol=0)


def test_jacobi_single_block_is_exact():
    """omega = 1 block Jacobi on a block-diagonal system solves it in one sweep."""
    rng = np.random.default_rng(7)
    Np, nr = 3, 4
    val = np.zeros((nr, Np, Np))
    for i in range(nr):
        X = rng.standard_normal((Np, Np))
        val[i] = X @ X.T + Np * np.eye(Np)
    rp = np.arange(nr + 1)
    A = mg.block_matrix(rp, np.arange(nr), val)
    Dinv, _ = mg.cell_block_inverses(A, np.arange(nr + 1), Np)
    b = rng.standard_normal(nr * Np)
    x = mg.jacobi(A, Dinv, b, np.zeros_like(b), 1.0, 1)
    assert np.allclose(A @ x, b, atol=1e-13)


@pytest.mark.parametrize("which", ["2d", "3d", "3d-same-degree"])
def test_mg_pcg_matches_dense_direct(which, pr2, pr3, pr3h):
    pr = {"2d": pr2, "3d": pr3, "3d-same-degree": pr3h}[which]
    H = mg.hierarchy_of(pr)
    A = H.A[0].toarray()
    xd = np.linalg.solve(A, pr.b)
    x, hist, it = mg.pcg(H.A[0], pr.b, H.vcycle, rtol=1e-14, maxit=400)
    kappa = np.linalg.cond(A)
    tol = max(1e-11, 10 * kappa * 2.0 ** -53)
    assert np.linalg.norm(x - xd) <= tol * np.linalg.norm(xd), (it, hist[-1])
    x2, hist2, it2 = mg.fgmres(H.A[0], pr.b, H.vcycle, rtol=1e-13, restart=30, maxit=400)
    assert np.linalg.norm(x2 - xd) <= tol * np.linalg.norm(xd)


def test_pcg_energy_error_monotone(pr2):
    H = mg.hierarchy_of(pr2)
    A = H.A[0].toarray()
    xd = np.linalg.solve(A, pr2.b)
    errs = []
    for k in range(1, 25):
        x, _, _ = mg.pcg(H.A[0], pr2.b, H.vcycle, rtol=0.0, maxit=k)
        e = x - xd
        errs.append(e @ (A @ e))
    assert all(b <= a * (1 + 1e-9) for a, b in zip(errs, errs[1:]))


def test_fgmres_residual_monotone_within_cycle(pr2):
    H = mg.hierarchy_of(pr2)
    x, hist, it = mg.fgmres(H.A[0], pr2.b, H.vcycle, rtol=1e-12, restart=10, maxit=60)
    for c in range(0, len(hist) - 1, 10):
        seg = hist[c:c + 11]
        assert all(b <= a * (1 + 1e-12) for a, b in zip(seg, seg[1:]))
    A = H.A[0].toarray()
    assert np.linalg.norm(pr2.b - A @ x) / np.linalg.norm(pr2.b) <= 1.01e-12


def test_lambda_max_matches_generalised_eigenproblem(pr2, pr3):
    """The power-iteration estimate of lambda_max(D^-1 A) against the largest
    eigenvalue of the symmetric-definite pencil (A, D) by a dense eigensolver
    (D = the cell-block diagonal of A).  The norm ratio of the power
    iteration converges to the spectral radius of D^-1 A from either side
    (the operator is not normal in the Euclidean inner product); 600 steps
    bring it within 2e-3 relative."""
    import scipy.linalg as sla
    for pr in (pr2, pr3):
        H = mg.hierarchy_of(pr)
        for l in range(H.nlev - 1):
            A = H.A[l].toarray()
            cp, npl = H.cell_ptr[l], H.np[l]
            D = np.zeros_like(A)
            for c in range(len(cp) - 1):
                s = slice(cp[c] * npl, cp[c + 1] * npl)
                D[s, s] = A[s, s]
            lam = sla.eigh(A, D, eigvals_only=True)[-1]
            est = H.lambda_max_DinvA(l, 600)
            assert abs(est - lam) <= 2e-3 * lam, (l, est, lam)
            # block Jacobi on an SPD matrix: 1 <= lambda_max < 2 bounds hold
            assert 1.0 <= lam < 2.0
