"""GPU parity of every C-ABI call against the FP64 oracle on the same seeded
problems (small sizes: full outputs; the 32^3 p=3 workload: sampled rows,
operator identities and the oracle's own residual check).

Tolerances (FP64, relative 2-norm unless stated):
  * spmv, restriction, prolongation, Galerkin levels: 1e-13 (same products,
    different summation order only);
  * smoother sweeps, cell-block inverses, V-cycle, coarsest inverse: the GPU
    inverts by Gauss-Jordan, the oracle by Cholesky; both are backward
    stable, so they agree to ~kappa * eps -- the bound is
    max(1e-11, 50 kappa eps) with kappa the measured condition number;
  * solves: both reach rel.res <= 1e-10; iterates agree to the same
    kappa-relaxed bound; iteration counts within 1.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a device"
    return t


def _make(name):
    from xdg_inputs import problems
    if name == "c1":
        return problems.c1()
    if name == "c2n8":
        return problems.c2(seed=3, n=8, hier=[("p", 1), ("h", 1)])
    if name in ("c2n16", "c2n16gen"):
        return problems.c2(seed=1, n=16)
    if name == "c2n8hp":
        # aggregation level at the fine degree (20 coarse modes per block)
        return problems.c2(seed=4, n=8, hier=problems.hierarchy("hp", 8, 3))
    if name == "c2n16h3p1":
        return problems.c2(seed=2, n=16, hier=problems.hierarchy("h3p1", 16, 3))
    if name == "c4n8p4":
        # p = 4 (35 modes per block: the one-row-per-lane stream), ellipsoid
        pr = problems.c4(seed=5, n=8, p=4, nrhs=1)
        pr.b = np.asarray(pr.b).reshape(-1)
        return pr
    raise KeyError(name)


_STATE = {}


def _case(name, torch):
    if name not in _STATE:
        from oracle import mg
        from paper_2003_02431_amd import binding as B
        _log(f"[gpu-parity] building case {name}")
        pr = _make(name)
        H = mg.hierarchy_of(pr)
        # "gen": the level-0 solve kernels read every block (symmetric = 0);
        # otherwise 20-mode levels use the symmetric (upper-block) storage
        sym = 0 if name.endswith("gen") else 1
        S = B.Solver(pr, B.options(rtol=1e-10, maxit=600, symmetric=sym))
        _STATE[name] = (pr, H, S)
    return _STATE[name]


CASES = ["c1", "c2n8", "c2n16", "c2n16gen", "c4n8p4", "c2n8hp", "c2n16h3p1"]


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _kappa_tol(kappa):
    return max(1e-11, 50.0 * kappa * EPS)


@pytest.mark.parametrize("name", CASES)
def test_level_matrices_and_spmv(name, torch):
    from oracle import mg
    from paper_2003_02431_amd import binding as B
    pr, H, S = _case(name, torch)
    rng = np.random.default_rng(11)
    for l in range(H.nlev):
        rp, ci, val = B.xdg_get_level_matrix(S.h, l)
        G = mg.block_matrix(rp, ci, val)
        O = H.A[l]
        d = abs(G - O).max() / abs(O).max()
        _log(f"  {name} level {l}: Galerkin max rel diff {d:.2e}")
        assert d <= 1e-13
        x = rng.uniform(-1, 1, O.shape[0])
        y = S.vec(l)
        B.xdg_spmv(S.h, l, S.vec(l, x), y)
        e = _rel(y.cpu().numpy(), O @ x)
        _log(f"  {name} level {l}: spmv rel err {e:.2e}")
        assert e <= 1e-13


@pytest.mark.parametrize("name", CASES)
def test_transfers(name, torch):
    from paper_2003_02431_amd import binding as B
    pr, H, S = _case(name, torch)
    rng = np.random.default_rng(12)
    for l in range(H.nlev - 1):
        R = H.R[l]
        rf = rng.uniform(-1, 1, R.shape[0])
        rc = S.vec(l + 1)
        B.xdg_restrict(S.h, l, S.vec(l, rf), rc)
        assert _rel(rc.cpu().numpy(), R.T @ rf) <= 1e-13
        xc = rng.uniform(-1, 1, R.shape[1])
        xf0 = rng.uniform(-1, 1, R.shape[0])
        xf = S.vec(l, xf0)
        B.xdg_prolong(S.h, l, S.vec(l + 1, xc), xf)
        assert _rel(xf.cpu().numpy(), xf0 + R @ xc) <= 1e-13


@pytest.mark.parametrize("name", CASES)
def test_cell_inverses_and_smoother(name, torch):
    from oracle import mg
    from paper_2003_02431_amd import binding as B
    pr, H, S = _case(name, torch)
    rng = np.random.default_rng(13)
    for l in range(H.nlev - 1):
        _, invs = mg.cell_block_inverses(H.A[l], H.cell_ptr[l], H.np[l])
        kmax = 1.0
        for c in np.unique(np.linspace(0, len(invs) - 1, 40).astype(int)):
            Dg = B.xdg_get_cell_inverse(S.h, l, int(c))
            k = np.linalg.cond(invs[c])
            kmax = max(kmax, k)
            assert _rel(Dg, invs[c]) <= _kappa_tol(k), (l, c, k)
        b = rng.uniform(-1, 1, H.A[l].shape[0])
        x0 = rng.uniform(-1, 1, H.A[l].shape[0])
        x = S.vec(l, x0)
        B.xdg_smooth(S.h, l, S.vec(l, b), x, 2)
        ref = mg.jacobi(H.A[l], H.Dinv[l], b, x0, 0.7, 2)
        e = _rel(x.cpu().numpy(), ref)
        _log(f"  {name} level {l}: smoother rel err {e:.2e} (max cell kappa {kmax:.1e})")
        assert e <= _kappa_tol(kmax)


@pytest.mark.parametrize("name", CASES)
def test_coarsest_inverse(name, torch):
    from paper_2003_02431_amd import binding as B
    pr, H, S = _case(name, torch)
    Ac = H.A[-1].toarray()
    Cg = B.xdg_get_cell_inverse(S.h, H.nlev - 1, 0)
    kappa = np.linalg.cond(Ac)
    e = _rel(Cg, np.linalg.inv(Ac))
    _log(f"  {name}: coarsest n={Ac.shape[0]} kappa={kappa:.2e} inverse rel diff {e:.2e}")
    assert e <= _kappa_tol(kappa)
    assert np.abs(Cg @ Ac - np.eye(Ac.shape[0])).max() <= _kappa_tol(kappa)


@pytest.mark.parametrize("name", CASES)
def test_vcycle(name, torch):
    from paper_2003_02431_amd import binding as B
    pr, H, S = _case(name, torch)
    rng = np.random.default_rng(14)
    r = rng.uniform(-1, 1, H.A[0].shape[0])
    z = S.vec(0)
    B.xdg_vcycle(S.h, S.vec(0, r), z)
    ref = H.vcycle(r)
    kappa = np.linalg.cond(H.A[-1].toarray())
    e = _rel(z.cpu().numpy(), ref)
    _log(f"  {name}: vcycle rel err {e:.2e} (coarse kappa {kappa:.1e})")
    assert e <= _kappa_tol(kappa)


@pytest.mark.parametrize("name", CASES)
def test_pcg_solve(name, torch):
    from oracle import mg
    from paper_2003_02431_amd import binding as B
    pr, H, S = _case(name, torch)
    b = pr.b
    xo, ho, ito = mg.pcg(H.A[0], b, H.vcycle, rtol=1e-10, maxit=600)
    x = S.vec(0)
    rc, it, fr, hist = B.xdg_solve(S.h, S.vec(0, b), x)
    xg = x.cpu().numpy()
    tr = np.linalg.norm(b - H.A[0] @ xg) / np.linalg.norm(b)
    e = _rel(xg, xo)
    hd = np.max(np.abs(hist[:min(len(hist), len(ho))] / np.array(ho[:len(hist)]) - 1.0))
    _log(f"  {name}: PCG gpu it={it} oracle it={ito} true relres={tr:.2e} "
         f"x rel diff={e:.2e} hist rel diff={hd:.2e}")
    assert rc == 0 and abs(it - ito) <= 1
    assert tr <= 1.05e-10 and abs(fr - tr) <= 1e-3 * tr
    assert hd <= 1e-6
    assert e <= 1e-8
    # the FP64 contract: the iterate after exactly the oracle's iteration
    # count matches the oracle's iterate to 1e-11 (only rounding order
    # separates the two runs of the same recurrence)
    B.xdg_set_tolerance(S.h, 1e-300, ito)
    xk = S.vec(0)
    rck, itk, _, _ = B.xdg_solve(S.h, S.vec(0, b), xk)
    B.xdg_set_tolerance(S.h, 1e-10, 600)
    ek = _rel(xk.cpu().numpy(), xo)
    _log(f"  {name}: PCG iterate {itk} rel diff to the oracle's {ek:.2e}")
    assert rck == B.XDG_ENOCONV and itk == ito and ek <= 1e-11


@pytest.mark.parametrize("name", ["c2n16", "c2n8hp", "c4n8p4"])
def test_coarse_sweeps(name, torch):
    """nu_coarse = 3 (three sweeps before and after the coarse correction on
    every level below the finest, one on level 0, omega 0.9: the benchmark's
    cycle): one V-cycle and the PCG iterate after the oracle's iteration count
    against the oracle's hierarchy with the same counts."""
    from oracle import mg
    from paper_2003_02431_amd import binding as B
    pr, _, _ = _case(name, torch)
    H = mg.hierarchy_of(pr, omega=0.9, nu=1, nu_coarse=3)
    S = B.Solver(pr, B.options(rtol=1e-10, maxit=600, nu_pre=1, nu_post=1, omega=0.9,
                               nu_coarse=3))
    n = S.level_len(0)
    r = np.random.default_rng(11).uniform(-1, 1, n)
    z = S.vec(0)
    B.xdg_vcycle(S.h, S.vec(0, r), z)
    kappa = np.linalg.cond(H.A[-1].toarray())
    ev = _rel(z.cpu().numpy(), H.vcycle(r))
    b = np.asarray(pr.b).reshape(-1)
    xo, ho, ito = mg.pcg(H.A[0], b, H.vcycle, rtol=1e-10, maxit=600)
    B.xdg_set_tolerance(S.h, 1e-300, ito)
    xk = S.vec(0)
    rck, itk, _, _ = B.xdg_solve(S.h, S.vec(0, b), xk)
    ek = _rel(xk.cpu().numpy(), xo)
    H1 = mg.hierarchy_of(pr, omega=0.9, nu=1)
    _, _, it1 = mg.pcg(H1.A[0], b, H1.vcycle, rtol=1e-10, maxit=600)
    S.close()
    _log(f"  {name}: nu_coarse 3: V-cycle rel err {ev:.2e} (coarse kappa {kappa:.1e}); "
         f"PCG iterate {itk} (oracle {ito}, one sweep everywhere {it1}) rel diff {ek:.2e}")
    assert ev <= _kappa_tol(kappa)
    assert rck == B.XDG_ENOCONV and itk == ito and ek <= 1e-11


@pytest.mark.parametrize("name", ["c2n8", "c2n16"])
def test_calls_after_a_solve(name, torch):
    """The FP64 CG fuses its x/r update with the next cycle's first level-0
    sweep and lets the cycle skip that sweep; a solve that stops right after
    such an update must not leak this into later calls: xdg_vcycle and
    xdg_smooth after a solve equal the same calls on a fresh handle, bit for
    bit, and a second solve repeats the first."""
    from paper_2003_02431_amd import binding as B
    pr, H, S = _case(name, torch)
    n = S.level_len(0)
    r = S.vec(0, np.random.default_rng(5).uniform(-1, 1, n))
    x = S.vec(0)
    rc1, it1, fr1, _ = B.xdg_solve(S.h, S.vec(0, pr.b), x)
    x1 = x.cpu().numpy().copy()
    z = S.vec(0)
    B.xdg_vcycle(S.h, r, z)
    F = B.Solver(pr, B.options(rtol=1e-10, maxit=600))
    zf = F.vec(0)
    B.xdg_vcycle(F.h, F.vec(0, r.cpu().numpy()), zf)
    d = float(np.max(np.abs(z.cpu().numpy() - zf.cpu().numpy())))
    xs = S.vec(0, np.zeros(n))
    B.xdg_smooth(S.h, 0, r, xs, 1)
    xsf = F.vec(0, np.zeros(n))
    B.xdg_smooth(F.h, 0, F.vec(0, r.cpu().numpy()), xsf, 1)
    ds = float(np.max(np.abs(xs.cpu().numpy() - xsf.cpu().numpy())))
    x.zero_()
    rc2, it2, fr2, _ = B.xdg_solve(S.h, S.vec(0, pr.b), x)
    dx = float(np.max(np.abs(x.cpu().numpy() - x1)))
    F.close()
    _log(f"  {name}: after a solve ({it1} it): V-cycle max diff {d:.1e}, sweep {ds:.1e}, "
         f"second solve {it2} it, max diff {dx:.1e}")
    assert rc1 == 0 and rc2 == 0 and it1 == it2
    assert d == 0.0 and ds == 0.0 and dx == 0.0


@pytest.mark.parametrize("name", ["c1", "c2n16"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fgmres_solve(name, prec, torch):
    from oracle import mg
    from paper_2003_02431_amd import binding as B
    pr, H, _ = _case(name, torch)
    P = B.XDG_FP64 if prec == "fp64" else B.XDG_MIXED
    rtol = 1e-10
    S = B.Solver(pr, B.options(krylov=B.XDG_FGMRES, restart=30, precision=P, rtol=rtol,
                               maxit=600))
    xs, _, _ = mg.pcg(H.A[0], pr.b, H.vcycle, rtol=1e-13, maxit=1000)
    x = S.vec(0)
    rc, it, fr, hist = B.xdg_solve(S.h, S.vec(0, pr.b), x)
    xg = x.cpu().numpy()
    tr = np.linalg.norm(pr.b - H.A[0] @ xg) / np.linalg.norm(pr.b)
    err = _rel(xg, xs)
    _log(f"  {name} FGMRES {prec}: it={it} relres={tr:.2e} err vs x*={err:.2e}")
    assert rc == 0 and tr <= 1.05 * rtol
    assert err <= 1e-8
    S.close()


@pytest.mark.parametrize("name", ["c1", "c2n16"])
def test_mixed_flexible_cg(name, torch):
    """FP32 V-cycle inside flexible CG (FP64 residuals, directions and inner
    products): the error against the oracle's x* follows the energy-norm
    minimisation of CG, so rel.res 1e-8 already gives error <= 1e-8."""
    from oracle import mg
    from paper_2003_02431_amd import binding as B
    pr, H, _ = _case(name, torch)
    rtol = 1e-8
    S = B.Solver(pr, B.options(krylov=B.XDG_CG, precision=B.XDG_MIXED, rtol=rtol, maxit=600))
    xs, _, ito = mg.pcg(H.A[0], pr.b, H.vcycle, rtol=1e-13, maxit=1000)
    _, _, it8 = mg.pcg(H.A[0], pr.b, H.vcycle, rtol=rtol, maxit=1000)
    x = S.vec(0)
    rc, it, fr, hist = B.xdg_solve(S.h, S.vec(0, pr.b), x)
    xg = x.cpu().numpy()
    tr = np.linalg.norm(pr.b - H.A[0] @ xg) / np.linalg.norm(pr.b)
    err = _rel(xg, xs)
    _log(f"  {name} flexible CG mixed: it={it} (oracle FP64 PCG {it8}) relres={tr:.2e} "
         f"err vs x*={err:.2e}")
    assert rc == 0 and tr <= 1.05 * rtol and abs(fr - tr) <= 1e-3 * tr
    assert err <= 1e-8
    S.close()


@pytest.mark.parametrize("krylov", ["cg", "fgmres"])
def test_zero_rhs(krylov, torch):
    """Degenerate input b = 0: the solution is zero whatever the start held,
    with no iteration and a zero residual."""
    from paper_2003_02431_amd import binding as B
    pr, H, _ = _case("c2n8", torch)
    K_ = B.XDG_CG if krylov == "cg" else B.XDG_FGMRES
    S = B.Solver(pr, B.options(krylov=K_, rtol=1e-10))
    x = S.vec(0, np.random.default_rng(2).uniform(-1, 1, H.A[0].shape[0]))
    rc, it, fr, hist = B.xdg_solve(S.h, S.vec(0), x)
    assert rc == 0 and it == 0 and fr == 0.0
    assert float(torch.count_nonzero(x)) == 0
    S.close()


@pytest.mark.parametrize("name", ["c1", "c2n8", "c4n8p4"])
def test_orthomg_one_cycle(name, torch):
    """One cycle of the orthonormalisation multigrid from x = 0 against the
    oracle's cycle (Gauss-Jordan vs Cholesky coarse inverses: the kappa bound
    of the V-cycle test)."""
    from oracle import orthomg
    from paper_2003_02431_amd import binding as B
    pr, H, _ = _case(name, torch)
    b = np.asarray(pr.b).reshape(-1)
    S = B.Solver(pr, B.options(krylov=B.XDG_ORTHOMG, restart=12, maxit=1, rtol=1e-30))
    x = S.vec(0)
    rc, it, fr, hist = B.xdg_solve(S.h, S.vec(0, b), x)
    xr, hr, kr = orthomg.solve(H, b, rtol=1e-30, max_cycles=1, restart=12)
    kappa = np.linalg.cond(H.A[-1].toarray())
    e = _rel(x.cpu().numpy(), xr)
    _log(f"  {name}: one OrthoMG cycle rel diff {e:.2e}, relres gpu {hist[-1]:.3e} oracle "
         f"{hr[-1]:.3e}")
    assert rc == B.XDG_ENOCONV and it == 1 and kr == 1
    assert e <= 10 * _kappa_tol(kappa)
    S.close()


@pytest.mark.parametrize("name", ["c1", "c2n8", "c2n16"])
def test_orthomg_solve(name, torch):
    """The orthonormalisation-multigrid solver to rel.res 1e-10 (restart 12):
    cycle count within 1 of the oracle's, residual histories alike, error
    against the oracle's x* <= 1e-8."""
    from oracle import mg, orthomg
    from paper_2003_02431_amd import binding as B
    pr, H, _ = _case(name, torch)
    b = np.asarray(pr.b).reshape(-1)
    S = B.Solver(pr, B.options(krylov=B.XDG_ORTHOMG, restart=12, maxit=400, rtol=1e-10))
    x = S.vec(0)
    rc, it, fr, hist = B.xdg_solve(S.h, S.vec(0, b), x)
    xr, hr, kr = orthomg.solve(H, b, rtol=1e-10, max_cycles=400, restart=12)
    xs, _, _ = mg.pcg(H.A[0], b, H.vcycle, rtol=1e-13, maxit=2000)
    xg = x.cpu().numpy()
    tr = np.linalg.norm(b - H.A[0] @ xg) / np.linalg.norm(b)
    m = min(len(hist), len(hr))
    hd = float(np.max(np.abs(np.log10(hist[:m]) - np.log10(hr[:m]))))
    err = _rel(xg, xs)
    _log(f"  {name}: OrthoMG gpu cycles={it} oracle={kr} relres={tr:.2e} "
         f"max |log10 hist diff|={hd:.2e} err vs x*={err:.2e}")
    assert rc == 0 and abs(it - kr) <= 1 and tr <= 1.05e-10
    assert hd <= 0.05 and err <= 1e-8
    assert all(h1 <= h0 * (1 + 1e-10) for h0, h1 in zip(hist, hist[1:]))
    S.close()


@pytest.mark.parametrize("krylov", ["cg", "fgmres", "orthomg"])
def test_non_finite_input_is_rejected(krylov, torch):
    """A NaN in b or in the initial guess returns XDG_EINVAL before any
    iteration (no NaN propagates into a 'converged' answer)."""
    from paper_2003_02431_amd import binding as B
    pr, H, _ = _case("c2n8", torch)
    K_ = {"cg": B.XDG_CG, "fgmres": B.XDG_FGMRES, "orthomg": B.XDG_ORTHOMG}[krylov]
    S = B.Solver(pr, B.options(krylov=K_, restart=12, rtol=1e-10))
    b = np.asarray(pr.b, dtype=np.float64).reshape(-1).copy()
    bad = b.copy()
    bad[5] = np.nan
    with pytest.raises(B.XdgError) as e:
        B.xdg_solve(S.h, S.vec(0, bad), S.vec(0))
    assert e.value.code == B.XDG_EINVAL
    x0 = np.zeros_like(b)
    x0[7] = np.inf
    with pytest.raises(B.XdgError) as e:
        B.xdg_solve(S.h, S.vec(0, b), S.vec(0, x0))
    assert e.value.code == B.XDG_EINVAL
    # the handle still solves afterwards
    x = S.vec(0)
    rc, it, fr, _ = B.xdg_solve(S.h, S.vec(0, b), x)
    assert rc == 0 and fr <= 1.05e-10
    S.close()


def test_mixed_vcycle_is_fp32(torch):
    """The mixed handle's V-cycle runs in FP32: it differs from the FP64 cycle
    by FP32 rounding, not by zero and not by more."""
    from paper_2003_02431_amd import binding as B
    pr, H, S = _case("c2n16", torch)
    Sm = B.Solver(pr, B.options(krylov=B.XDG_FGMRES, precision=B.XDG_MIXED))
    r = np.random.default_rng(16).uniform(-1, 1, H.A[0].shape[0])
    z64, z32 = S.vec(0), Sm.vec(0)
    B.xdg_vcycle(S.h, S.vec(0, r), z64)
    B.xdg_vcycle(Sm.h, Sm.vec(0, r), z32)
    d = _rel(z32.cpu().numpy(), z64.cpu().numpy())
    _log(f"  mixed vs fp64 V-cycle rel diff {d:.2e}")
    assert 1e-9 < d < 1e-3
    Sm.close()


def test_update_matrix_and_errors(torch):
    from paper_2003_02431_amd import binding as B
    pr, H, S = _case("c2n8", torch)
    b = S.vec(0, pr.b)
    x1 = S.vec(0)
    B.xdg_solve(S.h, b, x1)
    # same values again -> bitwise identical hierarchy and solve
    val = torch.as_tensor(np.ascontiguousarray(pr.val)).cuda()
    B.xdg_update_matrix(S.h, val)
    x2 = S.vec(0)
    B.xdg_solve(S.h, b, x2)
    assert torch.equal(x1, x2)
    # 2 M x = b  ->  x/2
    B.xdg_update_matrix(S.h, 2.0 * val)
    x3 = S.vec(0)
    B.xdg_solve(S.h, b, x3)
    assert _rel(x3.cpu().numpy(), 0.5 * x1.cpu().numpy()) <= 1e-9
    B.xdg_update_matrix(S.h, val)
    # iteration limit: status XDG_ENOCONV with a partial history
    S2 = B.Solver(pr, B.options(maxit=2))
    x4 = S2.vec(0)
    rc, it, fr, hist = B.xdg_solve(S2.h, b, x4)
    assert rc == B.XDG_ENOCONV and it == 2 and len(hist) == 3
    S2.close()
    # a negated diagonal block is not SPD
    bad = pr.val.copy()
    d0 = int(np.flatnonzero(pr.col_idx[pr.row_ptr[0]:pr.row_ptr[1]] == 0)[0])
    bad[d0] = -bad[d0]
    with pytest.raises(B.XdgError) as e:
        B.xdg_create(pr.row_ptr, pr.col_idx, bad, pr.cell_ptr, pr.transfers, B.options())
    assert e.value.code == B.XDG_ENOTSPD


@pytest.mark.parametrize("name", ["c2n8", "c2n16", "c4n8p4", "c2n8hp"])
def test_update_cells_equals_full_update(name, torch):
    """New values with the rows and columns of a set of cells scaled (the cut
    cells carrying both species, S M S with S = 1.25 there, still SPD): the
    partial update of those cells gives the hierarchy, every cell inverse,
    the coarsest inverse and the solve of the full update bit for bit, and
    differs from the hierarchy before the update."""
    from paper_2003_02431_amd import binding as B
    pr, H, S0 = _case(name, torch)
    cp = np.asarray(pr.cell_ptr)
    cells = np.flatnonzero(np.diff(cp) == 2)
    if cells.size == 0:
        cells = np.arange(0, len(cp) - 1, 7)
    scale = np.ones(pr.n_rows)
    for c in cells:
        scale[cp[c]:cp[c + 1]] = 1.25
    row_of = np.repeat(np.arange(pr.n_rows), np.diff(pr.row_ptr))
    val2 = pr.val * (scale[row_of] * scale[pr.col_idx])[:, None, None]
    v2 = torch.as_tensor(np.ascontiguousarray(val2)).cuda()
    opt = B.options(rtol=1e-10, maxit=600)
    Sf, Sp = B.Solver(pr, opt), B.Solver(pr, opt)
    B.xdg_update_matrix(Sf.h, v2)
    B.xdg_update_cells(Sp.h, v2, cells)
    nlev = H.nlev
    for l in range(nlev):
        a, b = B.xdg_get_level_matrix(Sf.h, l), B.xdg_get_level_matrix(Sp.h, l)
        assert all(np.array_equal(u, w) for u, w in zip(a, b)), f"level {l}"
    a0 = B.xdg_get_level_matrix(S0.h, 1)[2]
    assert not np.array_equal(a0, B.xdg_get_level_matrix(Sp.h, 1)[2])
    for l in range(nlev - 1):
        n_cells = len(H.cell_ptr[l]) - 1
        for c in range(n_cells):
            assert np.array_equal(B.xdg_get_cell_inverse(Sf.h, l, c),
                                  B.xdg_get_cell_inverse(Sp.h, l, c)), f"level {l} cell {c}"
    assert np.array_equal(B.xdg_get_cell_inverse(Sf.h, nlev - 1, 0),
                          B.xdg_get_cell_inverse(Sp.h, nlev - 1, 0))
    b = Sf.vec(0, pr.b)
    xf, xp = Sf.vec(0), Sp.vec(0)
    rf = B.xdg_solve(Sf.h, b, xf)
    rp = B.xdg_solve(Sp.h, b, xp)
    _log(f"  {name}: {cells.size} cells updated, solve it {rf[1]} / {rp[1]}")
    assert rf[0] == 0 and rp[0] == 0 and torch.equal(xf, xp)
    # against the oracle's hierarchy of the changed values: every Galerkin
    # level, sampled cell inverses and the solve
    from oracle import mg
    H2 = mg.Hierarchy(pr.row_ptr, pr.col_idx, val2, pr.cell_ptr, pr.transfers)
    for l in range(nlev):
        G = mg.block_matrix(*B.xdg_get_level_matrix(Sp.h, l))
        d = abs(G - H2.A[l]).max() / abs(H2.A[l]).max()
        assert d <= 1e-13, (l, d)
    for l in range(nlev - 1):
        _, invs = mg.cell_block_inverses(H2.A[l], H2.cell_ptr[l], H2.np[l])
        lv_cells = cells if l == 0 else np.unique(np.linspace(0, len(invs) - 1, 20).astype(int))
        for c in lv_cells[:40]:
            Dg = B.xdg_get_cell_inverse(Sp.h, l, int(c))
            assert _rel(Dg, invs[c]) <= _kappa_tol(np.linalg.cond(invs[c])), (l, c)
    Ac = H2.A[-1].toarray()
    kc = np.linalg.cond(Ac)
    assert _rel(B.xdg_get_cell_inverse(Sp.h, nlev - 1, 0), np.linalg.inv(Ac)) <= _kappa_tol(kc)
    xo, _, ito = mg.pcg(H2.A[0], pr.b, H2.vcycle, rtol=1e-10, maxit=600)
    eo = _rel(xp.cpu().numpy(), xo)
    _log(f"  {name}: partial update vs oracle hierarchy of the new values: solve it "
         f"{rp[1]} (oracle {ito}), x rel diff {eo:.2e}")
    assert abs(rp[1] - ito) <= 1 and eo <= 1e-8
    with pytest.raises(B.XdgError):
        B.xdg_update_cells(Sp.h, v2, [int(cells[0]), int(cells[0])])
    with pytest.raises(B.XdgError):
        B.xdg_update_cells(Sp.h, v2, [len(cp) - 1])
    Sf.close()
    Sp.close()


# the benchmark's smoother on the 32^3 workload (bench.py defaults)
BENCH_NU, BENCH_OMEGA, BENCH_NU_COARSE = 1, 0.9, 4


def test_full_size_sampled(torch):
    """The 32^3 p=3 workload in the launch configuration the benchmark uses
    (its hierarchy and smoother): sampled SpMV rows against the oracle, every
    Galerkin level in full, sweeps, a V-cycle and the PCG iterate against the
    oracle, and the oracle's residual of the GPU solution."""
    from oracle import mg
    from paper_2003_02431_amd import binding as B
    from xdg_inputs import problems
    _log("[gpu-parity] generating 32^3 p=3 workload")
    pr = problems.c2(seed=0, n=32, verbose=True)
    A = mg.block_matrix(pr.row_ptr, pr.col_idx, pr.val)
    S = B.Solver(pr, B.options(rtol=1e-10, maxit=600, nu_pre=BENCH_NU, nu_post=BENCH_NU,
                               omega=BENCH_OMEGA, nu_coarse=BENCH_NU_COARSE))
    rng = np.random.default_rng(15)
    x = rng.uniform(-1, 1, A.shape[0])
    y = S.vec(0)
    B.xdg_spmv(S.h, 0, S.vec(0, x), y)
    rows = rng.choice(pr.n_rows, 300, replace=False)
    idx = (rows[:, None] * pr.np + np.arange(pr.np)).reshape(-1)
    ref = A[idx] @ x
    assert _rel(y.cpu().numpy()[idx], ref) <= 1e-13
    _log("[gpu-parity] oracle hierarchy at 32^3")
    H = mg.hierarchy_of(pr, omega=BENCH_OMEGA, nu=BENCH_NU, nu_coarse=BENCH_NU_COARSE)
    for l in range(1, H.nlev):
        rp, ci, val = B.xdg_get_level_matrix(S.h, l)
        G = mg.block_matrix(rp, ci, val)
        assert abs(G - H.A[l]).max() / abs(H.A[l]).max() <= 1e-13
    xs = S.vec(0)
    rc, it, fr, hist = B.xdg_solve(S.h, S.vec(0, pr.b), xs)
    tr = np.linalg.norm(pr.b - A @ xs.cpu().numpy()) / np.linalg.norm(pr.b)
    _log(f"  32^3: PCG it={it} gpu relres={fr:.2e} oracle relres={tr:.2e}")
    assert rc == 0 and tr <= 1.05e-10
    # the preconditioner is symmetric: <B r1, r2> = <r1, B r2>
    r1, r2 = rng.uniform(-1, 1, (2, A.shape[0]))
    z1, z2 = S.vec(0), S.vec(0)
    B.xdg_vcycle(S.h, S.vec(0, r1), z1)
    B.xdg_vcycle(S.h, S.vec(0, r2), z2)
    a, b = float(z1.cpu().numpy() @ r2), float(r1 @ z2.cpu().numpy())
    assert abs(a - b) <= 1e-10 * abs(a)
    # two smoother sweeps on level 0 and one V-cycle against the oracle
    # largest condition number of the cell blocks: every cut cell with two
    # species (the ill-conditioned ones) and a sample of the others
    cp0, A0 = H.cell_ptr[0], H.A[0].tocsr()
    cand = np.union1d(np.flatnonzero(np.diff(cp0) == 2),
                      np.linspace(0, len(cp0) - 2, 400).astype(int))
    kmax = 1.0
    for c in cand:
        lo, hi = cp0[c] * pr.np, cp0[c + 1] * pr.np
        kmax = max(kmax, np.linalg.cond(A0[lo:hi, lo:hi].toarray()))
    bb, x0 = rng.uniform(-1, 1, (2, A.shape[0]))
    xsw = S.vec(0, x0)
    B.xdg_smooth(S.h, 0, S.vec(0, bb), xsw, 2)
    esw = _rel(xsw.cpu().numpy(), mg.jacobi(H.A[0], H.Dinv[0], bb, x0, BENCH_OMEGA, 2))
    kc = np.linalg.cond(H.A[-1].toarray())
    ev = _rel(z1.cpu().numpy(), H.vcycle(r1))
    _log(f"  32^3: two sweeps rel err {esw:.2e} (cell kappa {kmax:.1e}), V-cycle rel err "
         f"{ev:.2e} (coarse kappa {kc:.1e})")
    assert esw <= _kappa_tol(kmax) and ev <= _kappa_tol(kc)
    # the FP64 contract at the benchmarked size: the PCG iterate after the
    # oracle's iteration count (the plain-loop C++ oracle, pinned against the
    # numpy one, runs the 32^3 solve on all host cores)
    from oracle import mg_omp
    if not os.path.exists(mg_omp.LIB):
        mg_omp.build()
    O = mg_omp.OmpHierarchy(pr, omega=BENCH_OMEGA, nu=BENCH_NU, nu_coarse=BENCH_NU_COARSE)
    xo, ho, ito = O.pcg(pr.b, rtol=1e-10, maxit=600)
    O.close()
    B.xdg_set_tolerance(S.h, 1e-300, ito)
    xk = S.vec(0)
    rck, itk, _, _ = B.xdg_solve(S.h, S.vec(0, pr.b), xk)
    ek = _rel(xk.cpu().numpy(), xo)
    _log(f"  32^3: PCG iterate {itk} (oracle converged in {ito}) rel diff {ek:.2e}")
    assert rck == B.XDG_ENOCONV and itk == ito and abs(it - ito) <= 1 and ek <= 1e-11
    S.close()
