"""The 16-right-hand-side path at full size (64^3 ellipsoid workload at p = 3
and p = 4, the configurations the multi-RHS benchmark runs; at p = 4 the
level-0 block arrays hold 1,833,848 x 35^2 = 2.25e9 entries, more than 2^31,
so every block offset must be 64-bit), checked on sampled outputs that the
oracle's definitions give one row or one cell at a time:
  * FP64 MFMA block product: sampled rows y_i = sum_b M_ib X_b within 1e-13;
  * FP32 MFMA block product: sampled rows against the same sum over the
    operator and X rounded to FP32, within 1e-6 (the kernel's accumulation);
  * FP32 MFMA smoother sweep: sampled cells against
    x_c + omega D_c^{-1} (b - M x)_c with FP32-rounded operators, inside the
    componentwise bound of k-term FP32 accumulations (gamma_k = k 2^-24).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
K = 16
U32 = 2.0 ** -24


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=[3, 4])
def case(request, problem_cache):
    import torch
    from paper_2003_02431_amd import binding as B
    from xdg_inputs import problems
    assert torch.cuda.is_available()
    p = request.param
    _log(f"[gpu-fullsize] generating the 64^3 p={p} 16-column workload")
    if p == 3:
        pr = problem_cache(("c4", 0, 64, 3), lambda: problems.c4(seed=0, n=64, p=3, nrhs=K,
                                                                     verbose=True))
    else:
        pr = problems.c4(seed=0, n=64, p=p, nrhs=K, verbose=True)
        if pr.col_idx.size * pr.np * pr.np <= 2 ** 31:
            raise AssertionError("the p = 4 case must exceed 2^31 block entries")
    S = B.Solver(pr, B.options(krylov=B.XDG_FGMRES, precision=B.XDG_MIXED, nrhs=K,
                               restart=20, rtol=1e-8, maxit=2000))
    _log(f"[gpu-fullsize] rows={pr.n_rows} nnzb={pr.col_idx.size}")
    yield pr, S
    S.close()


def _row(pr, i, X, f32=False):
    """sum_b M_ib X_b for block row i (np x 16)."""
    out = np.zeros((pr.np, K))
    for b in range(pr.row_ptr[i], pr.row_ptr[i + 1]):
        Mb = pr.val[b]
        Xb = X[pr.col_idx[b] * pr.np:(pr.col_idx[b] + 1) * pr.np]
        if f32:
            Mb = Mb.astype(np.float32).astype(np.float64)
        out += Mb @ Xb
    return out


def test_spmm_sampled(case):
    from paper_2003_02431_amd import binding as B
    pr, S = case
    L = pr.n_rows * pr.np
    rng = np.random.default_rng(31)
    X = rng.uniform(-1, 1, (L, K))
    # random rows plus the last ones (at p = 4 their blocks lie beyond entry 2^31)
    rows = np.union1d(rng.choice(pr.n_rows - 20, 180, replace=False),
                      np.arange(pr.n_rows - 20, pr.n_rows))
    for prec, tol in ((B.XDG_FP64, 1e-13), (B.XDG_MIXED, 1e-6)):
        Y = S.vec(0)
        B.xdg_spmm(S.h, 0, prec, S.vec(0, X), Y)
        y = Y.cpu().numpy().reshape(L, K)
        Xr = X if prec == B.XDG_FP64 else X.astype(np.float32).astype(np.float64)
        got = np.concatenate([y[i * pr.np:(i + 1) * pr.np] for i in rows])
        ref = np.concatenate([_row(pr, i, Xr, prec != B.XDG_FP64) for i in rows])
        e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        _log(f"  64^3 {pr.np} modes spmm precision {prec}: sampled rel err {e:.2e} (tol {tol:g})")
        assert e <= tol


def test_smoother_sampled(case):
    from paper_2003_02431_amd import binding as B
    pr, S = case
    L = pr.n_rows * pr.np
    Np = pr.np
    rng = np.random.default_rng(32)
    b = rng.uniform(-1, 1, (L, K))
    x0 = rng.uniform(-1, 1, (L, K))
    x = S.vec(0, x0)
    B.xdg_smooth(S.h, 0, S.vec(0, b), x, 1)
    xg = x.cpu().numpy().reshape(L, K)
    r32 = lambda v: np.asarray(v, dtype=np.float32).astype(np.float64)
    b32, x32 = r32(b), r32(x0)
    cp = np.asarray(pr.cell_ptr)
    n_cells = len(cp) - 1
    cells = np.union1d(rng.choice(n_cells - 10, 90, replace=False),
                       np.arange(n_cells - 10, n_cells))
    worst = 0.0
    for c in cells:
        rows = np.arange(cp[c], cp[c + 1])
        n = len(rows) * Np
        # diagonal cell block and its inverse (FP64, then rounded like the stored copy)
        Dc = np.zeros((n, n))
        Aabs_x = np.zeros((n, K))
        Ax = np.zeros((n, K))
        kA = 0
        for ii, i in enumerate(rows):
            kA = max(kA, (pr.row_ptr[i + 1] - pr.row_ptr[i]) * Np)
            for bb in range(pr.row_ptr[i], pr.row_ptr[i + 1]):
                j = pr.col_idx[bb]
                M32 = r32(pr.val[bb])
                Xj = x32[j * Np:(j + 1) * Np]
                Ax[ii * Np:(ii + 1) * Np] += M32 @ Xj
                Aabs_x[ii * Np:(ii + 1) * Np] += abs(M32) @ abs(Xj)
                if j in rows:
                    jj = int(np.where(rows == j)[0][0])
                    Dc[ii * Np:(ii + 1) * Np, jj * Np:(jj + 1) * Np] = pr.val[bb]
        Dinv = r32(np.linalg.inv(Dc))
        idx = (rows[:, None] * Np + np.arange(Np)).reshape(-1)
        r = b32[idx] - Ax
        y = Dinv @ r
        ref = x32[idx] + np.float32(0.7) * y
        dr = kA * U32 * (abs(b32[idx]) + Aabs_x)
        dy = n * U32 * (abs(Dinv) @ abs(r)) + abs(Dinv) @ dr
        dx = U32 * (abs(ref) + 0.7 * abs(y)) + 0.7 * dy
        worst = max(worst, float(np.max(abs(xg[idx] - ref) / np.maximum(dx, 1e-300))))
    _log(f"  64^3 p={pr.np} modes MFMA smoother: {cells.size} sampled cells, worst |err| / bound "
         f"{worst:.2e}")
    assert worst <= 1.0
