"""The learned smoother's training pairs at full size (64^3 p=3 random
ellipsoid, the configuration of the learned-smoother benchmark), checked on
sampled cells against the definition evaluated one cell at a time:
    r = b - M x_k on the cell's rows,  j = omega D_c^{-1} r_c,  s = |j|,
    X = [ j / s in species slots | geometry ],  T = (x* - x_k - j) / s,
with the FP64 values rounded once to FP32 (relative 2.5e-7 per entry, a floor
of 1e-9 of the sample's norm for entries that cancel).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
NP = 20


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_pairs_sampled_64(problem_cache):
    import torch
    from paper_2003_02431_amd import binding as B
    from xdg_inputs import features, problems
    assert torch.cuda.is_available()
    _log("[gpu-fullsize-learned] generating the 64^3 p=3 ellipsoid workload and cell features")
    # the 16-column full-size test shares this problem (first right-hand side here)
    pr = problem_cache(("c4", 0, 64, 3), lambda: problems.c4(seed=0, n=64, p=3, nrhs=16,
                                                                     verbose=True))
    b = np.ascontiguousarray(np.asarray(pr.b)[:, 0])
    rs, g = features.cell_features(pr)
    S = B.Solver(pr, B.options(krylov=B.XDG_FGMRES, restart=30, rtol=1e-8, maxit=100))
    B.xdg_set_cell_features(S.h, rs, g)
    rng = np.random.default_rng(41)
    L = b.size
    xk, xs = rng.uniform(-1, 1, L), rng.uniform(-1, 1, L)
    cell0, step = 3, 97
    n_sel = len(range(cell0, S.n_cells, step))
    X = torch.empty((n_sel, 45), dtype=torch.float32, device="cuda")
    T = torch.empty((n_sel, 40), dtype=torch.float32, device="cuda")
    n = B.xdg_learned_pairs(S.h, S.vec(0, b), S.vec(0, xk), S.vec(0, xs), cell0, step, X, T)
    assert n == n_sel
    Xg, Tg = X.cpu().numpy().astype(np.float64), T.cpu().numpy().astype(np.float64)
    cp = np.asarray(pr.cell_ptr)
    worst_x = worst_t = 0.0
    for k in range(0, n_sel, max(1, n_sel // 200)):
        c = cell0 + k * step
        rows = np.arange(cp[c], cp[c + 1])
        m = len(rows) * NP
        Dc = np.zeros((m, m))
        r = np.zeros(m)
        for ii, i in enumerate(rows):
            acc = b[i * NP:(i + 1) * NP].copy()
            for bb in range(pr.row_ptr[i], pr.row_ptr[i + 1]):
                l = pr.col_idx[bb]
                acc -= pr.val[bb] @ xk[l * NP:(l + 1) * NP]
                if cp[c] <= l < cp[c + 1]:
                    jj = l - cp[c]
                    Dc[ii * NP:(ii + 1) * NP, jj * NP:(jj + 1) * NP] = pr.val[bb]
            r[ii * NP:(ii + 1) * NP] = acc
        j = 0.7 * np.linalg.solve(Dc, r)
        s = np.linalg.norm(j)
        F = np.zeros(45)
        Tt = np.zeros(40)
        for ii, i in enumerate(rows):
            sl = NP * int(rs[i])
            idx = slice(i * NP, (i + 1) * NP)
            F[sl:sl + NP] = j[ii * NP:(ii + 1) * NP] / s
            Tt[sl:sl + NP] = (xs[idx] - xk[idx] - j[ii * NP:(ii + 1) * NP]) / s
        F[40:] = g[c]

        def err(a, ref):
            floor = 1e-9 * np.linalg.norm(ref) + 1e-300
            return float(np.max(np.abs(a - ref) / (np.abs(ref) + floor)))
        worst_x = max(worst_x, err(Xg[k], F))
        worst_t = max(worst_t, err(Tg[k], Tt))
    _log(f"  64^3 pairs: {n_sel} selected, sampled max rel err X {worst_x:.2e} T {worst_t:.2e}")
    assert worst_x <= 2.5e-7 and worst_t <= 2.5e-7
    S.close()
