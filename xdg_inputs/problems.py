"""Seeded synthetic XDG Poisson workloads and their multigrid hierarchies.

A Problem holds exactly what the solver boundary takes in: the level-0 block
matrix (BSR over (aggregate, species) block rows, Np x Np blocks), the
smoother cell blocks, the transfer operators between consecutive levels
(p-truncation or per-fine-block dense R_i with parent map), and right-hand
sides.  Nothing here applies an operator, smooths, restricts or solves.

Workloads (Poisson with a jump in mu, Section 1.1 Eq. poisson-jump-problem-def,
Dirichlet data on the whole boundary as in Section 4):
  c1  2D, p=2, 16^2, circle r=0.7, mu 1 | 10, f = 2 pi^2 sin(pi x) sin(pi y),
      levels p2 -> p1 -> p0.
  c2  3D, p=3, 32^3, sphere r=0.6 with centre offset ~ U[-0.05, 0.05]^3,
      mu 1 | 1000, b ~ U[-1, 1] per coefficient, levels p3 -> p1 -> 16^3 -> 8^3.
  c4  3D, 64^3, p in {2,3,4}, axis-aligned ellipsoid with semi-axes ~ U[0.4,0.7],
      mu 1 | 1000, 16 right-hand sides ~ U[-1, 1], levels p -> p1 -> 32^3 ->
      16^3 -> 8^3.
  paper  sphere r=0.7 at the origin, mu 1 | 1000 (Section 4 workload).
Agglomeration threshold alpha = 0.1 everywhere.
"""
import time

import numpy as np

from . import rng as _rng
from .assembly import C_ETA_DEFAULT, assemble, compute_penalty, load_vector
from .basis import n_modes
from .geometry import Geometry
from .levelset import Quadric
from .partition import Level, alpha_edges, dense_transfer, level_labels

T_PTRUNC, T_DENSE = 0, 1


class Problem:
    """Container of the solver inputs plus bookkeeping for diagnostics."""

    def summary(self):
        return dict(name=self.name, D=self.D, n=self.n, p=self.p, np=self.np,
                    n_rows=self.n_rows, nnzb=int(self.col_idx.size),
                    levels=len(self.transfers) + 1, dofs=self.n_rows * self.np)


def build(name, D, n, p, phi, mu, alpha=0.1, hierarchy=(), rhs="random", nrhs=1,
          rng=None, f=None, g_dir=None, q_cut=None, q_std=None, c_eta=C_ETA_DEFAULT,
          verbose=False, force_agglomerate=None):
    """Generate one problem.  `hierarchy` lists the coarse levels in order as
    ("p", degree) for a p-level on the same aggregates, ("h", m) for the
    2^m-blocking aggregation level at degree 1, or ("h", m, degree) for that
    level at another degree (the paper's aggregation sequence keeps the
    degree of the fine level)."""
    t0 = time.time()
    q_cut = q_cut or max(2 * p + 4, 8)
    q_std = q_std or p + 2
    geom = Geometry(D, n, phi, q_cut)
    force = force_agglomerate(geom) if force_agglomerate else None
    a_edges = alpha_edges(geom, alpha, force)
    L0 = Level(geom, 0, p, level_labels(geom, a_edges, 0))
    L0.build_bases(q_std)
    pen = compute_penalty(geom, L0, c_eta)
    t1 = time.time()
    if verbose:
        print(f"[{name}] geometry, agglomeration and bases: {t1 - t0:.1f}s", flush=True)
    row_ptr, col_idx, val = assemble(geom, L0, mu, pen, q_std)
    t2 = time.time()
    if verbose:
        print(f"[{name}] assembly: {t2 - t1:.1f}s", flush=True)
    pr = Problem()
    pr.name, pr.D, pr.n, pr.p, pr.np = name, D, n, p, L0.np
    pr.mu, pr.alpha, pr.c_eta = tuple(mu), alpha, c_eta
    pr.n_rows = L0.n_rows
    pr.row_ptr = row_ptr.astype(np.int32)
    pr.col_idx = col_idx.astype(np.int32)
    pr.val = val
    pr.cell_ptr = L0.cell_ptr.astype(np.int32)
    pr.geom, pr.levels, pr.penalty = geom, [L0], pen
    pr.species = L0.species.copy()
    pr.rep = L0.rep.copy()
    # transfers
    pr.transfers = []
    fine = L0
    for kind, arg, *deg_h in hierarchy:
        if kind == "p":
            lv = Level.__new__(Level)
            lv.__dict__.update({k: v for k, v in fine.__dict__.items() if k != "bases"})
            lv.deg = arg
            lv.np = n_modes(D, arg)
            lv.truncate_from(fine)
            pr.transfers.append(dict(kind=T_PTRUNC, n_rows_c=lv.n_rows, np_c=lv.np,
                                     parent=np.arange(fine.n_rows, dtype=np.int32), R=None,
                                     cell_ptr_c=lv.cell_ptr.astype(np.int32)))
        else:
            deg = deg_h[0] if deg_h else (1 if fine.deg >= 1 else 0)
            lv = Level(geom, arg, deg, level_labels(geom, a_edges, arg))
            lv.build_bases(max(deg + 1, 2))
            parent, R = dense_transfer(fine, lv, max(fine.deg + 1, 2))
            pr.transfers.append(dict(kind=T_DENSE, n_rows_c=lv.n_rows, np_c=lv.np,
                                     parent=parent.astype(np.int32), R=R,
                                     cell_ptr_c=lv.cell_ptr.astype(np.int32)))
        pr.levels.append(lv)
        fine = lv
    t3 = time.time()
    # right-hand side(s)
    L = pr.n_rows * pr.np
    if rhs == "random":
        pr.b = _rng.uniform_rhs(rng, L, nrhs)
    elif rhs == "load":
        pr.b = load_vector(geom, L0, mu, pen, q_std, f=f, g_dir=g_dir)
    else:
        raise ValueError(rhs)
    pr.times = dict(geometry=t1 - t0, assembly=t2 - t1, hierarchy=t3 - t2)
    if verbose:
        print(f"[{name}] rows={pr.n_rows} nnzb={pr.col_idx.size} "
              f"geo={t1 - t0:.1f}s asm={t2 - t1:.1f}s hier={t3 - t2:.1f}s", flush=True)
    return pr


# ---------------------------------------------------------------------------
# named workloads

def c1(n=16, p=2):
    f = lambda X, s: 2.0 * np.pi ** 2 * np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1])
    hier = [("p", q) for q in range(p - 1, -1, -1)]
    return build(f"c1_2d_p{p}_n{n}", 2, n, p, Quadric.sphere([0.0, 0.0], 0.7), (1.0, 10.0),
                 hierarchy=hier, rhs="load", f=f, g_dir=lambda X, s: np.zeros(len(X)))


def hierarchy(kind, n, p):
    """Named coarse-level sequences of the 3D workloads (n a power of 2):
      "p1h"   p -> p1 on the fine aggregates, then aggregation levels at p1 down
              to the 8^3 blocking (4 levels at 32^3);
      "h3p1"  one aggregation level at the fine degree (2^3 blocking), then p1
              on it, then aggregation levels at p1 down to 8^3 (4 levels at 32^3);
      "hp"    aggregation levels at the fine degree down to the 4^3 blocking
              (the paper's sequence: the degree is kept on every level);
      "h2p"   aggregation levels at the fine degree down to the 8^3 blocking,
              then p1 on it (4 levels at 32^3, the coarsest of "p1h")."""
    L = int(np.log2(n))
    if kind == "h2p":
        return [("h", m, p) for m in range(1, L - 2)] + [("p", 1)]
    if kind == "p1h":
        return [("p", 1)] + [("h", m) for m in range(1, L - 2)]
    if kind == "h3p1":
        return [("h", 1, p), ("p", 1)] + [("h", m) for m in range(2, L - 2)]
    if kind == "hp":
        return [("h", m, p) for m in range(1, L - 1)]
    raise KeyError(kind)


def c2(seed=0, n=32, p=3, verbose=False, hier=None, c_eta=C_ETA_DEFAULT):
    g = _rng.problem_rng(seed)
    ctr = _rng.sphere_jitter(g, 0.05)
    hier = hier or hierarchy("p1h", n, p)
    return build(f"c2_3d_p{p}_n{n}_s{seed}", 3, n, p, Quadric.sphere(ctr, 0.6), (1.0, 1000.0),
                 hierarchy=hier, rhs="random", rng=g, verbose=verbose, c_eta=c_eta)


def c4(seed=0, n=64, p=3, nrhs=16, verbose=False):
    g = _rng.problem_rng(seed)
    axes = _rng.ellipsoid_axes(g, 0.4, 0.7)
    nh = int(np.log2(n)) - 3
    hier = [("p", 1)] + [("h", m) for m in range(1, nh + 1)]
    return build(f"c4_3d_p{p}_n{n}_s{seed}", 3, n, p, Quadric.ellipsoid([0.0, 0.0, 0.0], axes),
                 (1.0, 1000.0), hierarchy=hier, rhs="random", nrhs=nrhs, rng=g, verbose=verbose)


def paper(n=16, p=3, hier=None, c_eta=C_ETA_DEFAULT, verbose=False):
    """The Section 4 workload: sphere of radius 0.7 at the origin in (-1,1)^3,
    mu 1 inside | 1000 outside, f = 1, homogeneous Dirichlet data, alpha = 0.1.
    Default hierarchy: aggregation levels at the fine degree down to 4^3
    (the paper's multigrid keeps the degree on every level)."""
    nh = int(np.log2(n)) - 2
    hier = hier if hier is not None else [("h", m, p) for m in range(1, nh + 1)]
    return build(f"paper_3d_p{p}_n{n}", 3, n, p, Quadric.sphere([0.0, 0.0, 0.0], 0.7),
                 (1.0, 1000.0), hierarchy=hier, rhs="load", f=lambda X, s: np.ones(len(X)),
                 g_dir=lambda X, s: np.zeros(len(X)), c_eta=c_eta, verbose=verbose)


def paper_sphere_fractions(n, alpha=0.1):
    """Geometry and agglomerated level-0 row count of the Section 4 workload
    (sphere of radius 0.7 at the origin in (-1,1)^3)."""
    geom = Geometry(3, n, Quadric.sphere([0.0, 0.0, 0.0], 0.7), q_cut=8)
    a_edges = alpha_edges(geom, alpha)
    lv = Level(geom, 0, 0, level_labels(geom, a_edges, 0))
    return geom, lv.n_rows
