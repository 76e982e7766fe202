"""Two time levels of a moving interface (Section 2.3): the agglomerated
space of the new time level and the L2 re-projection of the old solution.

The paper agglomerates, for the step t0 -> t1, every cut part that is below
the volume-fraction threshold alpha and every part that is new (present at t1,
absent at t0) into its largest same-species neighbour, so that the meshes of
both time levels have the same topology.  After a time step the solution is
injected into the non-agglomerated cut-cell space and projected in L2 onto
the (possibly different) agglomerated space of the next step, where it serves
as the initial value.

moving_pair() builds both problems and that projection:
  * pr0: the t0 problem on its own agglomerated space (A_alpha at t0);
  * pr1: the t1 problem on the space of A_{alpha,t1,t0} (alpha rule at t1
    plus the new parts);
  * Pi: block-sparse operator from the t0 space to the t1 space, np x np
    row-major blocks: the old solution restricted to a cut part K_{j,s}(t0)
    is the polynomial of the t0 aggregate containing it; it is extended to
    the part K_{j,s}(t1) of the same cell (a part that is new at t1 takes the
    polynomial of the first cell of its t1 aggregate that carried species s
    at t0), and projected onto the orthonormal t1 basis:
        Pi[P, Q] = sum over the cells j of P whose polynomial comes from Q of
                   int_{K_{j,s}(t1)} phi^{t1}_P phi^{t0}_Q^T dV.
    A cell that is uncut and not agglomerated at both times keeps its basis,
    so its block is the identity.
Only input data is produced here; applying Pi is the solver's work.
"""
import numpy as np

from .levelset import Quadric
from .problems import build


def moving_pair(n=16, p=3, c0=(0.0, 0.0, 0.0), shift=(0.25, 0.0, 0.0), r=0.6,
                mu=(1.0, 1000.0), alpha=0.1, hierarchy=(), q_std=None, verbose=False):
    """The sphere of radius r centred at c0 (t0) and at c0 + shift * h (t1),
    f = 1 in both phases, homogeneous Dirichlet data.  Returns (pr0, pr1, Pi)
    with Pi = dict(row_ptr, col_idx, val, n_rows, n_cols, np)."""
    h = 2.0 / n
    c0 = np.asarray(c0, dtype=np.float64)
    c1 = c0 + h * np.asarray(shift, dtype=np.float64)
    one = lambda X, s: np.ones(len(X))
    zero = lambda X, s: np.zeros(len(X))
    common = dict(hierarchy=list(hierarchy), rhs="load", f=one, g_dir=zero, alpha=alpha,
                  q_std=q_std, verbose=verbose)
    pr0 = build(f"moving_t0_p{p}_n{n}", 3, n, p, Quadric.sphere(c0, r), mu, **common)
    g0 = pr0.geom

    def new_parts(g1):
        return {(int(j), s) for j in g1.cut for s in range(2)
                if g1.present[j, s] and not g0.present[j, s]}

    pr1 = build(f"moving_t1_p{p}_n{n}", 3, n, p, Quadric.sphere(c1, r), mu,
                force_agglomerate=new_parts, **common)
    Pi = projection(pr0, pr1, q_std or p + 2)
    return pr0, pr1, Pi


def projection(pr0, pr1, q_std):
    """The L2 re-projection operator from pr0's level-0 space to pr1's."""
    L0, L1 = pr0.levels[0], pr1.levels[0]
    g0, g1 = pr0.geom, pr1.geom
    Np = L1.np
    single0 = L0.standard & (np.diff(L0.piece_ptr) == 1)
    single1 = L1.standard & (np.diff(L1.piece_ptr) == 1)
    blocks = {}
    for P in range(L1.n_rows):
        s = int(L1.species[P])
        cells = L1.pieces(P)
        donors = [int(j) for j in cells if g0.present[j, s]]
        if not donors:
            raise ValueError(f"t1 aggregate {P} has no cell of species {s} at t0")
        for j in cells:
            jj = int(j) if g0.present[j, s] else donors[0]
            Q = int(L0.part_of[2 * jj + s])
            if single1[P] and single0[Q] and L0.pieces(Q)[0] == j and jj == j:
                blk = np.eye(Np)
            else:
                X, W = g1.volume_rule(j, s, q_std)
                if len(W) == 0:
                    continue
                b1 = L1.bases[P].eval(X, grad=False)
                b0 = L0.bases[Q].eval(X, grad=False)
                blk = (b1 * W[:, None]).T @ b0
            key = (P, Q)
            blocks[key] = blocks[key] + blk if key in blocks else blk
    keys = sorted(blocks)
    rows = np.array([k[0] for k in keys], dtype=np.int64)
    cols = np.array([k[1] for k in keys], dtype=np.int32)
    row_ptr = np.zeros(L1.n_rows + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    val = np.stack([blocks[k] for k in keys])
    return dict(row_ptr=row_ptr, col_idx=cols, val=val, n_rows=L1.n_rows, n_cols=L0.n_rows,
                np=Np)
