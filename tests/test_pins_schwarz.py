"""Pins of the additive Schwarz oracle (oracle/schwarz.py; Section 3.3,
Algorithms pMultigrid and Swz) and of the overlapping block generator, on the
2D p=2 problem (6 modes per row; np_lo = 3 keeps the p <= 1 modes):
  * one block holding every cell with np_lo = np is the direct solve;
  * single-cell blocks with np_lo = np are block Jacobi (Cholesky inverses);
  * np_lo < np: the result solves the low-order block system and then, per
    cell, the high-order system with the updated residual (the two steps of
    pMultigrid, checked through their residuals);
  * on a matrix without coupling between cells, overlapping blocks give the
    cell-block solve again (the division by the multiplicity);
  * listing every block twice changes nothing;
  * generated blocks: cores partition the cells, every block holds its core
    and stays within the low-order budget.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp


@pytest.fixture(scope="module")
def prob():
    from xdg_inputs import problems
    from oracle import mg
    pr = problems.c1(n=16, p=2)
    H = mg.hierarchy_of(pr)
    b = np.random.default_rng(3).uniform(-1, 1, H.A[0].shape[0])
    return pr, H, b


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _single_cells(n_cells):
    return np.arange(n_cells + 1, dtype=np.int32), np.arange(n_cells, dtype=np.int32)


def test_one_block_is_the_direct_solve(prob):
    from oracle import schwarz
    pr, H, b = prob
    n_cells = len(pr.cell_ptr) - 1
    A = H.A[0]
    x = schwarz.swz(A, b, pr.cell_ptr, [0, n_cells], np.arange(n_cells), H.np[0], H.np[0])
    ref = sla.cho_solve(sla.cho_factor(A.toarray()), b)
    assert _rel(x, ref) <= 1e-11


def test_single_cell_blocks_are_block_jacobi(prob):
    from oracle import schwarz
    pr, H, b = prob
    bp, bc = _single_cells(len(pr.cell_ptr) - 1)
    x = schwarz.swz(H.A[0], b, pr.cell_ptr, bp, bc, H.np[0], H.np[0])
    assert _rel(x, H.Dinv[0] @ b) <= 1e-12


def _lo_hi(rows, Np, np_lo):
    rows = np.asarray(rows)
    lo = (rows[:, None] * Np + np.arange(np_lo)[None, :]).reshape(-1)
    hi = (rows[:, None] * Np + np.arange(np_lo, Np)[None, :]).reshape(-1)
    return lo, hi


@pytest.mark.parametrize("whole", [False, True])
def test_pmg_steps_through_their_residuals(prob, whole):
    from oracle import schwarz
    pr, H, b = prob
    A = H.A[0].tocsr()
    Np, np_lo = H.np[0], 3
    cp = np.asarray(pr.cell_ptr)
    n_cells = len(cp) - 1
    cells = np.arange(n_cells) if whole else np.array([5])
    x = schwarz.pmg(A, b, cp, cells, Np, np_lo)
    rows = schwarz.block_rows(cp, cells)
    lo, hi = _lo_hi(rows, Np, np_lo)
    # low-order step: M_lo x_lo = b_lo on the block
    e_lo = A[lo][:, lo] @ x[lo] - b[lo]
    assert np.linalg.norm(e_lo) <= 1e-12 * np.linalg.norm(b[lo])
    # high-order step per cell with r = b - M x_lo
    x_lo = np.zeros_like(b)
    x_lo[lo] = x[lo]
    r = b - A @ x_lo
    for j in cells:
        _, hj = _lo_hi(np.arange(cp[j], cp[j + 1]), Np, np_lo)
        e = A[hj][:, hj] @ x[hj] - r[hj]
        assert np.linalg.norm(e) <= 1e-12 * max(np.linalg.norm(r[hj]), 1e-300)
    # nothing outside the block
    outside = np.setdiff1d(np.arange(b.size), np.concatenate([lo, hi]))
    assert np.all(x[outside] == 0.0)


def test_overlap_on_decoupled_cells_divides_by_multiplicity(prob):
    from oracle import schwarz, mg
    from xdg_inputs import schwarz_blocks as SB
    pr, H, b = prob
    Np = H.np[0]
    cp = np.asarray(pr.cell_ptr)
    # keep only the couplings inside each cell block
    A = H.A[0].tocoo()
    cell_of = np.repeat(np.arange(len(cp) - 1), np.diff(cp) * Np)
    keep = cell_of[A.row] == cell_of[A.col]
    Ad = sp.csr_matrix((A.data[keep], (A.row[keep], A.col[keep])), shape=A.shape)
    bp, bc = SB.schwarz_blocks(pr.row_ptr, pr.col_idx, pr.cell_ptr, 3, max_lo=60)
    assert len(bc) > len(cp) - 1                     # there is overlap
    x = schwarz.swz(Ad, b, cp, bp, bc, Np, Np)
    Dinv = mg.cell_block_inverses(Ad, cp, Np)[0]
    assert _rel(x, Dinv @ b) <= 1e-12


def test_duplicated_blocks_change_nothing(prob):
    from oracle import schwarz
    from xdg_inputs import schwarz_blocks as SB
    pr, H, b = prob
    bp, bc = SB.schwarz_blocks(pr.row_ptr, pr.col_idx, pr.cell_ptr, 3, max_lo=60)
    x1 = schwarz.swz(H.A[0], b, pr.cell_ptr, bp, bc, H.np[0], 3)
    blocks = [bc[bp[i]:bp[i + 1]] for i in range(len(bp) - 1)]
    twice = [blk for blk in blocks for _ in range(2)]
    bp2 = np.concatenate([[0], np.cumsum([len(t) for t in twice])])
    x2 = schwarz.swz(H.A[0], b, pr.cell_ptr, bp2, np.concatenate(twice), H.np[0], 3)
    assert _rel(x2, x1) <= 1e-14


def test_generated_blocks(prob):
    from xdg_inputs import schwarz_blocks as SB
    pr, H, b = prob
    cp = np.asarray(pr.cell_ptr)
    rows = np.diff(cp)
    nbr = SB.cell_graph(pr.row_ptr, pr.col_idx, pr.cell_ptr)
    for overlap in (True, False):
        bp, bc = SB.schwarz_blocks(pr.row_ptr, pr.col_idx, pr.cell_ptr, 3, max_lo=60,
                                   overlap=overlap)
        blocks = [set(bc[bp[i]:bp[i + 1]].tolist()) for i in range(len(bp) - 1)]
        assert set().union(*blocks) == set(range(len(rows)))
        for blk in blocks:
            assert rows[list(blk)].sum() * 3 <= 60
        if not overlap:
            assert sum(len(blk) for blk in blocks) == len(rows)      # a partition
        else:
            # some block holds a cell together with all of its neighbours
            assert any({c, *nbr[c]} <= blk for blk in blocks for c in blk)
    # the graph is symmetric (SIP couples both ways)
    for c, ns in enumerate(nbr):
        for d in ns:
            assert c in nbr[d]
