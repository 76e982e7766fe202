"""Overlapping cell blocks for the additive Schwarz smoother (Section 3.3,
Algorithm Swz takes a pre-computed partitioning of the cells as input; the
paper partitions with METIS and then enlarges every part by its neighbour
cells).  This module stands in for that partitioner: greedy graph growing on
the level-0 cell graph, then one layer of neighbour cells.  Pure index
bookkeeping on the matrix pattern; nothing here applies an operator.

Cell graph: smoother cells c, d are neighbours when some block row of c has a
block column in d (the SIP operator couples cells that share a face).
Cores: cells are visited in index order; an unassigned cell starts a core,
which grows breadth-first over unassigned neighbours while the enlarged block
(core plus neighbours) keeps at most `max_lo` low-order unknowns
(block rows x np_lo) and the core at most `max_core` cells.  Block = core plus
its neighbours (overlap); with overlap=False the block is the core alone.
"""
import numpy as np


def cell_graph(row_ptr, col_idx, cell_ptr):
    """Neighbour lists (sorted, without the cell itself) of the smoother cells."""
    cp = np.asarray(cell_ptr)
    n_cells = len(cp) - 1
    cell_of_row = np.repeat(np.arange(n_cells), np.diff(cp))
    rp = np.asarray(row_ptr)
    ci = np.asarray(col_idx)
    src = np.repeat(cell_of_row, np.diff(rp))
    dst = cell_of_row[ci]
    pairs = np.unique(np.stack([src, dst], axis=1), axis=0)
    pairs = pairs[pairs[:, 0] != pairs[:, 1]]
    starts = np.searchsorted(pairs[:, 0], np.arange(n_cells + 1))
    return [pairs[starts[c]:starts[c + 1], 1].tolist() for c in range(n_cells)]


def schwarz_blocks(row_ptr, col_idx, cell_ptr, np_lo, max_lo=88, max_core=64, overlap=True):
    """(block_ptr int32 [n_blocks + 1], block_cells int32) of the overlapping
    blocks; cells ascending within a block."""
    cp = np.asarray(cell_ptr)
    rows = np.diff(cp)
    nbr = cell_graph(row_ptr, col_idx, cell_ptr)
    n_cells = len(rows)
    assigned = np.zeros(n_cells, dtype=bool)
    blocks = []

    def lo(cells):
        return int(rows[list(cells)].sum()) * np_lo

    def enlarge(core):
        if not overlap:
            return set(core)
        out = set(core)
        for c in core:
            out.update(nbr[c])
        return out

    for c0 in range(n_cells):
        if assigned[c0]:
            continue
        core = [c0]
        assigned[c0] = True
        block = enlarge(core)
        queue = [d for d in nbr[c0] if not assigned[d]]
        qi = 0
        while qi < len(queue) and len(core) < max_core:
            d = queue[qi]
            qi += 1
            if assigned[d]:
                continue
            trial = block | enlarge([d])
            if lo(trial) > max_lo:
                continue
            core.append(d)
            assigned[d] = True
            block = trial
            queue.extend(e for e in nbr[d] if not assigned[e])
        if lo(block) > max_lo:
            # a single core cell whose neighbours exceed the budget: keep the
            # nearest neighbours in index order until the budget is reached
            keep = set(core)
            for d in sorted(block - set(core)):
                if lo(keep | {d}) <= max_lo:
                    keep.add(d)
            block = keep
        blocks.append(sorted(block))
    ptr = np.zeros(len(blocks) + 1, dtype=np.int32)
    ptr[1:] = np.cumsum([len(b) for b in blocks])
    return ptr, np.concatenate(blocks).astype(np.int32)
