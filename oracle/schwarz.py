"""FP64 oracle of the additive Schwarz smoother -- test infrastructure only
(imported by tests, never by the product path).

Section 3.3, Algorithm pMultigrid (PMG on a block of cells) and Algorithm Swz
(additive Schwarz over overlapping blocks, divided by the number of blocks
that contain a cell).  On a block I (a set of smoother cells; all species rows
of those cells) with np_lo leading (low-order) modes per row:
    x := 0
    x_lo := M_lo \\ b_lo      M_lo, b_lo: rows/columns m(I, -, -, < np_lo)
    r := b - M x              (x is non-zero only on the low modes of I)
    for every cell j of I:    x_hi,j := M_hi,j \\ r_hi,j
                              M_hi,j: rows/columns m(j, -, -, >= np_lo),
                              all species rows of cell j together
Swz(b) = (sum over blocks of PMG(b, I_i)) ./ alpha, alpha = per unknown the
number of blocks containing its cell.

Readings: the high-order step uses the residual r (the listing names b there
after computing r); the smoother inside the V-cycle acts on level 0 only and
is not damped beyond the division by alpha: pre-smoothing from x = 0 is
x = Swz(r) followed by x += Swz(r - M x) sweeps, post-smoothing the same
sweeps; coarser levels keep damped block Jacobi.
"""
import numpy as np



def block_rows(cell_ptr, cells):
    """Block rows of the given smoother cells, in cell order."""
    cp = np.asarray(cell_ptr)
    return np.concatenate([np.arange(cp[c], cp[c + 1]) for c in cells])


def _unknowns(rows, Np, modes):
    return (np.asarray(rows)[:, None] * Np + np.asarray(modes)[None, :]).reshape(-1)


def pmg(A, b, cell_ptr, cells, Np, np_lo):
    """Algorithm pMultigrid on the block of `cells`: returns x (full length,
    zero outside the block)."""
    A = A.tocsr()
    x = np.zeros_like(b)
    rows = block_rows(cell_ptr, cells)
    if np_lo > 0:
        I_lo = _unknowns(rows, Np, range(np_lo))
        M_lo = A[I_lo][:, I_lo].toarray()
        x[I_lo] += np.linalg.solve(M_lo, b[I_lo])
    r = b - A @ x
    if np_lo < Np:
        cp = np.asarray(cell_ptr)
        for j in cells:
            I_hi = _unknowns(np.arange(cp[j], cp[j + 1]), Np, range(np_lo, Np))
            M_hi = A[I_hi][:, I_hi].toarray()
            x[I_hi] += np.linalg.solve(M_hi, r[I_hi])
    return x


def swz(A, b, cell_ptr, block_ptr, block_cells, Np, np_lo):
    """Algorithm Swz: additive Schwarz over the blocks, scaled by 1/alpha."""
    x = np.zeros_like(b)
    alpha = np.zeros_like(b)
    for i in range(len(block_ptr) - 1):
        cells = block_cells[block_ptr[i]:block_ptr[i + 1]]
        x += pmg(A, b, cell_ptr, cells, Np, np_lo)
        rows = block_rows(cell_ptr, cells)
        alpha[_unknowns(rows, Np, range(Np))] += 1.0
    return x / alpha


class Smoother:
    """The level-0 Schwarz smoother of a hierarchy (oracle.mg.Hierarchy)."""

    def __init__(self, H, block_ptr, block_cells, np_lo):
        self.H, self.np_lo = H, np_lo
        self.block_ptr, self.block_cells = np.asarray(block_ptr), np.asarray(block_cells)

    def apply(self, r):
        H = self.H
        return swz(H.A[0], r, H.cell_ptr[0], self.block_ptr, self.block_cells, H.np[0],
                   self.np_lo)

    def sweeps(self, b, x, n):
        """x <- x + Swz(b - M x), n times."""
        for _ in range(n):
            x = x + self.apply(b - self.H.A[0] @ x)
        return x

    def vcycle(self, r):
        """The V-cycle of oracle.mg.Hierarchy.vcycle with Schwarz smoothing
        on level 0 (nu_pre sweeps from x = 0, nu_post sweeps after the
        coarse correction)."""
        H = self.H
        if H.nlev == 1:
            return H.coarse_solve(r)
        A = H.A[0]
        x = self.sweeps(r, np.zeros_like(r), H.nu_pre)
        rc = H.R[0].T @ (r - A @ x)
        x = x + H.R[0] @ H.vcycle(rc, 1)
        return self.sweeps(r, x, H.nu_post)
