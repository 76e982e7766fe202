"""FP64 oracle of the learned per-cell smoother -- test infrastructure only
(imported by tests, the smoke check and the CPU baseline, never by the
product path).

The learned smoother is a project extension beyond the paper: it replaces the
first damped block-Jacobi sweep of the level-0 smoother (Section 3.3, the
cell-block Jacobi method with pre-inverted diagonal blocks) inside the
V-cycle.  With x_in = 0 and residual r, per smoother cell c (rows
[cell_ptr[c], cell_ptr[c+1]), np = 20 modes per row):
    j_c = omega D_c^{-1} r_c,  s_c = ||j_c||_2,
    features f_c = [ j_c / s_c placed in species slots | geom_c (5) ]
      (species-A row -> slots 0..19, species-B row -> 20..39, zeros else),
    y_c = MLP(f_c) (oracle.mlp.forward),
    x_c = j_c + s_c * y_c[slots of the cell's rows],
unless y_c is non-finite or ||y_c||_2 > guard, then x_c = j_c.
Training pairs from an iterate x_k of a plain solve (residual r_k = b - M x_k)
and the converged x*: features of r_k, target (x* - x_k - j_c) / s_c in the
same slots, optionally scaled down to a maximum norm (the error of a smooth
mode is many Jacobi steps long and no cell-local map can predict it; the
clipped target keeps the network's proposal in the range of a sweep).
"""
import numpy as np

from . import mlp

NP = 20


def _slots(cell_ptr, row_species):
    """For every level-0 row: (cell, first slot).  Slot block of a row =
    20 * species."""
    cp = np.asarray(cell_ptr)
    cell_of_row = np.repeat(np.arange(len(cp) - 1), np.diff(cp))
    return cell_of_row, NP * np.asarray(row_species, dtype=np.int64)


def features(H, row_species, cell_geom, r):
    """(F [n_cells, 45], j [level-0 vector], s [n_cells]) for residual r."""
    cp = H.cell_ptr[0]
    n_cells = len(cp) - 1
    j = H.omega * (H.Dinv[0] @ r)
    cell_of_row, slot0 = _slots(cp, row_species)
    jr = j.reshape(-1, NP)
    s = np.sqrt(np.bincount(cell_of_row, weights=np.sum(jr * jr, axis=1), minlength=n_cells))
    inv = np.where(s > 0.0, 1.0 / np.where(s > 0.0, s, 1.0), 0.0)
    F = np.zeros((n_cells, mlp.N_IN))
    for row in range(jr.shape[0]):
        c = cell_of_row[row]
        F[c, slot0[row]:slot0[row] + NP] = jr[row] * inv[c]
    F[:, 2 * NP:] = cell_geom
    return F, j, s


def first_sweep(H, row_species, cell_geom, theta, r, guard, bf16=False):
    """x after the learned first sweep from x = 0; also the number of cells
    that kept the plain Jacobi step.  bf16: the network runs with bfloat16
    operands (mlp.forward_bf16)."""
    F, j, s = features(H, row_species, cell_geom, r)
    Y = mlp.forward_bf16(theta, F) if bf16 else mlp.forward(theta, F)[0]
    bad = ~np.all(np.isfinite(Y), axis=1) | ~(np.linalg.norm(Y, axis=1) <= guard)
    Y[bad] = 0.0
    cp = H.cell_ptr[0]
    cell_of_row, slot0 = _slots(cp, row_species)
    x = j.reshape(-1, NP).copy()
    for row in range(x.shape[0]):
        c = cell_of_row[row]
        x[row] += s[c] * Y[c, slot0[row]:slot0[row] + NP]
    return x.reshape(-1), int(bad.sum())


def pairs(H, row_species, cell_geom, b, xk, xs, clip=0.0):
    """(X [n_cells, 45], T [n_cells, 40]) training pairs of iterate xk; with
    clip > 0 every target longer than clip is scaled to length clip."""
    r = b - H.A[0] @ xk
    F, j, s = features(H, row_species, cell_geom, r)
    cp = H.cell_ptr[0]
    cell_of_row, slot0 = _slots(cp, row_species)
    inv = np.where(s > 0.0, 1.0 / np.where(s > 0.0, s, 1.0), 0.0)
    E = (xs - xk - j).reshape(-1, NP)
    T = np.zeros((len(cp) - 1, mlp.N_OUT))
    for row in range(E.shape[0]):
        c = cell_of_row[row]
        T[c, slot0[row]:slot0[row] + NP] = E[row] * inv[c]
    if clip > 0.0:
        nt = np.linalg.norm(T, axis=1)
        big = nt > clip
        T[big] *= (clip / nt[big])[:, None]
    return F, T


def vcycle(H, row_species, cell_geom, theta, r, guard, level=0, bf16=False):
    """The V-cycle of oracle.mg.Hierarchy.vcycle with the learned first sweep
    on level 0 (the remaining nu_pre - 1 sweeps and the post-smoothing are
    plain damped block Jacobi)."""
    if level > 0:
        return H.vcycle(r, level)
    from .mg import jacobi
    A, D = H.A[0], H.Dinv[0]
    x, _ = first_sweep(H, row_species, cell_geom, theta, r, guard, bf16)
    x = jacobi(A, D, r, x, H.omega, H.nu_pre - 1)
    rc = H.R[0].T @ (r - A @ x)
    x = x + H.R[0] @ H.vcycle(rc, 1)
    return jacobi(A, D, r, x, H.omega, H.nu_post)
