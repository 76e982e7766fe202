"""Per-cell geometric descriptors of a generated problem for the learned
smoother's input: which species each level-0 block row carries, and per
smoother cell the volume fraction of species A, the mean unit interface
normal and the log10 diffusivity ratio.  Pure geometry bookkeeping; nothing
here applies an operator or solves."""
import numpy as np


def cell_features(pr):
    """(row_species int32 [n_rows], cell_geom float32 [n_cells, 5]) of the
    level-0 rows and smoother cells of problem `pr`.

    cell_geom[c] = [f_A, n_x, n_y, n_z, log10(mu_B / mu_A)]:
      f_A   = |A part| / (|A part| + |B part|) over the pieces of the cell's rows,
      n     = quadrature-weighted mean of the interface normals (pointing from
              A to B) over the cut pieces, normalised; zero if no piece is cut,
      last  = log10 of the diffusivity ratio if the cell carries both species,
              else zero.
    """
    L0, geom = pr.levels[0], pr.geom
    cp = np.asarray(pr.cell_ptr)
    n_cells = len(cp) - 1
    out = np.zeros((n_cells, 5))
    ratio = np.log10(pr.mu[1] / pr.mu[0])
    for c in range(n_cells):
        vol = np.zeros(2)
        nrm = np.zeros(geom.D)
        seen = set()
        for r in range(cp[c], cp[c + 1]):
            s = int(L0.species[r])
            for q in L0.pieces(r):
                vol[s] += geom.vol[q, s]
                if q in seen:
                    continue
                seen.add(q)
                iface = geom.interface_rule(q)
                if iface is not None:
                    _, W, N = iface
                    nrm += W @ N
        out[c, 0] = vol[0] / vol.sum()
        nn = np.linalg.norm(nrm)
        if nn > 0.0:
            out[c, 1:1 + geom.D] = nrm / nn
        if cp[c + 1] - cp[c] == 2:
            out[c, 4] = ratio
    return L0.species.astype(np.int32), out.astype(np.float32)
