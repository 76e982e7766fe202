"""Agglomeration maps, aggregation levels and their bases.

* Small-cut-cell agglomeration A_alpha (Section 2.3): every present cut part
  K_{j,s} with volume fraction <= alpha is joined to the face neighbour l of the
  same species with the largest |K_{l,s}| (ties to the smaller index); a
  neighbour counts only if the two parts share a face portion of species s
  (a logical edge of the cut-cell mesh graph).  Aggregates are the connected
  components of the edge set (Def. Aggregation maps).
* Multigrid aggregation sequence (Section 3.1, Eq. MultigridAggMeshSeq): level
  m joins the cells of every 2^m-per-direction block of the background mesh.
  It is mapped onto the cut-cell mesh by duplicating every edge per species
  when both parts have positive volume (Def. Mapping of an aggregation map) and
  united with A_alpha.
* Index convention (Section 3.2): an aggregate's representative is the
  minimum background cell index it contains.  Rows are ordered by (level-m
  block of the representative, species A before B, representative); the
  smoother's cell blocks group the rows whose representatives lie in the same
  level-m block (the block m(j,-,-,.) over all species of a cell).
* Bases (Section 3.2): Legendre family on each aggregate's bounding box,
  orthonormalised on the aggregate by Cholesky; a full non-agglomerated
  background cell keeps the unscaled family (S = I).
"""
import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

from .basis import BoxBasis, PartBasis, n_modes, orthonormalize


def alpha_edges(geom, alpha, force=None):
    """Edges (part_u, part_v), part = 2*j + s, of the agglomeration map.
    force: parts (j, s) that must be agglomerated whatever their volume
    fraction (cut parts that are new at this time level, Section 2.3)."""
    edges = []
    force = force or set()
    for j in sorted(geom.cut):
        for s in range(2):
            if not geom.present[j, s] or (geom.frac[j, s] > alpha and (j, s) not in force):
                continue
            best, best_vol = -1, -1.0
            for d, plane, t, sg in geom.cell_faces(j):
                if geom.farea[d][plane, t, s] <= 0.0:
                    continue
                below, above = geom.face_cells(d, plane, t)
                l = int(above if sg > 0 else below)
                if l < 0 or not geom.present[l, s]:
                    continue
                v = geom.vol[l, s]
                if v > best_vol or (v == best_vol and l < best):
                    best, best_vol = l, v
            if best >= 0:
                edges.append((2 * j + s, 2 * best + s))
    return edges


def blocking_edges(geom, m):
    """Level-m aggregation edges of the background mesh mapped per species."""
    if m == 0:
        return []
    n, D = geom.n, geom.D
    nt = n ** (D - 1)
    out = []
    for d in range(D):
        planes = np.repeat(np.arange(1, n), nt)
        ts = np.tile(np.arange(nt), n - 1)
        inside = (planes % (1 << m)) != 0
        below, above = geom.face_cells(d, planes[inside], ts[inside])
        for s in range(2):
            ok = geom.present[below, s] & geom.present[above, s]
            out.append(np.stack([2 * below[ok] + s, 2 * above[ok] + s], axis=1))
    return [tuple(e) for e in np.concatenate(out, axis=0).tolist()] if out else []


class Level:
    """One aggregation/p level: rows (aggregate, species), pieces, bases."""

    def __init__(self, geom, m, deg, part_labels):
        self.geom, self.m, self.deg = geom, m, deg
        D = geom.D
        self.np = n_modes(D, deg)
        present_parts = np.flatnonzero(geom.present.reshape(-1))
        lab = part_labels[present_parts]
        uniq, inv = np.unique(lab, return_inverse=True)
        nrow = len(uniq)
        cells = present_parts // 2
        spec = present_parts % 2
        rep = np.full(nrow, np.iinfo(np.int64).max)
        np.minimum.at(rep, inv, cells)
        rspec = np.zeros(nrow, dtype=np.int64)
        rspec[inv] = spec
        I = geom.cell_multi(rep)
        nb = geom.n >> m
        block = sum((I[:, d] >> m) * nb ** d for d in range(D))
        order = np.lexsort((rep, rspec, block))
        rank = np.empty(nrow, dtype=np.int64)
        rank[order] = np.arange(nrow)
        self.n_rows = nrow
        self.rep = rep[order]
        self.species = rspec[order]
        self.block = block[order]
        row_of_piece = rank[inv]
        self.part_of = np.full(2 * geom.ncells, -1, dtype=np.int64)
        self.part_of[present_parts] = row_of_piece
        o = np.argsort(row_of_piece, kind="stable")
        self.piece_cell = cells[o]
        self.piece_ptr = np.zeros(nrow + 1, dtype=np.int64)
        np.add.at(self.piece_ptr, row_of_piece + 1, 1)
        self.piece_ptr = np.cumsum(self.piece_ptr)
        chg = np.flatnonzero(np.diff(self.block)) + 1
        self.cell_ptr = np.concatenate([[0], chg, [nrow]]).astype(np.int64)
        self.bases = None

    def pieces(self, r):
        return self.piece_cell[self.piece_ptr[r]:self.piece_ptr[r + 1]]

    def is_standard(self):
        """Rows whose aggregate is a full axis-aligned box of uncut cells: the
        Legendre family on that box is already orthonormal (S = I exactly).
        On level 0 these are the non-agglomerated uncut cells."""
        geom = self.geom
        std = np.zeros(self.n_rows, dtype=bool)
        full = geom.state[self.piece_cell] != 2
        allfull = np.logical_and.reduceat(full, self.piece_ptr[:-1])
        cnt = np.diff(self.piece_ptr)
        std[allfull & (cnt == 1)] = True
        for r in np.flatnonzero(allfull & (cnt > 1)):
            I = geom.cell_multi(self.pieces(r))
            ext = I.max(axis=0) - I.min(axis=0) + 1
            std[r] = int(np.prod(ext)) == int(cnt[r])
        return std

    def build_bases(self, q_std):
        geom = self.geom
        std = self.is_standard()
        self.standard = std
        self.bases = [None] * self.n_rows
        for r in range(self.n_rows):
            cells = self.pieces(r)
            I = geom.cell_multi(cells)
            lo = -1.0 + geom.h * I.min(axis=0)
            hi = -1.0 + geom.h * (I.max(axis=0) + 1)
            box = BoxBasis(lo, hi, self.deg)
            if std[r]:
                self.bases[r] = PartBasis(box, None)
                continue
            G = np.zeros((self.np, self.np))
            s = int(self.species[r])
            for j in cells:
                P, W = geom.volume_rule(j, s, q_std)
                psi = box.eval(P, grad=False)
                G += (psi * W[:, None]).T @ psi
            self.bases[r] = PartBasis(box, orthonormalize(G))

    def truncate_from(self, fine):
        """Same partition as `fine`, leading modes of its bases (p-level)."""
        self.standard = fine.standard
        nlo = self.np
        self.bases = []
        for b in fine.bases:
            box = BoxBasis(b.box.lo, b.box.hi, self.deg)
            self.bases.append(PartBasis(box, None if b.C is None else b.C[:nlo, :nlo].copy()))


def level_labels(geom, a_edges, m):
    edges = list(a_edges) + blocking_edges(geom, m)
    N = 2 * geom.ncells
    if edges:
        E = np.array(edges, dtype=np.int64)
        A = coo_matrix((np.ones(len(E)), (E[:, 0], E[:, 1])), shape=(N, N))
    else:
        A = coo_matrix((N, N))
    _, labels = connected_components(A, directed=False)
    return labels


def dense_transfer(fine, coarse, q_std):
    """parent[i] and R_i[nf, nc] = int_{P_i} phi_{i,nf} phi_{c(i),nc}
    (projection of the coarse basis onto each fine part, Section 3.2)."""
    geom = fine.geom
    first_piece = fine.piece_cell[fine.piece_ptr[:-1]]
    parent = coarse.part_of[2 * first_piece + fine.species]
    R = np.zeros((fine.n_rows, fine.np, coarse.np))
    cache = {}
    for i in range(fine.n_rows):
        c = int(parent[i])
        s = int(fine.species[i])
        fb, cb = fine.bases[i], coarse.bases[c]
        tkey = None
        if fine.standard[i] and coarse.standard[c]:
            # translation-invariant case: key on the child offset in the block
            off = np.round((fb.box.lo - cb.box.lo) / geom.h).astype(int)
            ext = np.round((fb.box.hi - fb.box.lo) / geom.h).astype(int)
            tkey = tuple(off) + tuple(ext) + (s,)
            if tkey in cache:
                R[i] = cache[tkey]
                continue
        acc = np.zeros((fine.np, coarse.np))
        for j in fine.pieces(i):
            P, W = geom.volume_rule(j, s, q_std)
            pf = fb.eval(P, grad=False)
            pc = cb.eval(P, grad=False)
            acc += (pf * W[:, None]).T @ pc
        R[i] = acc
        if tkey is not None:
            cache[tkey] = acc
    return parent.astype(np.int64), R
