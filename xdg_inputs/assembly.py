"""Symmetric interior penalty (SIP) assembly on an aggregated cut-cell level.

Bilinear form (Section 2.2, Eq. DefSIP):
    a(u, v) = sum_parts int mu grad u . grad v
            - oint_{I u Gamma} ({mu grad u}.n [v] + {mu grad v}.n [u])
            + oint_{I u Gamma} eta max(mu_in, mu_out) [u][v]
with the jump [u] = u_in - u_out on interior faces and the interface, u_in on
the domain boundary, and the mean {w} = (w_in + w_out)/2 (u_in on the
boundary) (Section 2.1, Eqs. defJumpOperator / defMeanOperator).  "in" is the
side the normal points away from: on a background face the lower cell (normal
+e_d), on the interface species A (normal from A to B, Section 1.1).
Right-hand side (Eq. SIPrhs), Dirichlet data on the whole boundary:
    b(v) = int f v - oint_{dOmega} mu g_D (grad v . n - eta v).
Matrix convention (Eq. GenericMatrixSystem): M[m(i, a), m(l, b)] =
a(phi_{l,b}, phi_{i,a}) -- block row = test part, block column = trial part.

Faces between two pieces of the same aggregate carry no jump and are skipped;
that is what makes the system the one on the agglomerated space
(Eq. GenericVarSchemeAgglommSpace).

Penalty (Section 2.2 asks for eta ~ const k^2 / h' with h' a length scale of
the agglomerated cut cell):  eta = C_eta (p+1)(p+D)/D * max over the adjacent
aggregates of |dP| / |P|  (|dP| includes interface and faces to other parts).
"""
import numpy as np

from .basis import BoxBasis, PartBasis
from .quadrature import tensor_rule

C_ETA_DEFAULT = 1.0


class Penalty:
    def __init__(self, face, iface):
        self.face = face      # list over d of [n+1, n^(D-1), 2]
        self.iface = iface    # [ncells]


def _face_arrays(geom, d):
    n, D = geom.n, geom.D
    nt = n ** (D - 1)
    planes = np.repeat(np.arange(n + 1), nt)
    ts = np.tile(np.arange(nt), n + 1)
    below, above = geom.face_cells(d, planes, ts)
    return planes, ts, below, above


def _rows_of(level, cells, s):
    return np.where(cells >= 0, level.part_of[2 * np.maximum(cells, 0) + s], -1)


def compute_penalty(geom, level, c_eta=C_ETA_DEFAULT):
    """Penalty factors from the aggregates of `level` (level 0)."""
    D, h = geom.D, geom.h
    nrow = level.n_rows
    row_of_piece = np.repeat(np.arange(nrow), np.diff(level.piece_ptr))
    volP = np.zeros(nrow)
    np.add.at(volP, row_of_piece, geom.vol[level.piece_cell, level.species[row_of_piece]])
    bnd = np.zeros(nrow)
    for d in range(D):
        planes, ts, below, above = _face_arrays(geom, d)
        for s in range(2):
            area = geom.farea[d][:, :, s].reshape(-1)
            rb = _rows_of(level, below, s)
            ra = _rows_of(level, above, s)
            diff = (area > 0.0) & (rb != ra)
            m = diff & (rb >= 0)
            np.add.at(bnd, rb[m], area[m])
            m = diff & (ra >= 0)
            np.add.at(bnd, ra[m], area[m])
    for j in geom.cut:
        a = geom.interface_area(j)
        bnd[level.part_of[2 * j]] += a
        bnd[level.part_of[2 * j + 1]] += a
    ratio = bnd / volP
    ratio[level.standard] = 2.0 * D / h
    p = level.deg
    base = c_eta * (p + 1) * (p + D) / D
    face = []
    for d in range(D):
        planes, ts, below, above = _face_arrays(geom, d)
        eta = np.zeros(geom.farea[d].shape)
        for s in range(2):
            rb = _rows_of(level, below, s)
            ra = _rows_of(level, above, s)
            rr = np.maximum(np.where(rb >= 0, ratio[np.maximum(rb, 0)], 0.0),
                            np.where(ra >= 0, ratio[np.maximum(ra, 0)], 0.0))
            eta[:, :, s] = (base * rr).reshape(eta.shape[:2])
        face.append(eta)
    iface = np.zeros(geom.ncells)
    for j in geom.cut:
        iface[j] = base * max(ratio[level.part_of[2 * j]], ratio[level.part_of[2 * j + 1]])
    pen = Penalty(face, iface)
    pen.eta_standard = base * 2.0 * D / h
    pen.ratio = ratio
    return pen


def _stiff(W, g):
    """sum_q W_q grad phi_a . grad phi_b  for g [N, Np, D]."""
    out = 0.0
    for d in range(g.shape[2]):
        gd = g[:, :, d]
        out = out + (gd * W[:, None]).T @ gd
    return out


def _normal_deriv(g, nrm):
    return (g * np.broadcast_to(nrm, (g.shape[0], g.shape[2]))[:, None, :]).sum(axis=2)


def face_blocks(P, W, nrm, b_in, b_out, mu_in, mu_out, eta):
    """SIP face/interface blocks {(X, Y): M[X, Y]} for X, Y in {in, out};
    b_out None means a Dirichlet boundary face.  nrm is [D] or [N, D]."""
    v_i, g_i = b_in.eval(P)
    dn_i = _normal_deriv(g_i, nrm)
    Wv = W[:, None]
    if b_out is None:
        # [u] = u_in, {mu grad u} = mu grad u_in
        A = -mu_in * (Wv * v_i).T @ dn_i
        return {("in", "in"): A + A.T + eta * mu_in * (Wv * v_i).T @ v_i}
    v_o, g_o = b_out.eval(P)
    dn_o = _normal_deriv(g_o, nrm)
    vals = {"in": v_i, "out": v_o}
    dns = {"in": dn_i, "out": dn_o}
    mus = {"in": mu_in, "out": mu_out}
    sg = {"in": 1.0, "out": -1.0}
    mmax = max(mu_in, mu_out)
    out = {}
    for X in ("in", "out"):
        for Y in ("in", "out"):
            t1 = -0.5 * mus[Y] * sg[X] * (Wv * vals[X]).T @ dns[Y]
            t2 = -0.5 * mus[X] * sg[Y] * (Wv * dns[X]).T @ vals[Y]
            t3 = eta * mmax * sg[X] * sg[Y] * (Wv * vals[X]).T @ vals[Y]
            out[(X, Y)] = t1 + t2 + t3
    return out


class _Batches:
    def __init__(self, nrow, Np):
        self.nrow, self.Np = nrow, Np
        self.keys, self.items = [], []

    def template(self, rows, cols, T):
        if len(rows):
            self.keys.append(np.asarray(rows, np.int64) * self.nrow + np.asarray(cols, np.int64))
            self.items.append(("t", T))

    def blocks(self, rows, cols, B):
        if len(rows):
            self.keys.append(np.asarray(rows, np.int64) * self.nrow + np.asarray(cols, np.int64))
            self.items.append(("b", np.asarray(B)))

    def to_bsr(self):
        keys = np.concatenate(self.keys)
        uniq, inv = np.unique(keys, return_inverse=True)
        val = np.zeros((len(uniq), self.Np, self.Np))
        off = 0
        for k, (kind, item) in zip(self.keys, self.items):
            idx = inv[off:off + len(k)]
            off += len(k)
            if kind == "t":
                val[idx] += item          # unique within a template batch
            else:
                np.add.at(val, idx, item)
        rows = uniq // self.nrow
        cols = uniq % self.nrow
        row_ptr = np.zeros(self.nrow + 1, dtype=np.int64)
        np.add.at(row_ptr, rows + 1, 1)
        return np.cumsum(row_ptr), cols.astype(np.int64), val


def assemble(geom, level, mu, pen, q_std):
    """Level matrix as BSR (row_ptr, col_idx, val[nnzb, Np, Np])."""
    D, h = geom.D, geom.h
    Np, nrow = level.np, level.n_rows
    std = level.standard
    bt = _Batches(nrow, Np)
    # reference cell and its (unscaled-family) stiffness
    ref = BoxBasis(np.full(D, -0.5 * h), np.full(D, 0.5 * h), level.deg)
    P, W = tensor_rule(ref.lo, ref.hi, q_std)
    _, g = ref.eval(P)
    Kref = _stiff(W, g)
    single_cell = std & (np.diff(level.piece_ptr) == 1)
    for s in range(2):
        rows = np.flatnonzero(single_cell & (level.species == s))
        bt.template(rows, rows, mu[s] * Kref)
    for r in np.flatnonzero(~single_cell):
        s = int(level.species[r])
        acc = np.zeros((Np, Np))
        for j in level.pieces(r):
            Pq, Wq = geom.volume_rule(j, s, q_std)
            _, gq = level.bases[r].eval(Pq)
            acc += mu[s] * _stiff(Wq, gq)
        bt.blocks([r], [r], acc[None])

    # background faces
    for d in range(D):
        e = np.zeros(D)
        e[d] = 1.0
        planes, ts, below, above = _face_arrays(geom, d)
        nt = geom.n ** (D - 1)
        cutmask = np.zeros(len(planes), dtype=bool)
        for (dd, pl, t) in geom.fcut:
            if dd == d:
                cutmask[pl * nt + t] = True
        lo_c = np.full(D, -0.5 * h)
        hi_c = np.full(D, 0.5 * h)
        for s in range(2):
            area = geom.farea[d][:, :, s].reshape(-1)
            eta = pen.face[d][:, :, s].reshape(-1)
            rb = _rows_of(level, below, s)
            ra = _rows_of(level, above, s)
            has = area > 0.0
            inter = has & (rb >= 0) & (ra >= 0) & (rb != ra)
            bnd_lo = has & (rb < 0) & (ra >= 0)
            bnd_hi = has & (ra < 0) & (rb >= 0)
            sc_b = np.where(rb >= 0, single_cell[np.maximum(rb, 0)], False)
            sc_a = np.where(ra >= 0, single_cell[np.maximum(ra, 0)], False)
            etaok = eta == getattr(pen, "eta_standard", np.nan)
            # -- interior template
            tm = inter & sc_b & sc_a & ~cutmask & etaok
            if np.any(tm):
                bl = BoxBasis(lo_c - 0.5 * h * e, hi_c - 0.5 * h * e, level.deg)
                ab = BoxBasis(lo_c + 0.5 * h * e, hi_c + 0.5 * h * e, level.deg)
                Pf, Wf = tensor_rule(np.delete(lo_c, d), np.delete(hi_c, d), q_std)
                Pf = np.insert(Pf, d, 0.0, axis=1)
                Tb = face_blocks(Pf, Wf, e, PartBasis(bl), PartBasis(ab), mu[s], mu[s],
                                 pen.eta_standard)
                R_b, R_a = rb[tm], ra[tm]
                bt.template(R_b, R_b, Tb[("in", "in")])
                bt.template(R_b, R_a, Tb[("in", "out")])
                bt.template(R_a, R_b, Tb[("out", "in")])
                bt.template(R_a, R_a, Tb[("out", "out")])
            for f in np.flatnonzero(inter & ~tm):
                Pq, Wq = geom.face_rule(d, planes[f], ts[f], s, q_std)
                i, l = int(rb[f]), int(ra[f])
                B = face_blocks(Pq, Wq, e, level.bases[i], level.bases[l], mu[s], mu[s], eta[f])
                bt.blocks([i, i, l, l], [i, l, i, l],
                          [B[("in", "in")], B[("in", "out")], B[("out", "in")], B[("out", "out")]])
            # -- boundary faces (outward normal -e on plane 0, +e on plane n)
            for mask, rows, sign in ((bnd_lo, ra, -1.0), (bnd_hi, rb, 1.0)):
                tmb = mask & np.where(rows >= 0, single_cell[np.maximum(rows, 0)], False) \
                    & ~cutmask & etaok
                if np.any(tmb):
                    ref_c = BoxBasis(lo_c, hi_c, level.deg)
                    Pf, Wf = tensor_rule(np.delete(lo_c, d), np.delete(hi_c, d), q_std)
                    Pf = np.insert(Pf, d, sign * 0.5 * h, axis=1)
                    Tb = face_blocks(Pf, Wf, sign * e, PartBasis(ref_c), None, mu[s], None,
                                     pen.eta_standard)
                    rr = rows[tmb]
                    bt.template(rr, rr, Tb[("in", "in")])
                for f in np.flatnonzero(mask & ~tmb):
                    Pq, Wq = geom.face_rule(d, planes[f], ts[f], s, q_std)
                    i = int(rows[f])
                    B = face_blocks(Pq, Wq, sign * e, level.bases[i], None, mu[s], None, eta[f])
                    bt.blocks([i], [i], [B[("in", "in")]])

    # interface: in = A, out = B, normal from A to B
    for j in sorted(geom.cut):
        rA, rB = int(level.part_of[2 * j]), int(level.part_of[2 * j + 1])
        Pq, Wq, Nq = geom.interface_rule(j)
        if len(Wq) == 0:
            continue
        B = face_blocks(Pq, Wq, Nq, level.bases[rA], level.bases[rB], mu[0], mu[1],
                        pen.iface[j])
        bt.blocks([rA, rA, rB, rB], [rA, rB, rA, rB],
                  [B[("in", "in")], B[("in", "out")], B[("out", "in")], B[("out", "out")]])
    return bt.to_bsr()


def load_vector(geom, level, mu, pen, q_std, f=None, g_dir=None):
    """b(phi_{i,a}) for source f(X, s) and Dirichlet data g_dir(X, s) (Eq. SIPrhs)."""
    D = geom.D
    b = np.zeros((level.n_rows, level.np))
    if f is not None:
        for r in range(level.n_rows):
            s = int(level.species[r])
            for j in level.pieces(r):
                Pq, Wq = geom.volume_rule(j, s, q_std)
                if len(Wq) == 0:
                    continue
                v = level.bases[r].eval(Pq, grad=False)
                b[r] += (Wq * f(Pq, s)) @ v
    if g_dir is not None:
        for d in range(D):
            e = np.zeros(D)
            e[d] = 1.0
            planes, ts, below, above = _face_arrays(geom, d)
            for s in range(2):
                area = geom.farea[d][:, :, s].reshape(-1)
                eta = pen.face[d][:, :, s].reshape(-1)
                for f_, rows_cells, sign in (((planes == 0), above, -1.0),
                                             ((planes == geom.n), below, 1.0)):
                    for fi in np.flatnonzero(f_ & (area > 0.0)):
                        r = int(level.part_of[2 * rows_cells[fi] + s])
                        Pq, Wq = geom.face_rule(d, planes[fi], ts[fi], s, q_std)
                        v, gv = level.bases[r].eval(Pq)
                        dn = gv @ (sign * e)
                        gd = g_dir(Pq, s)
                        b[r] += -mu[s] * ((Wq * gd) @ dn) + eta[fi] * mu[s] * ((Wq * gd) @ v)
    return b.reshape(-1)


def l2_error(geom, level, x, u_exact, q_std):
    """|| u_h - u ||_{L2(Omega)} for the coefficient vector x on `level`."""
    X = x.reshape(level.n_rows, level.np)
    err2 = 0.0
    for r in range(level.n_rows):
        s = int(level.species[r])
        for j in level.pieces(r):
            Pq, Wq = geom.volume_rule(j, s, q_std)
            if len(Wq) == 0:
                continue
            uh = level.bases[r].eval(Pq, grad=False) @ X[r]
            err2 += float(Wq @ (uh - u_exact(Pq, s)) ** 2)
    return np.sqrt(err2)
