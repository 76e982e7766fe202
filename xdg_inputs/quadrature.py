"""High-order quadrature on hyperrectangles cut by quadric level sets.

The paper integrates on cut cells either by hierarchical moment fitting or by
Saye's method for hyperrectangles (Section 2.1, cut-cell quadrature paragraph).
This module implements the latter idea from its published description
(Saye, SIAM J. Sci. Comput. 37 (2015)): pick a height direction k in which
every level function is monotone, build a rule on the (d-1)-dimensional base
box whose pieces are bounded by the zero sets of the level functions restricted
to the bottom and top faces, and along each base abscissa split [lo_k, hi_k]
at the (at most one per function) roots, placing a Gauss-Legendre rule on every
piece.  Boxes with no admissible height direction are bisected.

Two rules are produced:
  * partition_rule: points/weights covering the whole box, each point tagged
    with the sign of every level function on the piece it belongs to (a volume
    rule for every species at once);
  * surface_rule: points/weights/normals on {phi = 0} inside the box, weights
    carrying the surface measure |grad phi| / |d phi / d x_k|.
"""
import numpy as np

_GL = {}
MAX_DEPTH = 7
# a height direction is accepted only if |d phi/dx_k| stays above this
# fraction of max|grad phi| on the box (keeps the height function smooth)
SLOPE_FRACTION = 0.2


def gauss_legendre(q):
    if q not in _GL:
        x, w = np.polynomial.legendre.leggauss(q)
        _GL[q] = (x, w)
    return _GL[q]


def tensor_rule(lo, hi, q):
    """Tensor Gauss-Legendre rule with q points per direction on a box."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    d = len(lo)
    x, w = gauss_legendre(q)
    grids = [lo[i] + 0.5 * (x + 1.0) * (hi[i] - lo[i]) for i in range(d)]
    wts = [0.5 * w * (hi[i] - lo[i]) for i in range(d)]
    P = np.stack(np.meshgrid(*grids, indexing="ij"), axis=-1).reshape(-1, d)
    W = wts[0]
    for i in range(1, d):
        W = np.multiply.outer(W, wts[i])
    return P, W.reshape(-1)


def _classify(funcs, lo, hi):
    """Split functions into those with a sign change in the box and the
    fixed sign of the others (+1 / -1)."""
    active, fixed = [], np.zeros(len(funcs))
    for i, f in enumerate(funcs):
        m, M = f.bounds(lo, hi)
        if m >= 0.0:
            fixed[i] = 1.0
        elif M <= 0.0:
            fixed[i] = -1.0
        else:
            active.append(i)
    return active, fixed


def _height_direction(fs, lo, hi):
    """Coordinate direction in which every function is strictly monotone
    (with a bounded height-function slope), preferring the largest partial
    derivative of the first function at the box centre."""
    c = 0.5 * (np.asarray(lo) + np.asarray(hi))
    g = np.abs(fs[0].grad(c))
    for k in np.argsort(-g, kind="stable"):
        ok = True
        for f in fs:
            m, M = f.dbounds(k, lo, hi)
            if m <= 0.0 <= M:
                ok = False
                break
            if min(abs(m), abs(M)) < SLOPE_FRACTION * f.grad_norm_max(lo, hi):
                ok = False
                break
        if ok:
            return int(k)
    return None


def _subboxes(lo, hi):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    mid = 0.5 * (lo + hi)
    d = len(lo)
    for code in range(1 << d):
        sl, sh = lo.copy(), hi.copy()
        for i in range(d):
            if code >> i & 1:
                sl[i] = mid[i]
            else:
                sh[i] = mid[i]
        yield sl, sh


def _insert(Xb, k, z):
    """Insert coordinate column z at position k of base points Xb."""
    return np.concatenate([Xb[:, :k], z[:, None], Xb[:, k:]], axis=1)


def partition_rule(funcs, lo, hi, q, depth=0):
    """Rule over the whole box; returns (P [N,d], W [N], S [N,nf]) where
    S[:, i] is the sign of funcs[i] on the piece each point lies in."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    d = len(lo)
    nf = len(funcs)
    active, fixed = _classify(funcs, lo, hi)
    if not active:
        P, W = tensor_rule(lo, hi, q)
        return P, W, np.tile(fixed, (len(W), 1))

    if d == 1:
        brk = sorted(set(r for i in active for r in funcs[i].roots_1d(lo[0], hi[0])))
        edges = [lo[0]] + brk + [hi[0]]
        x, w = gauss_legendre(q)
        Ps, Ws, Ss = [], [], []
        for a, b in zip(edges[:-1], edges[1:]):
            if b <= a:
                continue
            mid = np.array([[0.5 * (a + b)]])
            sg = fixed.copy()
            for i in active:
                sg[i] = 1.0 if funcs[i](mid)[0] > 0.0 else -1.0
            Ps.append(a + 0.5 * (x + 1.0) * (b - a))
            Ws.append(0.5 * w * (b - a))
            Ss.append(np.tile(sg, (q, 1)))
        return (np.concatenate(Ps)[:, None], np.concatenate(Ws),
                np.concatenate(Ss, axis=0))

    fs = [funcs[i] for i in active]
    k = _height_direction(fs, lo, hi)
    if k is None:
        if depth >= MAX_DEPTH:
            # last resort on a tiny box: tensor rule with pointwise signs
            P, W = tensor_rule(lo, hi, q)
            S = np.tile(fixed, (len(W), 1))
            for i in active:
                S[:, i] = np.where(funcs[i](P) > 0.0, 1.0, -1.0)
            return P, W, S
        parts = [partition_rule(funcs, sl, sh, q, depth + 1) for sl, sh in _subboxes(lo, hi)]
        return (np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]),
                np.concatenate([p[2] for p in parts], axis=0))

    base = []
    for f in fs:
        base.append(f.restrict(k, lo[k]))
        base.append(f.restrict(k, hi[k]))
    blo = np.delete(lo, k)
    bhi = np.delete(hi, k)
    Pb, Wb, _ = partition_rule(base, blo, bhi, q, depth)
    nb = len(Wb)
    na = len(fs)
    R = np.full((nb, na), np.nan)
    for j, f in enumerate(fs):
        flo = f(_insert(Pb, k, np.full(nb, lo[k])))
        fhi = f(_insert(Pb, k, np.full(nb, hi[k])))
        has = flo * fhi < 0.0
        if np.any(has):
            R[has, j] = f.root_along(Pb[has], k, lo[k], hi[k])
    R = np.sort(R, axis=1)
    R = np.where(np.isnan(R), hi[k], R)
    bp = np.concatenate([np.full((nb, 1), lo[k]), R, np.full((nb, 1), hi[k])], axis=1)
    a = bp[:, :-1]
    L = bp[:, 1:] - a                       # [nb, na+1]
    x, w = gauss_legendre(q)
    Z = a[:, :, None] + 0.5 * (x + 1.0)[None, None, :] * L[:, :, None]   # [nb, na+1, q]
    WZ = (0.5 * w)[None, None, :] * L[:, :, None] * Wb[:, None, None]
    mid = a + 0.5 * L                       # [nb, na+1]
    nseg = na + 1
    Pmid = _insert(np.repeat(Pb, nseg, axis=0), k, mid.reshape(-1))
    S = np.tile(fixed, (nb * nseg, 1))
    for i in active:
        S[:, i] = np.where(funcs[i](Pmid) > 0.0, 1.0, -1.0)
    keep = (L.reshape(-1) > 0.0)
    # expand to points
    Pfull = _insert(np.repeat(Pb, nseg * q, axis=0), k, Z.reshape(-1))
    Wfull = WZ.reshape(-1)
    Sfull = np.repeat(S, q, axis=0)
    kp = np.repeat(keep, q)
    return Pfull[kp], Wfull[kp], Sfull[kp]


def surface_rule(f, lo, hi, q, depth=0):
    """Rule on {f = 0} inside the box: (P [N,d], W [N], normals [N,d]);
    normals are grad f / |grad f| (pointing from {f<0} to {f>0})."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    d = len(lo)
    m, M = f.bounds(lo, hi)
    if m >= 0.0 or M <= 0.0:
        return np.zeros((0, d)), np.zeros(0), np.zeros((0, d))
    k = _height_direction([f], lo, hi)
    if k is None:
        if depth >= MAX_DEPTH:
            return np.zeros((0, d)), np.zeros(0), np.zeros((0, d))
        parts = [surface_rule(f, sl, sh, q, depth + 1) for sl, sh in _subboxes(lo, hi)]
        return (np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]),
                np.concatenate([p[2] for p in parts]))
    if d == 1:
        raise ValueError("surface rules are needed in 2D and 3D only")
    base = [f.restrict(k, lo[k]), f.restrict(k, hi[k])]
    Pb, Wb, _ = partition_rule(base, np.delete(lo, k), np.delete(hi, k), q, depth)
    nb = len(Wb)
    flo = f(_insert(Pb, k, np.full(nb, lo[k])))
    fhi = f(_insert(Pb, k, np.full(nb, hi[k])))
    has = flo * fhi < 0.0
    Pb, Wb = Pb[has], Wb[has]
    z = f.root_along(Pb, k, lo[k], hi[k])
    P = _insert(Pb, k, z)
    G = f.grad(P)
    gn = np.linalg.norm(G, axis=1)
    W = Wb * gn / np.abs(G[:, k])
    return P, W, G / gn[:, None]
