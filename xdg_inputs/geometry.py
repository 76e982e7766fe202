"""Cartesian background mesh, cut-cell classification and cut-cell rules.

Background mesh: n^D equal cells on [-1, 1]^D, cell j = i_0 + n i_1 + n^2 i_2
(first coordinate fastest).  Cut cells K_{j,s} = K_j intersected with species s
(Section 2.1, Def. Cut-cell mesh).  A species is present in a cell when its
volume fraction exceeds PRESENT_TOL (parts below that are treated as absent).

Faces are addressed as (d, plane, t): the face normal to direction d on
coordinate plane x_d = -1 + plane*h, t the index of the adjacent cells'
transverse position (remaining coordinates in increasing order, first fastest).
The cell below a face has i_d = plane - 1, the cell above i_d = plane.
"""
import numpy as np

from .quadrature import partition_rule, surface_rule, tensor_rule

PRESENT_TOL = 1e-14
SPECIES_A, SPECIES_B = 0, 1


class CutCellData:
    __slots__ = ("vol_rules", "iface")

    def __init__(self, vol_rules, iface):
        self.vol_rules = vol_rules      # [(P, W) for species A, B]
        self.iface = iface              # (P, W, normals A->B) or None


class Geometry:
    def __init__(self, D, n, phi, q_cut=10):
        self.D, self.n, self.phi = D, n, phi
        self.h = 2.0 / n
        self.q_cut = q_cut
        self.ncells = n ** D
        self.vol_full = self.h ** D
        self.area_full = self.h ** (D - 1)
        self._classify_cells()
        self._cut_cells()
        self._faces()

    # -- indexing -------------------------------------------------------
    def cell_multi(self, j):
        j = np.asarray(j)
        return np.stack([(j // self.n ** d) % self.n for d in range(self.D)], axis=-1)

    def cell_index(self, I):
        I = np.asarray(I)
        return sum(I[..., d] * self.n ** d for d in range(self.D))

    def cell_box(self, j):
        I = self.cell_multi(j)
        lo = -1.0 + self.h * I
        return lo, lo + self.h

    def transverse_dims(self, d):
        return [e for e in range(self.D) if e != d]

    def face_cells(self, d, plane, t):
        """(below, above) cell indices of face (d, plane, t); -1 on the boundary."""
        dims = self.transverse_dims(d)
        t = np.asarray(t)
        I = np.zeros(t.shape + (self.D,), dtype=np.int64)
        for k, e in enumerate(dims):
            I[..., e] = (t // self.n ** k) % self.n
        plane = np.asarray(plane)
        Ib = I.copy()
        Ib[..., d] = plane - 1
        Ia = I.copy()
        Ia[..., d] = plane
        below = np.where(plane >= 1, self.cell_index(np.maximum(Ib, 0)), -1)
        above = np.where(plane <= self.n - 1, self.cell_index(np.minimum(Ia, self.n - 1)), -1)
        return below, above

    def face_box(self, d, plane, t):
        dims = self.transverse_dims(d)
        lo = np.empty(self.D - 1)
        for k, e in enumerate(dims):
            lo[k] = -1.0 + self.h * ((t // self.n ** k) % self.n)
        return lo, lo + self.h, -1.0 + self.h * plane

    # -- classification --------------------------------------------------
    def _term_bounds_1d(self, d):
        """Bounds of a_d x^2 + b_d x over every cell interval of direction d."""
        lo = -1.0 + self.h * np.arange(self.n)
        hi = lo + self.h
        a, b = self.phi.a[d], self.phi.b[d]
        v0 = a * lo * lo + b * lo
        v1 = a * hi * hi + b * hi
        mn = np.minimum(v0, v1)
        mx = np.maximum(v0, v1)
        if a != 0.0:
            tv = -b / (2.0 * a)
            inside = (lo < tv) & (tv < hi)
            ext = a * tv * tv + b * tv
            mn = np.where(inside, np.minimum(mn, ext), mn)
            mx = np.where(inside, np.maximum(mx, ext), mx)
        return mn, mx

    def _classify_cells(self):
        I = self.cell_multi(np.arange(self.ncells))
        mn = np.full(self.ncells, self.phi.c)
        mx = np.full(self.ncells, self.phi.c)
        for d in range(self.D):
            tmn, tmx = self._term_bounds_1d(d)
            mn += tmn[I[:, d]]
            mx += tmx[I[:, d]]
        # state: 0 all A, 1 all B, 2 cut (refined below by actual volumes)
        self.state = np.where(mx <= 0.0, 0, np.where(mn >= 0.0, 1, 2)).astype(np.int8)
        self.vol = np.zeros((self.ncells, 2))
        self.vol[self.state == 0, 0] = self.vol_full
        self.vol[self.state == 1, 1] = self.vol_full

    def _cut_cells(self):
        self.cut = {}
        q = self.q_cut
        for j in np.flatnonzero(self.state == 2):
            lo, hi = self.cell_box(j)
            P, W, S = partition_rule([self.phi], lo, hi, q)
            a = S[:, 0] < 0.0
            vA, vB = W[a].sum(), W[~a].sum()
            if vA <= PRESENT_TOL * self.vol_full:
                self.state[j] = 1
                self.vol[j] = (0.0, self.vol_full)
                continue
            if vB <= PRESENT_TOL * self.vol_full:
                self.state[j] = 0
                self.vol[j] = (self.vol_full, 0.0)
                continue
            self.vol[j] = (vA, vB)
            iface = surface_rule(self.phi, lo, hi, q)
            self.cut[int(j)] = CutCellData([(P[a], W[a]), (P[~a], W[~a])], iface)
        self.present = self.vol > 0.0
        self.frac = self.vol / self.vol_full

    def _faces(self):
        """Species areas of every face and rules for cut faces.
        farea[d]: [n+1, n^(D-1), 2];  fcut[(d, plane, t)] = [(P, W) A, (P, W) B]."""
        n, D = self.n, self.D
        nt = n ** (D - 1)
        self.farea = []
        self.fcut = {}
        q = self.q_cut
        for d in range(D):
            planes = np.repeat(np.arange(n + 1), nt)
            ts = np.tile(np.arange(nt), n + 1)
            below, above = self.face_cells(d, planes, ts)
            # face bounds of phi: plane term exact, transverse terms from cells
            x = -1.0 + self.h * planes
            mn = self.phi.c + self.phi.a[d] * x * x + self.phi.b[d] * x
            mx = mn.copy()
            dims = self.transverse_dims(d)
            for k, e in enumerate(dims):
                tmn, tmx = self._term_bounds_1d(e)
                ie = (ts // n ** k) % n
                mn = mn + tmn[ie]
                mx = mx + tmx[ie]
            area = np.zeros((n + 1, nt, 2))
            allA = (mx <= 0.0).reshape(n + 1, nt)
            allB = (mn >= 0.0).reshape(n + 1, nt)
            area[..., 0][allA] = self.area_full
            area[..., 1][allB] = self.area_full
            cutf = np.flatnonzero(~(allA | allB).reshape(-1))
            for f in cutf:
                plane, t = divmod(int(f), nt)
                lo, hi, xp = self.face_box(d, plane, t)
                fphi = self.phi.restrict(d, xp)
                P, W, S = partition_rule([fphi], lo, hi, q)
                Pf = np.insert(P, d, xp, axis=1)
                a = S[:, 0] < 0.0
                rules = [(Pf[a], W[a]), (Pf[~a], W[~a])]
                ar = [W[a].sum(), W[~a].sum()]
                area[plane, t] = ar
                self.fcut[(d, plane, t)] = rules
            # a face piece of species s needs species s in the adjacent cell(s)
            b = below.reshape(n + 1, nt)
            ab = above.reshape(n + 1, nt)
            for s in range(2):
                okb = np.where(b >= 0, self.present[np.maximum(b, 0), s], True)
                oka = np.where(ab >= 0, self.present[np.maximum(ab, 0), s], True)
                tiny = area[..., s] <= PRESENT_TOL * self.area_full
                area[..., s] = np.where(okb & oka & ~tiny, area[..., s], 0.0)
            self.farea.append(area)

    # -- rules ------------------------------------------------------------
    def volume_rule(self, j, s, q_std):
        """Rule for K_j intersected with species s (empty if absent)."""
        j = int(j)
        if j in self.cut:
            return self.cut[j].vol_rules[s]
        if not self.present[j, s]:
            return np.zeros((0, self.D)), np.zeros(0)
        lo, hi = self.cell_box(j)
        return tensor_rule(lo, hi, q_std)

    def face_rule(self, d, plane, t, s, q_std):
        key = (d, int(plane), int(t))
        if self.farea[d][plane, t, s] <= 0.0:
            return np.zeros((0, self.D)), np.zeros(0)
        if key in self.fcut:
            return self.fcut[key][s]
        lo, hi, xp = self.face_box(d, plane, t)
        P, W = tensor_rule(lo, hi, q_std)
        return np.insert(P, d, xp, axis=1), W

    def interface_rule(self, j):
        j = int(j)
        if j in self.cut:
            return self.cut[j].iface
        return None

    def interface_area(self, j):
        r = self.interface_rule(j)
        return 0.0 if r is None else float(r[1].sum())

    def cell_faces(self, j):
        """The 2D faces of cell j as (d, plane, t, outward sign)."""
        I = self.cell_multi(j)
        out = []
        for d in range(self.D):
            dims = self.transverse_dims(d)
            t = sum(int(I[e]) * self.n ** k for k, e in enumerate(dims))
            out.append((d, int(I[d]), t, -1.0))
            out.append((d, int(I[d]) + 1, t, +1.0))
        return out
