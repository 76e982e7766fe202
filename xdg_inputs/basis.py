"""Polynomial bases on aggregate cells.

Section 3.2 builds the basis of an aggregated (cut) cell from an ansatz on the
bounding box of the aggregation cell and re-orthonormalises it on the actual
(cut, agglomerated) part through a Cholesky factor (Eq. XdgMgBasis, matrix S).
Here the ansatz is the tensor Legendre family of total degree <= p on the
axis-aligned bounding box, ordered by total degree; for a part P with Gram
matrix G = int_P psi psi^T = L L^T the orthonormal basis is phi = psi L^{-T}.
Because L^{-T} is upper triangular and the family is graded by degree, the
first N_k functions of phi span exactly the polynomials of degree <= k on P,
which makes the p-multigrid restriction a truncation of the mode vector.
"""
from functools import lru_cache
from math import comb

import numpy as np
from scipy.linalg import solve_triangular


def n_modes(D, p):
    """Dimension of the total-degree-p polynomial space in D dims."""
    return comb(p + D, D)


@lru_cache(maxsize=None)
def multi_indices(D, p):
    """Exponent tuples of total degree <= p, graded by degree, lexicographic
    (first coordinate varying slowest) within a degree."""
    out = []
    for deg in range(p + 1):
        def rec(prefix, left, dims):
            if dims == 1:
                yield prefix + (left,)
                return
            for e in range(left, -1, -1):
                yield from rec(prefix + (e,), left - e, dims - 1)
        out.extend(rec((), deg, D))
    return tuple(out)


def legendre_1d(t, p):
    """Orthonormal Legendre values and derivatives on [-1, 1]:
    L_n(t) = sqrt((2n+1)/2) P_n(t), n = 0..p.  Returns (V, dV) [..., p+1]."""
    t = np.asarray(t, dtype=np.float64)
    P = np.zeros(t.shape + (p + 1,))
    dP = np.zeros(t.shape + (p + 1,))
    P[..., 0] = 1.0
    if p >= 1:
        P[..., 1] = t
        dP[..., 1] = 1.0
    for n in range(1, p):
        P[..., n + 1] = ((2 * n + 1) * t * P[..., n] - n * P[..., n - 1]) / (n + 1)
        dP[..., n + 1] = dP[..., n - 1] + (2 * n + 1) * P[..., n]
    scale = np.sqrt((2.0 * np.arange(p + 1) + 1.0) / 2.0)
    return P * scale, dP * scale


class BoxBasis:
    """Tensor Legendre family of total degree <= p on the box [lo, hi],
    scaled to be orthonormal on the full box."""

    def __init__(self, lo, hi, p):
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.p = p
        self.D = len(self.lo)
        self.idx = np.array(multi_indices(self.D, p), dtype=np.int64)   # [Np, D]
        self.np = len(self.idx)
        self.ctr = 0.5 * (self.lo + self.hi)
        self.half = 0.5 * (self.hi - self.lo)

    def eval(self, X, grad=True):
        """psi [N, Np] and, if grad, dpsi [N, Np, D] at points X [N, D]."""
        X = np.asarray(X, dtype=np.float64)
        xi = (X - self.ctr) / self.half
        D = self.D
        norm = np.prod(1.0 / np.sqrt(self.half))
        V, dV = [], []
        for d in range(D):
            v, dv = legendre_1d(xi[:, d], self.p)
            V.append(v[:, self.idx[:, d]])              # [N, Np]
            dV.append(dv[:, self.idx[:, d]] / self.half[d])
        psi = np.ones((X.shape[0], self.np))
        for d in range(D):
            psi = psi * V[d]
        psi = psi * norm
        if not grad:
            return psi
        dpsi = np.empty((X.shape[0], self.np, D))
        for d in range(D):
            g = np.ones((X.shape[0], self.np))
            for e in range(D):
                g = g * (dV[e] if e == d else V[e])
            dpsi[:, :, d] = g * norm
        return psi, dpsi


class PartBasis:
    """Orthonormal basis phi = psi C on one part (C upper triangular, or the
    identity for a full, non-agglomerated background cell)."""

    def __init__(self, box, C=None):
        self.box = box
        self.C = C          # None means identity
        self.np = box.np

    def eval(self, X, grad=True):
        if grad:
            psi, dpsi = self.box.eval(X, True)
            if self.C is None:
                return psi, dpsi
            return psi @ self.C, np.matmul(dpsi.transpose(0, 2, 1), self.C).transpose(0, 2, 1)
        psi = self.box.eval(X, False)
        return psi if self.C is None else psi @ self.C

    def truncated(self, nlo):
        """Basis of the leading nlo modes (same part, lower degree)."""
        return self.C is None, (None if self.C is None else self.C[:nlo, :nlo])


def orthonormalize(G):
    """C = L^{-T} with G = L L^T, so that C^T G C = I (C upper triangular)."""
    L = np.linalg.cholesky(G)
    return solve_triangular(L.T, np.eye(G.shape[0]), lower=False, check_finite=False)
