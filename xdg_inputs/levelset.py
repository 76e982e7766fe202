"""Separable quadric level sets  phi(x) = c + sum_d (a_d x_d^2 + b_d x_d).

The interface of the paper's two-phase problems is the zero set of a level-set
function phi; species A is {phi < 0}, species B is {phi > 0}, and the interface
normal grad(phi)/|grad(phi)| points from A to B (Section 1.1, Eq.
poisson-jump-problem-def; Section 2.1).  Every workload used here (circle,
sphere, axis-aligned ellipsoid, plane) is a separable quadric, which gives
exact bounds on a box, exact restrictions to a coordinate plane and closed-form
roots along a coordinate line -- the three primitives the cut-cell quadrature
needs.
"""
import numpy as np


class Quadric:
    """phi(x) = c + sum_d a[d] x_d^2 + b[d] x_d  on R^dim."""

    def __init__(self, a, b, c):
        self.a = np.asarray(a, dtype=np.float64).copy()
        self.b = np.asarray(b, dtype=np.float64).copy()
        self.c = float(c)
        self.dim = len(self.a)

    # -- constructors -----------------------------------------------------
    @staticmethod
    def sphere(center, r):
        """|x - center|^2 - r^2 (circle in 2D, sphere in 3D)."""
        ctr = np.asarray(center, dtype=np.float64)
        return Quadric(np.ones_like(ctr), -2.0 * ctr, float(ctr @ ctr) - r * r)

    @staticmethod
    def ellipsoid(center, semi_axes):
        """sum_d ((x_d - c_d)/s_d)^2 - 1, axis aligned."""
        ctr = np.asarray(center, dtype=np.float64)
        s = np.asarray(semi_axes, dtype=np.float64)
        a = 1.0 / (s * s)
        return Quadric(a, -2.0 * a * ctr, float(np.sum(a * ctr * ctr)) - 1.0)

    @staticmethod
    def plane(normal, offset):
        """normal . x - offset (linear level set, exact polytope cuts)."""
        nrm = np.asarray(normal, dtype=np.float64)
        return Quadric(np.zeros_like(nrm), nrm, -float(offset))

    # -- evaluation -------------------------------------------------------
    def __call__(self, X):
        X = np.asarray(X, dtype=np.float64)
        return self.c + (X * X) @ self.a + X @ self.b

    def grad(self, X):
        X = np.asarray(X, dtype=np.float64)
        return 2.0 * self.a * X + self.b

    def hessian_trace(self):
        """Laplacian of phi (a constant)."""
        return 2.0 * float(np.sum(self.a))

    # -- interval arithmetic on boxes (exact for separable quadrics) ------
    def _term_bounds(self, d, lo, hi):
        a, b = self.a[d], self.b[d]
        cand = [a * lo * lo + b * lo, a * hi * hi + b * hi]
        if a != 0.0:
            t = -b / (2.0 * a)
            if lo < t < hi:
                cand.append(a * t * t + b * t)
        return min(cand), max(cand)

    def bounds(self, lo, hi):
        mn = mx = self.c
        for d in range(self.dim):
            m, M = self._term_bounds(d, lo[d], hi[d])
            mn += m
            mx += M
        return mn, mx

    def dbounds(self, k, lo, hi):
        """Range of d(phi)/dx_k over the box (depends on x_k only)."""
        v0 = 2.0 * self.a[k] * lo[k] + self.b[k]
        v1 = 2.0 * self.a[k] * hi[k] + self.b[k]
        return min(v0, v1), max(v0, v1)

    def grad_norm_max(self, lo, hi):
        s = 0.0
        for d in range(self.dim):
            v0 = abs(2.0 * self.a[d] * lo[d] + self.b[d])
            v1 = abs(2.0 * self.a[d] * hi[d] + self.b[d])
            s += max(v0, v1) ** 2
        return np.sqrt(s)

    # -- restriction and roots -------------------------------------------
    def restrict(self, k, t):
        """phi with x_k fixed to t, as a quadric in the remaining dims."""
        keep = [d for d in range(self.dim) if d != k]
        return Quadric(self.a[keep], self.b[keep],
                       self.c + self.a[k] * t * t + self.b[k] * t)

    def partial_sum(self, Xb, k):
        """c + sum_{d != k} (a_d x_d^2 + b_d x_d) for base points Xb (dims != k)."""
        keep = [d for d in range(self.dim) if d != k]
        a, b = self.a[keep], self.b[keep]
        return self.c + (Xb * Xb) @ a + Xb @ b

    def root_along(self, Xb, k, lo, hi):
        """Root in [lo, hi] of t -> phi(xb, x_k = t) where the caller has
        established a sign change over [lo, hi] and monotonicity in x_k."""
        C = self.partial_sum(Xb, k)
        a, b = self.a[k], self.b[k]
        if a == 0.0:
            z = -C / b
        else:
            disc = np.maximum(b * b - 4.0 * a * C, 0.0)
            sq = np.sqrt(disc)
            qq = -0.5 * (b + np.where(b >= 0.0, sq, -sq))
            with np.errstate(divide="ignore", invalid="ignore"):
                r1 = qq / a
                r2 = np.where(qq != 0.0, C / qq, r1)
            mid = 0.5 * (lo + hi)
            z = np.where(np.abs(r1 - mid) <= np.abs(r2 - mid), r1, r2)
        return np.clip(z, lo, hi)

    def roots_1d(self, lo, hi):
        """All roots of a 1D quadric strictly inside (lo, hi), sorted."""
        assert self.dim == 1
        a, b, c = self.a[0], self.b[0], self.c
        out = []
        if a == 0.0:
            if b != 0.0:
                out.append(-c / b)
        else:
            disc = b * b - 4.0 * a * c
            if disc >= 0.0:
                sq = np.sqrt(disc)
                qq = -0.5 * (b + (sq if b >= 0.0 else -sq))
                out.append(qq / a)
                if qq != 0.0:
                    out.append(c / qq)
        return sorted(r for r in out if lo < r < hi)
