"""FP64 oracle of the paper's orthonormalisation multigrid -- test
infrastructure only (imported by tests, never by the product path).

Section 3.3, Algorithm ResMinimi (residual minimisation RM) and Algorithm
OrthoMG.  RM(x0, z, W, Z) appends the new direction z: w = M z is made
orthonormal to the stored W by Gram-Schmidt (z receives the same
combination, so W = M Z keeps holding), both are scaled by 1/|w|, and the
coefficients alpha_i = w_i . r0 give x = x0 + Z alpha, r = r0 - W alpha, the
residual of least 2-norm over x0 + span(Z).  OrthoMG applies RM after the
pre-smoother, after the coarse-grid correction and after the post-smoother;
the coarse correction is one OrthoMG cycle on the Galerkin level below, with
the direct solve on the coarsest level.

Readings (the printed listing is ambiguous there): the smoothers act on the
current residual, from zero, with the damped block-Jacobi sweeps of the V-cycle
(standing in for the additive Schwarz smoother); z is scaled together with w;
the top level restarts (x0 := x, r0 := r, Z = W = empty) once `restart`
directions are stored, as GMRES(m) does; coarse levels run one cycle from
x0 = 0.
"""
import numpy as np

from .mg import jacobi


class _Store:
    """The family Z, W = M Z (W orthonormal) and the coefficients alpha of
    one level, together with the x0 and r0 they refer to."""

    def __init__(self, x0, r0):
        self.x0, self.r0 = x0.copy(), r0.copy()
        self.Z, self.W, self.alpha = [], [], []

    def x(self):
        x = self.x0.copy()
        for a, z in zip(self.alpha, self.Z):
            x = x + a * z
        return x

    def r(self):
        r = self.r0.copy()
        for a, w in zip(self.alpha, self.W):
            r = r - a * w
        return r


def rm(M, st, z):
    """Algorithm ResMinimi: append direction z to the store; returns (x, r)."""
    w = M @ z
    z = z.copy()
    for wi, zi in zip(st.W, st.Z):          # Gram-Schmidt, one vector at a time
        beta = wi @ w
        w = w - beta * wi
        z = z - beta * zi
    gamma = 1.0 / np.linalg.norm(w)
    w, z = gamma * w, gamma * z
    st.W.append(w)
    st.Z.append(z)
    st.alpha.append(w @ st.r0)
    return st.x(), st.r()


def cycle(H, level, st):
    """One pass of the OrthoMG loop body on `level` for the store st (three
    RM steps); returns (x, r)."""
    M, D = H.A[level], H.Dinv[level]
    r = st.r()
    z = jacobi(M, D, r, np.zeros_like(r), H.omega, H.nu_pre)     # pre-smoother
    x, r = rm(M, st, z)
    rc = H.R[level].T @ r                                          # restrict residual
    zc = solve_level(H, level + 1, rc)                             # coarse correction
    x, r = rm(M, st, H.R[level] @ zc)
    z = jacobi(M, D, r, np.zeros_like(r), H.omega, H.nu_post)    # post-smoother
    return rm(M, st, z)


def solve_level(H, level, b):
    """OrthoMG(0, b, M^level) with one cycle (direct solve on the coarsest)."""
    if level == H.nlev - 1:
        return H.coarse_solve(b)
    st = _Store(np.zeros_like(b), b)
    x, _ = cycle(H, level, st)
    return x


def solve(H, b, rtol=1e-10, max_cycles=500, restart=30, x0=None):
    """The top-level OrthoMG solver.  Returns (x, history of |r|/|b| after
    every cycle, cycles)."""
    M = H.A[0]
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - M @ x
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / nb]
    st = _Store(x, r)
    k = 0
    while hist[-1] > rtol and k < max_cycles:
        if len(st.Z) + 3 > restart:
            st = _Store(x, r)
        x, r = cycle(H, 0, st)
        k += 1
        hist.append(np.linalg.norm(r) / nb)
    return x, hist, k
