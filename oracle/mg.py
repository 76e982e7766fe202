"""FP64 oracle: block operator, transfers, Galerkin hierarchy, damped block
Jacobi, V-cycle, PCG and FGMRES -- test infrastructure only.

Every routine is the textbook definition written out with scipy/numpy
primitives (sparse products, dense Cholesky); no blocking or fusion beyond
the definitions.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

T_PTRUNC, T_DENSE = 0, 1


def block_matrix(row_ptr, col_idx, val):
    """The level matrix M of Eq. GenericMatrixSystem from its block rows:
    block b of row i is M[m(i, r), m(col_idx[b], c)] = val[b, r, c]."""
    n_rows = len(row_ptr) - 1
    Np = val.shape[1]
    return sp.bsr_matrix((val, np.asarray(col_idx), np.asarray(row_ptr)),
                         shape=(n_rows * Np, n_rows * Np)).tocsr()


def block_operator(row_ptr, col_idx, val, n_cols):
    """A rectangular block operator (n_rows block rows, n_cols block columns,
    Np x Np blocks) as a sparse matrix: the L2 re-projection between the
    agglomerated spaces of two time levels (Section 2.3) is applied as
    x_new = P x_old."""
    n_rows = len(row_ptr) - 1
    Np = val.shape[1]
    return sp.bsr_matrix((val, np.asarray(col_idx), np.asarray(row_ptr)),
                         shape=(n_rows * Np, n_cols * Np)).tocsr()


def transfer_matrix(T, n_rows_f, np_f):
    """R^{X,lambda} in R^{L_f x L_c} (Eq. XDGrestrictionMatrix): the
    coefficients of the coarse basis in the fine basis.  p-levels keep the
    leading np_c modes of every block row (R_i = [I; 0]); aggregation levels
    place the per-fine-row projection block R_i at (i, parent[i])."""
    np_c, n_c = T["np_c"], T["n_rows_c"]
    parent = np.asarray(T["parent"], dtype=np.int64)
    if T["kind"] == T_PTRUNC:
        Ri = np.zeros((np_f, np_c))
        Ri[:np_c, :np_c] = np.eye(np_c)
        blocks = np.broadcast_to(Ri, (n_rows_f, np_f, np_c))
    else:
        blocks = np.asarray(T["R"])
    rows = (np.arange(n_rows_f)[:, None, None] * np_f + np.arange(np_f)[None, :, None])
    cols = parent[:, None, None] * np_c + np.arange(np_c)[None, None, :]
    rows, cols = np.broadcast_arrays(rows, cols)
    return sp.csr_matrix((blocks.reshape(-1), (rows.reshape(-1), cols.reshape(-1))),
                         shape=(n_rows_f * np_f, n_c * np_c))


def galerkin(A, R):
    """M^{lambda+1} = R^T M^lambda R (Eq. XDGsysRestriction)."""
    return (R.T @ A @ R).tocsr()


def cell_block_inverses(A, cell_ptr, Np):
    """Inverse of every diagonal cell block D_c = M[I_c, I_c], I_c all rows of
    one cell block (all species of one representative cell; the per-cell
    dense solves of Section 3.3, Alg. pMultigrid), by FP64 Cholesky.
    Returns the block-diagonal D^{-1} as a sparse matrix and the list of
    dense inverses."""
    A = A.tocsr()
    invs = []
    for c in range(len(cell_ptr) - 1):
        lo, hi = cell_ptr[c] * Np, cell_ptr[c + 1] * Np
        Dc = A[lo:hi, lo:hi].toarray()
        fac = sla.cho_factor(Dc, lower=True)
        invs.append(sla.cho_solve(fac, np.eye(hi - lo)))
    return sp.block_diag(invs, format="csr"), invs


def jacobi(A, Dinv, b, x, omega, sweeps):
    """Damped block Jacobi: x <- x + omega D^{-1} (b - M x), `sweeps` times."""
    for _ in range(sweeps):
        x = x + omega * (Dinv @ (b - A @ x))
    return x


class Hierarchy:
    """Galerkin multigrid hierarchy from the level-0 matrix and transfers."""

    def __init__(self, row_ptr, col_idx, val, cell_ptr, transfers, omega=0.7, nu_pre=2,
                 nu_post=2, nu_coarse=0):
        # nu_coarse > 0: that many sweeps before and after the coarse
        # correction on every level below the finest (else nu_pre / nu_post)
        self.omega, self.nu_pre, self.nu_post = omega, nu_pre, nu_post
        self.nu_coarse = nu_coarse
        Np = val.shape[1]
        self.A = [block_matrix(row_ptr, col_idx, val)]
        self.np = [Np]
        self.cell_ptr = [np.asarray(cell_ptr)]
        self.n_rows = [len(row_ptr) - 1]
        self.R = []
        for T in transfers:
            R = transfer_matrix(T, self.n_rows[-1], self.np[-1])
            self.R.append(R)
            self.A.append(galerkin(self.A[-1], R))
            self.np.append(T["np_c"])
            self.n_rows.append(T["n_rows_c"])
            self.cell_ptr.append(np.asarray(T["cell_ptr_c"]))
        self.nlev = len(self.A)
        self.Dinv = []
        for l in range(self.nlev - 1):
            self.Dinv.append(cell_block_inverses(self.A[l], self.cell_ptr[l], self.np[l])[0])
        # coarsest level: dense FP64 Cholesky (the low-order direct solve)
        self.coarse = sla.cho_factor(self.A[-1].toarray(), lower=True)

    def coarse_solve(self, r):
        return sla.cho_solve(self.coarse, r)

    def vcycle(self, r, level=0):
        """z = B r: symmetric V-cycle (pre-smoothing from zero, residual,
        restriction R^T, recursive coarse correction, prolongation R,
        post-smoothing; exact solve on the coarsest level)."""
        if level == self.nlev - 1:
            return self.coarse_solve(r)
        A, D = self.A[level], self.Dinv[level]
        coarse = level > 0 and self.nu_coarse > 0
        nu_pre = self.nu_coarse if coarse else self.nu_pre
        nu_post = self.nu_coarse if coarse else self.nu_post
        x = jacobi(A, D, r, np.zeros_like(r), self.omega, nu_pre)
        rc = self.R[level].T @ (r - A @ x)
        x = x + self.R[level] @ self.vcycle(rc, level + 1)
        return jacobi(A, D, r, x, self.omega, nu_post)

    def lambda_max_DinvA(self, level, iters=200, seed=0):
        """Power-iteration estimate of the largest eigenvalue of D^{-1} A
        (diagnostic for the smoother's damping)."""
        A, D = self.A[level], self.Dinv[level]
        v = np.random.default_rng(seed).standard_normal(A.shape[0])
        lam = 0.0
        for _ in range(iters):
            w = D @ (A @ v)
            lam = float(np.linalg.norm(w) / np.linalg.norm(v))
            v = w / np.linalg.norm(w)
        return lam


def pcg(A, b, precond, rtol=1e-10, maxit=500, x0=None):
    """Preconditioned conjugate gradients (textbook form).  Returns
    (x, history of ||r_k||/||b|| for k = 0..iters, iters)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / nb]
    if hist[-1] <= rtol:
        return x, hist, 0
    z = precond(r)
    p = z.copy()
    rz = r @ z
    for k in range(1, maxit + 1):
        q = A @ p
        alpha = rz / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= rtol:
            return x, hist, k
        z = precond(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, hist, maxit


def fgmres(A, b, precond, rtol=1e-8, restart=30, maxit=500, x0=None):
    """Flexible GMRES(restart) with modified Gram-Schmidt Arnoldi and Givens
    rotations (Saad's right-preconditioned flexible variant).  Returns
    (x, history of ||r||/||b|| per inner iteration, total iterations)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    nb = np.linalg.norm(b)
    r = b - A @ x
    beta = np.linalg.norm(r)
    hist = [beta / nb]
    it = 0
    while hist[-1] > rtol and it < maxit:
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        j = 0
        for j in range(restart):
            z = precond(V[j])
            Z.append(z)
            w = A @ z
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j] if H[j + 1, j] != 0.0 else w)
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            hist.append(abs(g[j + 1]) / nb)
            if hist[-1] <= rtol or it >= maxit:
                break
        m = j + 1
        y = sla.solve_triangular(H[:m, :m], g[:m])
        x = x + np.column_stack(Z) @ y
        r = b - A @ x
        beta = np.linalg.norm(r)
        hist[-1] = beta / nb
    return x, hist, it


def hierarchy_of(pr, omega=0.7, nu=2, nu_coarse=0):
    """Hierarchy of a generated problem (any object carrying row_ptr, col_idx,
    val, cell_ptr and transfers)."""
    return Hierarchy(pr.row_ptr, pr.col_idx, pr.val, pr.cell_ptr, pr.transfers,
                     omega=omega, nu_pre=nu, nu_post=nu, nu_coarse=nu_coarse)
