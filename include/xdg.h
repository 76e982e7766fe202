/*
 * libxdg -- multigrid-preconditioned solve of the agglomerated cut-cell SIP
 * system of the extended discontinuous Galerkin (XDG) method on one MI355X.
 *
 * The linear system is the matrix form of the discretisation on the
 * agglomerated XDG space (paper Section 3.2, Eq. GenericMatrixSystem):
 *     M U = b,  M[m(j,s,n), m(l,r,k)] = a(Phi_{l,r,k}, Phi_{j,s,n}),
 * one block row per (aggregate cell, species), Np = dim P_k modes per block.
 * Coarse levels come from transfer matrices R^{X,lambda} (Eq.
 * XDGrestrictionMatrix) through the Galerkin product
 * M^{lambda+1} = R^T M^lambda R (Eq. XDGsysRestriction).
 *
 * Conventions for every call:
 *   - return value: 0 = XDG_OK, > 0 warning, < 0 error; no call aborts or
 *     throws across this interface; xdg_last_error() describes the last
 *     failure of the calling thread.
 *   - host arrays passed to xdg_create are owned by the caller and may be
 *     freed when it returns (everything is copied to the device).
 *   - *_dev pointers are caller-owned device buffers on the handle's device;
 *     outputs must not alias inputs.
 *   - every call is enqueued on the handle's HIP stream; only xdg_create,
 *     the set-up calls xdg_update_matrix / xdg_update_cells (they report
 *     non-positive pivots), xdg_solve and the xdg_get_* copies synchronise
 *     it, and those return with the stream idle.
 *   - vectors are FP64, laid out [block row][mode] (row-major), length
 *     n_rows * np of the level they live on; a handle created with
 *     nrhs = 16 takes 16 columns per vector, laid out [block row][mode][16].
 */
#ifndef XDG_H
#define XDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    XDG_OK = 0,
    XDG_ENOCONV = 1,      /* iteration limit reached; x and history are valid  */
    XDG_EINVAL = -1,      /* bad sizes/indices, unsorted rows, NaN/Inf input   */
    XDG_ENOMEM = -2,      /* device allocation failed                          */
    XDG_EHIP = -3,        /* HIP runtime error                                 */
    XDG_ENOTSPD = -4,     /* non-positive pivot in a cell block or the coarse  */
                          /* matrix                                            */
    XDG_EBREAKDOWN = -5   /* Krylov breakdown (p^T A p <= 0 or zero Arnoldi)   */
};

enum { XDG_T_PTRUNC = 0, XDG_T_DENSE = 1 };
enum { XDG_CG = 0, XDG_FGMRES = 1, XDG_ORTHOMG = 2 };
enum { XDG_FP64 = 0, XDG_MIXED = 1 };
enum { XDG_JACOBI = 0, XDG_LEARNED = 1, XDG_LEARNED_BF16 = 2 };

typedef struct xdg_handle xdg_handle;

/* Level-0 system matrix (host memory, caller-owned).
 * Block rows are (aggregate, species) pairs (Section 3.2, index convention);
 * block b of row i holds M[m(i, r), m(col_idx[b], c)] = val[b*np*np + r*np + c].
 * col_idx must be sorted within each row and contain the diagonal.
 * Smoother cell blocks: cell c owns the consecutive block rows
 * [cell_ptr[c], cell_ptr[c+1]) (all species of one representative cell, the
 * blocks m(j,-,-,.) of Section 3.3). */
typedef struct {
    int32_t n_rows, np, nnzb;
    const int32_t *row_ptr;   /* [n_rows + 1], row_ptr[0] = 0, row_ptr[n_rows] = nnzb */
    const int32_t *col_idx;   /* [nnzb] */
    const double  *val;       /* [nnzb * np * np] */
    int32_t n_cells;
    const int32_t *cell_ptr;  /* [n_cells + 1] */
} xdg_matrix;

/* Transfer from level lambda (fine, n_rows_f x np_f) to lambda+1 (Section 3.2).
 * kind XDG_T_PTRUNC: same block rows, the coarse space keeps the leading np_c
 *   modes of every block (graded orthonormal bases: R_i = [I; 0]); parent and
 *   R are ignored (may be NULL).
 * kind XDG_T_DENSE: fine row i lies in coarse row parent[i]; its projection
 *   block R_i (np_f x np_c, row-major) is R[i*np_f*np_c + a*np_c + m] =
 *   int_{P_i} phi_{i,a} phi_{parent(i),m}. */
typedef struct {
    int32_t kind, n_rows_c, np_c;
    const int32_t *parent;    /* [n_rows_f] */
    const double  *R;         /* [n_rows_f * np_f * np_c] */
    int32_t n_cells_c;
    const int32_t *cell_ptr_c;/* [n_cells_c + 1] coarse smoother blocks */
} xdg_transfer;

typedef struct {
    int32_t krylov;           /* XDG_CG (flexible CG with XDG_MIXED) | XDG_FGMRES */
                              /* | XDG_ORTHOMG (see xdg_solve)                  */
    int32_t restart;          /* FGMRES restart length (<= 64)                  */
    int32_t maxit;            /* Krylov iteration limit                         */
    int32_t nu_pre, nu_post;  /* block-Jacobi sweeps per level                  */
    int32_t precision;        /* XDG_FP64 | XDG_MIXED (FP32 V-cycle)            */
    int32_t smoother;         /* XDG_JACOBI | XDG_LEARNED | XDG_LEARNED_BF16    */
    int32_t nrhs;             /* 1, or 16 (needs XDG_FGMRES + XDG_MIXED): block */
                              /* products of the V-cycle on FP32 MFMA, Arnoldi  */
                              /* matvec and restart residuals on FP64 MFMA      */
    double  rtol;             /* stop at ||b - M x||_2 / ||b||_2 <= rtol        */
    double  omega;            /* Jacobi damping                                 */
    int32_t symmetric;        /* 1: the level-0 matrix is symmetric (the SIP    */
                              /* form of Eq. DefSIP is): single-column solves   */
                              /* read its diagonal and upper blocks only and    */
                              /* take each lower block (i, j) as the transpose  */
                              /* of the stored (j, i); used for np = 20, other  */
                              /* block sizes read every block.  The pattern     */
                              /* must then be symmetric (else XDG_EINVAL); the  */
                              /* values of the lower blocks are not read by the */
                              /* solve (set-up and xdg_get_level_matrix use     */
                              /* all blocks).  0: every block is read.          */
    int32_t nu_coarse;        /* > 0: block-Jacobi sweeps before and after the  */
                              /* coarse correction on every level below the     */
                              /* finest in the V-cycle of xdg_vcycle/xdg_solve  */
                              /* (CG, FGMRES; the orthonormalisation MG keeps   */
                              /* nu_pre/nu_post); 0: nu_pre/nu_post there too   */
} xdg_options;

/* Copies the level-0 system and transfers to the device, forms every coarse
 * level by the Galerkin product, inverts every smoother cell block (FP64
 * Gauss-Jordan) and the coarsest matrix, and (XDG_MIXED) makes FP32 copies.
 * hip_stream: a hipStream_t (NULL = default stream).  On error *out is NULL. */
int xdg_create(const xdg_matrix *A0, int32_t n_levels, const xdg_transfer *T,
               const xdg_options *opt, void *hip_stream, xdg_handle **out);

/* y = M^lambda x on level `level`: the operator of the level's system
 * (Eq. GenericMatrixSystem on level 0, the Galerkin matrix of Eq.
 * XDGsysRestriction below it), one dense Np x Np block per stored
 * (row, column) pair.  x_dev, y_dev: n_rows * np doubles of that level
 * (caller-owned, device).  A 16-column handle computes the FP64
 * matrix-core product of level 0 on [row][mode][16] vectors and returns
 * XDG_EINVAL for level > 0 (xdg_spmm with XDG_MIXED covers those). */
int xdg_spmv(xdg_handle *h, int32_t level, const double *x_dev, double *y_dev);

/* `sweeps` damped block-Jacobi sweeps x <- x + omega D^{-1} (b - M x) on
 * `level` (level < n_levels - 1), D the cell-block diagonal.  The blocks are
 * the per-cell dense solves of Section 3.3 (Algorithm pMultigrid solves the
 * system restricted to the modes m(j,-,-,.) of one cell j directly), taken
 * over all modes and all species of a cell and applied to every cell at once
 * with damping omega.  b_dev is read, x_dev updated in place (both n_rows * np
 * doubles of the level, times 16 on a 16-column handle, which sweeps in FP32
 * on the matrix cores).  sweeps >= 0. */
int xdg_smooth(xdg_handle *h, int32_t level, const double *b_dev, double *x_dev,
               int32_t sweeps);

/* rc = (R^{X,level})^T rf : fine level `level` -> level+1, with R^{X,level}
 * the prolongation matrix of Eq. XDGrestrictionMatrix (per fine block row
 * the projection of the fine basis onto the coarse one; on a p-level the
 * leading coarse modes, Section 3.2) and its transpose the restriction of
 * Eq. XDGsysRestriction.  rf_dev: fine level vector, rc_dev: coarse level
 * vector (overwritten); [row][mode][16] on a 16-column handle (FP64). */
int xdg_restrict(xdg_handle *h, int32_t level, const double *rf_dev, double *rc_dev);

/* xf += R^{X,level} xc : level+1 -> fine level `level` (Eq.
 * XDGrestrictionMatrix); xf_dev is accumulated into, xc_dev read;
 * [row][mode][16] on a 16-column handle (FP64). */
int xdg_prolong(xdg_handle *h, int32_t level, const double *xc_dev, double *xf_dev);

/* z = B r, one symmetric V-cycle from level 0: on every level nu_pre damped
 * block-Jacobi sweeps from zero, residual, restriction, the cycle of the
 * level below, prolongation-add, nu_post sweeps; the coarsest level is
 * solved exactly (its explicit FP64 inverse).  This is the classical cycle
 * of multigrid textbooks over the hierarchy of Section 3.1 (Eq.
 * MultigridAggMeshSeq, Galerkin levels of Eq. XDGsysRestriction); Section
 * 3.3 warns that this cycle can diverge for (X)DG systems, which the
 * orthonormalisation multigrid of Algorithm OrthoMG (krylov XDG_ORTHOMG)
 * guards against.  Pre and post smoothing are alike, so B is symmetric and
 * serves as the CG preconditioner.  r_dev read, z_dev overwritten
 * (level-0 vectors; 16 columns on a 16-column handle). */
int xdg_vcycle(xdg_handle *h, const double *r_dev, double *z_dev);

/* xdg_vcycle for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same cycle with the same kernels and a bit-identical result, but the work
 * vectors of every level live in one fixed device array of 2^22 doubles
 * (32 MiB) that the library reserves once per device and keeps until the
 * process ends.  The call makes no hipMalloc, hipFree or other allocating
 * call.  Single-column handles with the block-Jacobi smoother only (else
 * XDG_EINVAL).  The cycle needs about five doubles per level-0 unknown in
 * FP64 and two and a half in the FP32 cycle (the 32^3 p = 3 workload: about
 * 3.3 million in FP64); a larger one returns XDG_EINVAL.  Every call on one
 * device shares the array and leaves its contents behind: calls that overlap
 * on one device (other streams or threads) race, and the caller must order
 * them.  r_dev read, z_dev overwritten (level-0 vectors). */
int xdg_vcycle_noalloc(xdg_handle *h, const double *r_dev, double *z_dev);

/* Solves M^0 x = b (Eq. GenericMatrixSystem on level 0) with the V-cycle
 * above as preconditioner of CG (XDG_CG; flexible CG with XDG_MIXED) or of
 * flexible GMRES(restart) with FP64 restarts (XDG_FGMRES), until the
 * residual criterion of Section 4, read relative:
 * ||b - M x||_2 / ||b||_2 <= rtol on the coefficient vectors (the paper
 * stops at an absolute 2-norm of 1e-10).  x_dev holds the initial guess on
 * entry and the solution on return.  hist_host[k] = ||r_k||_2/||b||_2, k = 0..*iters (at most
 * hist_cap entries are written); *final_relres is the recomputed true FP64
 * residual.  Returns XDG_ENOCONV (x valid) when maxit is reached.
 * krylov = XDG_ORTHOMG solves with the orthonormalisation multigrid of
 * Section 3.3 (Algorithms ResMinimi and OrthoMG): residual minimisation over
 * the directions of the pre-smoother, the coarse-grid correction (one such
 * cycle on the level below, direct solve on the coarsest) and the
 * post-smoother; the top level's family restarts once `restart` directions
 * would be exceeded; hist_host[k] is the residual after k cycles; FP64 only.
 * b = 0
 * (or a zero column of a 16-column b) gives x = 0 in that column whatever
 * x held, with relative residual 0.  A non-finite b or initial residual
 * returns XDG_EINVAL before any iteration. */
int xdg_solve(xdg_handle *h, const double *b_dev, double *x_dev, double *hist_host,
              int32_t hist_cap, int32_t *iters, double *final_relres);

/* Y = M^level X for 16 columns (handle created with nrhs = 16) on the matrix
 * cores: precision XDG_FP64 uses the FP64 blocks (level 0 only), XDG_MIXED
 * the FP32 copy of the level (accumulation in FP32); X, Y are FP64
 * [row][mode][16] either way. */
int xdg_spmm(xdg_handle *h, int32_t level, int32_t precision, const double *X_dev,
             double *Y_dev);

/* Level sizes (for callers allocating level vectors). */
int xdg_level_info(xdg_handle *h, int32_t level, int32_t *n_rows, int32_t *np,
                   int32_t *nnzb);

/* Host copies of the device-built level matrix (row-major blocks) -- the
 * Galerkin product for level > 0.  Arrays sized from xdg_level_info. */
int xdg_get_level_matrix(xdg_handle *h, int32_t level, int32_t *row_ptr,
                         int32_t *col_idx, double *val);

/* Host copy of the inverse of smoother cell block `cell` on `level`
 * (n x n row-major, n = rows_in_cell * np); *n receives its order.
 * On the coarsest level, cell = 0 returns the inverse of the whole matrix. */
int xdg_get_cell_inverse(xdg_handle *h, int32_t level, int32_t cell, double *out,
                         int32_t cap, int32_t *n);

/* New level-0 values with the sparsity pattern given at xdg_create: val_dev
 * is a device buffer (caller-owned, nnzb*np*np FP64, row-major blocks as in
 * xdg_matrix.val).  Recomputes every Galerkin level, every smoother inverse
 * and the coarsest inverse on the device (the numeric part of xdg_create;
 * the hierarchy set-up of the paper's phase (ii), Section 4).  Synchronises
 * the stream; returns XDG_ENOTSPD on a non-positive pivot. */
int xdg_update_matrix(xdg_handle *h, const double *val_dev);

/* Partial form of xdg_update_matrix for new values that differ from the
 * current ones only in the block rows and block columns of the listed level-0
 * smoother cells -- the cut cells of an interface that moves without changing
 * the agglomeration (Section 3.1: the hierarchy's operators are computed once
 * on the background mesh and renewed only in cut cells).  val_dev holds all
 * level-0 values, laid out as for xdg_update_matrix.  Only the affected blocks
 * are re-laid out, only the Galerkin blocks and cell-block inverses they reach
 * are recomputed on every level; the coarsest inverse is rebuilt.  When the
 * values outside those rows and columns are unchanged the result equals
 * xdg_update_matrix's bit for bit.  cells_host: n >= 1 distinct indices in
 * [0, n_cells).  Single-column handles (nrhs = 1); the level-0 block pattern
 * must be symmetric (checked on the first call, XDG_EINVAL otherwise).
 * Synchronises the stream; XDG_ENOTSPD on a non-positive pivot. */
int xdg_update_cells(xdg_handle *h, const double *val_dev, int32_t n,
                     const int32_t *cells_host);

/* Block-sparse operator from the level-0 space of an earlier time level
 * (n_cols block rows of np modes) into the level-0 space of this handle: the
 * L2 re-projection that Section 2.3 prescribes between time steps (the
 * finished step's solution, injected into the non-agglomerated cut-cell
 * space, projected onto the agglomerated space of the next step, whose
 * agglomeration map -- and so the block pattern of this handle -- may
 * differ).  Block b of row i is P[m(i, r), m_old(col_idx[b], c)] =
 * val[b*np*np + r*np + c]; n_rows and np must equal level 0's.  Host arrays,
 * copied (they may be freed on return); replaces an earlier operator. */
typedef struct {
    int32_t n_rows, n_cols, np, nnzb;
    const int32_t *row_ptr;   /* [n_rows + 1], row_ptr[0] = 0, row_ptr[n_rows] = nnzb */
    const int32_t *col_idx;   /* [nnzb], strictly increasing per row, in [0, n_cols) */
    const double  *val;       /* [nnzb * np * np], finite */
} xdg_projection;

int xdg_set_projection(xdg_handle *h, const xdg_projection *P);

/* x_new_dev = P x_old_dev with the operator of xdg_set_projection: x_old_dev
 * holds n_cols * np doubles (the earlier level-0 vector), x_new_dev receives
 * this handle's n_rows * np (a starting guess for xdg_solve).  Single-column
 * handles; XDG_EINVAL without an operator. */
int xdg_project(xdg_handle *h, const double *x_old_dev, double *x_new_dev);

/* New stopping rule for later xdg_solve calls: rtol > 0, maxit >= 1. */
int xdg_set_tolerance(xdg_handle *h, double rtol, int32_t maxit);

/* Milliseconds spent in xdg_create on the device (Galerkin products,
 * inversions), measured with HIP events. */
int xdg_setup_time(xdg_handle *h, double *ms);

/* ---- Learned per-cell smoother (a project extension, not in the paper) ----
 * A 45 -> 64 -> 64 -> 40 multilayer perceptron (GELU after both hidden
 * layers, FP32) corrects the first damped block-Jacobi sweep of the level-0
 * smoother (Section 3.3) in every V-cycle.  With x_in = 0 and residual r,
 * per smoother cell c:
 *   j_c = omega D_c^{-1} r_c,  s_c = ||j_c||_2,
 *   features f_c = [ j_c / s_c in species slots | cell_geom[c][0..4] ],
 *     slots: the species-A row of the cell -> 0..19, species B -> 20..39,
 *     zero where the cell has no row of that species;
 *   x_c = j_c + s_c * y_c,  y_c = MLP(f_c) read back from the same slots.
 * The map is scale-equivariant (x scales with r).  Needs np = 20 (p = 3 in
 * 3D), nrhs = 1, XDG_FGMRES, XDG_FP64 and nu_pre >= 1; it is active once
 * parameters (xdg_mlp_set) and cell features (xdg_set_cell_features) exist.
 * Fallbacks: a cell whose proposal is non-finite or has ||y_c||_2 > guard
 * keeps the plain Jacobi step (counted); an FGMRES step that reduces the
 * residual estimate by less than a factor 0.99 while the network is active
 * switches the network off for the rest of that solve (flexible GMRES
 * accepts the changed preconditioner).
 * XDG_LEARNED_BF16 runs the same network on bf16 matrix cores: features,
 * weights and both hidden activations rounded to bfloat16 (nearest even),
 * products accumulated and biases added in FP32, 16 cells per MFMA tile;
 * the weights are repacked after every xdg_mlp_set / xdg_mlp_train.
 * Parameters: 9704 FP32 values, weights row-major [out][in]:
 *   W1[64][45] b1[64] W2[64][64] b2[64] W3[40][64] b3[40]. */
int32_t xdg_mlp_param_count(void);

/* Copies the parameters from the host and resets the Adam state. */
int xdg_mlp_set(xdg_handle *h, const float *params_host);

/* Copies the current parameters to the host (synchronises). */
int xdg_mlp_get(xdg_handle *h, float *params_host);

/* Y_dev[n][40] = MLP(X_dev[n][45]). */
int xdg_mlp_forward(xdg_handle *h, int32_t n, const float *X_dev, float *Y_dev);

/* grad_dev[9704] = d loss / d parameters and *loss_host = loss for
 * loss = sum_{s,o} (MLP(X)[s][o] - T[s][o])^2 / n (synchronises).  The sum
 * over samples is taken in a fixed order: results are reproducible. */
int xdg_mlp_gradient(xdg_handle *h, int32_t n, const float *X_dev, const float *T_dev,
                     float *grad_dev, float *loss_host);

/* `steps` Adam steps (Kingma and Ba; beta1 0.9, beta2 0.999, eps 1e-8, step
 * size lr) on the loss above over minibatches of `batch` samples: step k uses
 * samples [(k mod nb) * batch, +batch), nb = floor(n / batch); the caller
 * shuffles.  loss_hist_host[k] (NULL allowed) receives the minibatch loss
 * before step k.  The Adam step count runs on across calls until
 * xdg_mlp_set (synchronises). */
int xdg_mlp_train(xdg_handle *h, int32_t n, const float *X_dev, const float *T_dev,
                  int32_t batch, int32_t steps, float lr, float *loss_hist_host);

/* Level-0 cell data of the features (host arrays, copied):
 * row_species_host[n_rows] in {0 = A (phi < 0), 1 = B}, distinct within a
 * cell (1 or 2 rows per cell); cell_geom_host[n_cells][5] = volume fraction
 * of species A, mean unit interface normal (zero if uncut), log10 of the
 * diffusivity ratio mu_B / mu_A (zero if uncut). */
int xdg_set_cell_features(xdg_handle *h, const int32_t *row_species_host,
                          const float *cell_geom_host);

/* Training pairs from an iterate x_k of a plain solve of M x = b and the
 * converged solution xs (level-0 device vectors): with r = b - M x_k, for the
 * cells c = cell0 + i * cell_step (i = 0 .. *n_out - 1, 0 <= cell0 < n_cells,
 * cell_step >= 1), X_dev[i][45] = the features of r on cell c and
 * T_dev[i][40] = (xs - x_k - j_c) / s_c in the same slots (zero where
 * s_c = 0), scaled to norm `clip` where it is longer (clip = 0: no scaling).
 * X_dev, T_dev must hold ceil((n_cells - cell0) / cell_step) samples;
 * *n_out receives that count. */
int xdg_learned_pairs(xdg_handle *h, const double *b_dev, const double *xk_dev,
                      const double *xs_dev, int32_t cell0, int32_t cell_step, float clip,
                      float *X_dev, float *T_dev, int32_t *n_out);

/* Switches the smoother of an existing handle (same requirements as
 * xdg_options.smoother) and sets the per-cell guard (> 0, default 4). */
int xdg_set_smoother(xdg_handle *h, int32_t smoother, float guard);

/* Cells that kept the plain step and solver-level fallbacks since creation. */
int xdg_learned_stats(xdg_handle *h, int64_t *guarded_cells, int32_t *fallbacks);

void xdg_destroy(xdg_handle *h);

const char *xdg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* XDG_H */
