// Plain-loop FP64 multigrid-preconditioned CG on the host (C++17, OpenMP) --
// TEST INFRASTRUCTURE ONLY: the timed CPU baseline of the solve and a second
// oracle of it.  Written from the definitions, independent of the GPU library
// (no shared source, header, layout or helper):
//   * the level matrices are scalar CSR matrices, the level-0 one expanded from
//     its blocks M[m(i,r), m(col,c)] (Eq. GenericMatrixSystem);
//   * the transfer R^{X,lambda} is a scalar CSR matrix holding the coarse basis
//     in fine coefficients (Eq. XDGrestrictionMatrix): [I; 0] per block row for
//     a p-level, the block R_i at (i, parent(i)) for an aggregation level;
//   * coarse levels are the Galerkin products R^T (M R) (Eq. XDGsysRestriction)
//     by a generic sparse-times-sparse product;
//   * the smoother blocks D_c = M[I_c, I_c] (all modes of all species of one
//     cell block, the per-cell solves of Section 3.3) are inverted explicitly
//     through a Cholesky factorisation (solving L L^T X = I);
//   * the coarsest matrix is factorised by dense Cholesky and solved by
//     forward and back substitution (the low-order direct solve);
//   * the V-cycle, damped block Jacobi and PCG are the textbook recursions.
// Every loop over rows is split statically over OpenMP threads; inner products
// add per-thread partials in thread order, so a run is reproducible for a
// fixed thread count.
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <vector>

namespace {

struct Csr {
    int64_t n_rows = 0, n_cols = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> val;
};

// y = M x
void spmv(const Csr& M, const double* x, double* y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M.n_rows; ++i) {
        double s = 0.0;
        for (int64_t k = M.ptr[i]; k < M.ptr[i + 1]; ++k) s += M.val[k] * x[M.col[k]];
        y[i] = s;
    }
}

Csr transpose(const Csr& M) {
    Csr T;
    T.n_rows = M.n_cols;
    T.n_cols = M.n_rows;
    T.ptr.assign(T.n_rows + 1, 0);
    for (int64_t k = 0; k < M.ptr[M.n_rows]; ++k) T.ptr[M.col[k] + 1]++;
    for (int64_t i = 0; i < T.n_rows; ++i) T.ptr[i + 1] += T.ptr[i];
    T.col.resize(M.ptr[M.n_rows]);
    T.val.resize(M.ptr[M.n_rows]);
    std::vector<int64_t> fill(T.ptr.begin(), T.ptr.end() - 1);
    for (int64_t i = 0; i < M.n_rows; ++i)          // ascending rows: sorted columns of T
        for (int64_t k = M.ptr[i]; k < M.ptr[i + 1]; ++k) {
            const int64_t d = fill[M.col[k]]++;
            T.col[d] = (int32_t)i;
            T.val[d] = M.val[k];
        }
    return T;
}

// C = A B (rows of C: columns in ascending order; the products of one entry
// are added in the order of A's row, then B's row)
Csr multiply(const Csr& A, const Csr& B) {
    Csr C;
    C.n_rows = A.n_rows;
    C.n_cols = B.n_cols;
    std::vector<std::vector<int32_t>> rcol(A.n_rows);
    std::vector<std::vector<double>> rval(A.n_rows);
#pragma omp parallel
    {
        std::vector<double> acc(B.n_cols, 0.0);
        std::vector<char> used(B.n_cols, 0);
        std::vector<int32_t> cols;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < A.n_rows; ++i) {
            cols.clear();
            for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                const double a = A.val[k];
                const int32_t r = A.col[k];
                for (int64_t q = B.ptr[r]; q < B.ptr[r + 1]; ++q) {
                    const int32_t j = B.col[q];
                    if (!used[j]) {
                        used[j] = 1;
                        cols.push_back(j);
                    }
                    acc[j] += a * B.val[q];
                }
            }
            std::sort(cols.begin(), cols.end());
            rcol[i] = cols;
            rval[i].resize(cols.size());
            for (size_t t = 0; t < cols.size(); ++t) {
                rval[i][t] = acc[cols[t]];
                acc[cols[t]] = 0.0;
                used[cols[t]] = 0;
            }
        }
    }
    C.ptr.assign(C.n_rows + 1, 0);
    for (int64_t i = 0; i < C.n_rows; ++i) C.ptr[i + 1] = C.ptr[i] + (int64_t)rcol[i].size();
    C.col.resize(C.ptr[C.n_rows]);
    C.val.resize(C.ptr[C.n_rows]);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < C.n_rows; ++i) {
        std::copy(rcol[i].begin(), rcol[i].end(), C.col.begin() + C.ptr[i]);
        std::copy(rval[i].begin(), rval[i].end(), C.val.begin() + C.ptr[i]);
    }
    return C;
}

// lower Cholesky factor of the dense SPD matrix a (n x n, row-major, in place:
// the lower triangle receives L); false on a non-positive pivot
bool cholesky(double* a, int64_t n) {
    for (int64_t k = 0; k < n; ++k) {
        double d = a[k * n + k];
        for (int64_t p = 0; p < k; ++p) d -= a[k * n + p] * a[k * n + p];
        if (!(d > 0.0)) return false;
        const double lkk = std::sqrt(d);
        a[k * n + k] = lkk;
#pragma omp parallel for schedule(static) if (n - k > 256)
        for (int64_t i = k + 1; i < n; ++i) {
            double s = a[i * n + k];
            for (int64_t p = 0; p < k; ++p) s -= a[i * n + p] * a[k * n + p];
            a[i * n + k] = s / lkk;
        }
    }
    return true;
}

// x = (L L^T)^{-1} b with the lower factor L and its transpose U = L^T
// (both row-major, n x n): forward substitution with L, back substitution
// with U (row access in both)
void cholesky_solve(const double* L, const double* U, int64_t n, const double* b, double* x) {
    for (int64_t i = 0; i < n; ++i) {
        double s = b[i];
        for (int64_t p = 0; p < i; ++p) s -= L[i * n + p] * x[p];
        x[i] = s / L[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int64_t p = i + 1; p < n; ++p) s -= U[i * n + p] * x[p];
        x[i] = s / U[i * n + i];
    }
}

// U = L^T (n x n row-major)
std::vector<double> transposed(const double* L, int64_t n) {
    std::vector<double> U(n * n, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) U[j * n + i] = L[i * n + j];
    return U;
}

struct Level {
    Csr A;                          // level matrix
    Csr R, Rt;                      // transfer to the next coarser level
    int64_t n_blocks = 0;           // block rows
    int np = 0;
    std::vector<int32_t> cell_ptr;  // block rows of every smoother cell block
    std::vector<int64_t> doff;      // offsets of the dense inverses
    std::vector<double> dinv;       // explicit cell-block inverses, row-major
    std::vector<double> b, x, y, r; // work vectors
};

}  // namespace

struct mgo_handle {
    std::vector<Level> L;
    std::vector<double> coarse_L;   // dense Cholesky factor of the coarsest matrix
    std::vector<double> coarse_U;   // its transpose
    int64_t coarse_n = 0;
    double omega = 0.7;
    int nu_pre = 2, nu_post = 2;
    int nu_coarse = 0;              // > 0: sweeps on every level below the finest
    std::vector<double> partial;    // per-thread partial sums of inner products
};

namespace {

double dot(mgo_handle* h, int64_t n, const double* a, const double* b) {
    const int nt = omp_get_max_threads();
    h->partial.assign(nt, 0.0);
#pragma omp parallel num_threads(nt)
    {
        const int t = omp_get_thread_num();
        const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i) s += a[i] * b[i];
        h->partial[t] = s;
    }
    double s = 0.0;
    for (int t = 0; t < nt; ++t) s += h->partial[t];
    return s;
}

// x <- x + omega D^{-1} (b - A x), `sweeps` times (damped block Jacobi)
void jacobi(mgo_handle* h, Level& lv, const double* b, double* x, int sweeps) {
    const int64_t n = lv.A.n_rows;
    const int64_t nc = (int64_t)lv.cell_ptr.size() - 1;
    for (int s = 0; s < sweeps; ++s) {
        spmv(lv.A, x, lv.y.data());
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) lv.r[i] = b[i] - lv.y[i];
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nc; ++c) {
            const int64_t lo = (int64_t)lv.cell_ptr[c] * lv.np, hi = (int64_t)lv.cell_ptr[c + 1] * lv.np;
            const int64_t m = hi - lo;
            const double* D = lv.dinv.data() + lv.doff[c];
            for (int64_t i = 0; i < m; ++i) {
                double t = 0.0;
                for (int64_t j = 0; j < m; ++j) t += D[i * m + j] * lv.r[lo + j];
                x[lo + i] += h->omega * t;
            }
        }
    }
}

// z = B r on level l (recursive V-cycle); r and z are level vectors
void vcycle(mgo_handle* h, int l, const double* r, double* z) {
    Level& lv = h->L[l];
    const int64_t n = lv.A.n_rows;
    if (l == (int)h->L.size() - 1) {
        cholesky_solve(h->coarse_L.data(), h->coarse_U.data(), h->coarse_n, r, z);
        return;
    }
    Level& cl = h->L[l + 1];
    const bool coarse = l > 0 && h->nu_coarse > 0;
    std::fill(z, z + n, 0.0);
    jacobi(h, lv, r, z, coarse ? h->nu_coarse : h->nu_pre);
    spmv(lv.A, z, lv.y.data());
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) lv.r[i] = r[i] - lv.y[i];
    spmv(lv.Rt, lv.r.data(), cl.b.data());
    vcycle(h, l + 1, cl.b.data(), cl.x.data());
    spmv(lv.R, cl.x.data(), lv.y.data());
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) z[i] += lv.y[i];
    jacobi(h, lv, r, z, coarse ? h->nu_coarse : h->nu_post);
}

}  // namespace

extern "C" {

int mgo_threads(void) { return omp_get_max_threads(); }

void mgo_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
}

// sweeps before and after the coarse correction on the levels below the
// finest (0: the finest level's counts)
void mgo_set_coarse_sweeps(mgo_handle* h, int32_t nu_coarse) { h->nu_coarse = nu_coarse; }

// Level-0 block matrix (val row-major per block) and its smoother cells.
mgo_handle* mgo_new(int32_t n_rows, int32_t np, int32_t nnzb, const int32_t* row_ptr,
                    const int32_t* col_idx, const double* val, int32_t n_cells,
                    const int32_t* cell_ptr, double omega, int32_t nu_pre, int32_t nu_post) {
    auto* h = new mgo_handle();
    h->omega = omega;
    h->nu_pre = nu_pre;
    h->nu_post = nu_post;
    h->L.resize(1);
    Level& lv = h->L[0];
    lv.np = np;
    lv.n_blocks = n_rows;
    Csr& A = lv.A;
    A.n_rows = A.n_cols = (int64_t)n_rows * np;
    A.ptr.assign(A.n_rows + 1, 0);
    for (int32_t i = 0; i < n_rows; ++i)
        for (int r = 0; r < np; ++r)
            A.ptr[(int64_t)i * np + r + 1] = (int64_t)(row_ptr[i + 1] - row_ptr[i]) * np;
    for (int64_t i = 0; i < A.n_rows; ++i) A.ptr[i + 1] += A.ptr[i];
    A.col.resize(A.ptr[A.n_rows]);
    A.val.resize(A.ptr[A.n_rows]);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n_rows; ++i)
        for (int r = 0; r < np; ++r) {
            int64_t d = A.ptr[(int64_t)i * np + r];
            for (int32_t b = row_ptr[i]; b < row_ptr[i + 1]; ++b)
                for (int c = 0; c < np; ++c) {
                    A.col[d] = col_idx[b] * np + c;
                    A.val[d++] = val[(int64_t)b * np * np + (int64_t)r * np + c];
                }
        }
    (void)nnzb;
    lv.cell_ptr.assign(cell_ptr, cell_ptr + n_cells + 1);
    return h;
}

// Transfer from the current coarsest level to a new one.
void mgo_add_transfer(mgo_handle* h, int32_t kind, int32_t n_rows_c, int32_t np_c,
                      const int32_t* parent, const double* R, int32_t n_cells_c,
                      const int32_t* cell_ptr_c) {
    Level& f = h->L.back();
    const int64_t nf = f.n_blocks;
    Csr& T = f.R;
    T.n_rows = nf * f.np;
    T.n_cols = (int64_t)n_rows_c * np_c;
    T.ptr.assign(T.n_rows + 1, 0);
    for (int64_t i = 0; i < nf; ++i)
        for (int a = 0; a < f.np; ++a) {
            const int64_t row = i * f.np + a;
            if (kind == 0) {                       // p-level: [I; 0]
                if (a < np_c) {
                    T.col.push_back((int32_t)(i * np_c + a));
                    T.val.push_back(1.0);
                }
            } else {                               // aggregation level: R_i at (i, parent(i))
                for (int m = 0; m < np_c; ++m) {
                    T.col.push_back(parent[i] * np_c + m);
                    T.val.push_back(R[(i * f.np + a) * np_c + m]);
                }
            }
            T.ptr[row + 1] = (int64_t)T.col.size();
        }
    f.Rt = transpose(f.R);
    Level c;
    c.np = np_c;
    c.n_blocks = n_rows_c;
    c.cell_ptr.assign(cell_ptr_c, cell_ptr_c + n_cells_c + 1);
    h->L.push_back(std::move(c));
}

// Galerkin levels, cell-block inverses, coarsest factor.  Returns 0, or -1 on
// a non-positive pivot.
int mgo_setup(mgo_handle* h) {
    const int nl = (int)h->L.size();
    for (int l = 0; l + 1 < nl; ++l) h->L[l + 1].A = multiply(h->L[l].Rt, multiply(h->L[l].A, h->L[l].R));
    int bad = 0;
    for (int l = 0; l + 1 < nl; ++l) {
        Level& lv = h->L[l];
        const int64_t nc = (int64_t)lv.cell_ptr.size() - 1;
        lv.doff.assign(nc + 1, 0);
        for (int64_t c = 0; c < nc; ++c) {
            const int64_t m = (int64_t)(lv.cell_ptr[c + 1] - lv.cell_ptr[c]) * lv.np;
            lv.doff[c + 1] = lv.doff[c] + m * m;
        }
        lv.dinv.assign(lv.doff[nc], 0.0);
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (int64_t c = 0; c < nc; ++c) {
            const int64_t lo = (int64_t)lv.cell_ptr[c] * lv.np, hi = (int64_t)lv.cell_ptr[c + 1] * lv.np;
            const int64_t m = hi - lo;
            std::vector<double> D(m * m, 0.0), e(m), col(m);
            for (int64_t i = lo; i < hi; ++i)
                for (int64_t k = lv.A.ptr[i]; k < lv.A.ptr[i + 1]; ++k) {
                    const int64_t j = lv.A.col[k];
                    if (j >= lo && j < hi) D[(i - lo) * m + (j - lo)] = lv.A.val[k];
                }
            if (!cholesky(D.data(), m)) {
                bad |= 1;
                continue;
            }
            double* out = lv.dinv.data() + lv.doff[c];
            const std::vector<double> U = transposed(D.data(), m);
            for (int64_t j = 0; j < m; ++j) {          // column j of D^{-1}
                std::fill(e.begin(), e.end(), 0.0);
                e[j] = 1.0;
                cholesky_solve(D.data(), U.data(), m, e.data(), col.data());
                for (int64_t i = 0; i < m; ++i) out[i * m + j] = col[i];
            }
        }
    }
    Level& lc = h->L[nl - 1];
    h->coarse_n = lc.A.n_rows;
    const int64_t n = h->coarse_n;
    h->coarse_L.assign(n * n, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = lc.A.ptr[i]; k < lc.A.ptr[i + 1]; ++k)
            h->coarse_L[i * n + lc.A.col[k]] = lc.A.val[k];
    if (!cholesky(h->coarse_L.data(), n)) bad |= 1;
    h->coarse_U = transposed(h->coarse_L.data(), n);
    for (auto& lv : h->L) {
        const int64_t m = lv.A.n_rows;
        lv.b.assign(m, 0.0);
        lv.x.assign(m, 0.0);
        lv.y.assign(m, 0.0);
        lv.r.assign(m, 0.0);
    }
    return bad ? -1 : 0;
}

int32_t mgo_levels(mgo_handle* h) { return (int32_t)h->L.size(); }

int64_t mgo_level_size(mgo_handle* h, int32_t l) { return h->L[l].A.n_rows; }

int64_t mgo_level_nnz(mgo_handle* h, int32_t l) { return h->L[l].A.ptr[h->L[l].A.n_rows]; }

// scalar CSR of level l: ptr [n+1], col [nnz], val [nnz]
void mgo_level_csr(mgo_handle* h, int32_t l, int64_t* ptr, int32_t* col, double* val) {
    const Csr& A = h->L[l].A;
    std::memcpy(ptr, A.ptr.data(), (A.n_rows + 1) * sizeof(int64_t));
    std::memcpy(col, A.col.data(), A.col.size() * sizeof(int32_t));
    std::memcpy(val, A.val.data(), A.val.size() * sizeof(double));
}

void mgo_spmv(mgo_handle* h, int32_t l, const double* x, double* y) { spmv(h->L[l].A, x, y); }

void mgo_smooth(mgo_handle* h, int32_t l, const double* b, double* x, int32_t sweeps) {
    jacobi(h, h->L[l], b, x, sweeps);
}

void mgo_vcycle(mgo_handle* h, const double* r, double* z) { vcycle(h, 0, r, z); }

// Textbook PCG from x0 = x (in place) until ||r||/||b|| <= rtol or maxit.
// hist[k] = ||r_k||/||b|| for k = 0..iters (cap entries at most).  Returns
// the iteration count.
int32_t mgo_pcg(mgo_handle* h, const double* b, double* x, double rtol, int32_t maxit,
                double* hist, int32_t cap) {
    Level& lv = h->L[0];
    const int64_t n = lv.A.n_rows;
    std::vector<double> r(n), z(n), p(n), q(n);
    spmv(lv.A, x, q.data());
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    const double nb = std::sqrt(dot(h, n, b, b));
    double rel = std::sqrt(dot(h, n, r.data(), r.data())) / nb;
    if (cap > 0) hist[0] = rel;
    if (rel <= rtol) return 0;
    vcycle(h, 0, r.data(), z.data());
    p = z;
    double rz = dot(h, n, r.data(), z.data());
    for (int32_t k = 1; k <= maxit; ++k) {
        spmv(lv.A, p.data(), q.data());
        const double alpha = rz / dot(h, n, p.data(), q.data());
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        rel = std::sqrt(dot(h, n, r.data(), r.data())) / nb;
        if (k < cap) hist[k] = rel;
        if (rel <= rtol) return k;
        vcycle(h, 0, r.data(), z.data());
        const double rz_new = dot(h, n, r.data(), z.data());
        const double beta = rz_new / rz;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rz = rz_new;
    }
    return maxit;
}

void mgo_free(mgo_handle* h) { delete h; }

}  // extern "C"
