// C-ABI of libxdg: hierarchy construction and the solver loops (host side).
// Every arithmetic step runs in the kernels of k_level.hip / k_setup.hip /
// k_blas.hip; this file only validates input, does the integer bookkeeping of
// the sparsity patterns, and sequences launches on the handle's stream (the
// numeric set-up also on an internal side stream, joined back by an event
// before anything reads its results).
#include <numeric>

#include <mutex>
#include <unordered_map>

#include "xdg_handle.h"

using namespace xdg;

namespace xdg {
static thread_local std::string g_err_text;
int fail(int code, const std::string& msg) {
    g_err_text = msg;
    return code;
}
const std::string& last_error_text() { return g_err_text; }
}  // namespace xdg

// ---------------------------------------------------------------------------
// validation

static int check_pattern(int n_rows, int nnzb, const int32_t* rp, const int32_t* ci,
                         const char* what) {
    if (!rp || !ci) return fail(XDG_EINVAL, std::string(what) + ": NULL row_ptr/col_idx");
    if (rp[0] != 0 || rp[n_rows] != nnzb)
        return fail(XDG_EINVAL, std::string(what) + ": row_ptr does not span [0, nnzb]");
    for (int i = 0; i < n_rows; ++i) {
        if (rp[i + 1] <= rp[i]) return fail(XDG_EINVAL, std::string(what) + ": empty block row");
        bool diag = false;
        for (int b = rp[i]; b < rp[i + 1]; ++b) {
            if (ci[b] < 0 || ci[b] >= n_rows)
                return fail(XDG_EINVAL, std::string(what) + ": column index out of range");
            if (b > rp[i] && ci[b] <= ci[b - 1])
                return fail(XDG_EINVAL, std::string(what) + ": columns not strictly sorted");
            diag |= ci[b] == i;
        }
        if (!diag) return fail(XDG_EINVAL, std::string(what) + ": missing diagonal block");
    }
    return XDG_OK;
}

static int check_cells(int n_rows, int np, int n_cells, const int32_t* cp, const char* what) {
    if (n_cells < 1 || !cp) return fail(XDG_EINVAL, std::string(what) + ": no cell blocks");
    if (cp[0] != 0 || cp[n_cells] != n_rows)
        return fail(XDG_EINVAL, std::string(what) + ": cell_ptr does not span the rows");
    for (int c = 0; c < n_cells; ++c) {
        if (cp[c + 1] <= cp[c]) return fail(XDG_EINVAL, std::string(what) + ": empty cell block");
        if ((int64_t)(cp[c + 1] - cp[c]) * np > kMaxCell)
            return fail(XDG_EINVAL, std::string(what) + ": cell block larger than " +
                                        std::to_string(kMaxCell));
    }
    return XDG_OK;
}

static bool finite_all(const double* v, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

// ---------------------------------------------------------------------------
// set-up helpers

static int setup_cells(xdg_handle* h, Level& lv, const int32_t* cp, int n_cells) {
    lv.n_cells = n_cells;
    lv.h_cp.assign(cp, cp + n_cells + 1);
    lv.h_doff.resize(n_cells + 1);
    int64_t off = 0;
    lv.max_nc = 0;
    for (int c = 0; c < n_cells; ++c) {
        const int nc = (cp[c + 1] - cp[c]) * lv.np;
        lv.h_doff[c] = off;
        off += (int64_t)nc * nc;
        lv.max_nc = std::max(lv.max_nc, nc);
    }
    lv.h_doff[n_cells] = off;
    lv.dsize = off;
    CHK(h->upload(&lv.cp, lv.h_cp.data(), lv.h_cp.size()));
    CHK(h->upload(&lv.doff, lv.h_doff.data(), lv.h_doff.size()));
    return XDG_OK;
}

static int setup_vectors(xdg_handle* h, Level& lv, bool mixed) {
    const int64_t n = lv.len();
    CHK(h->alloc(&lv.b64, n));
    CHK(h->alloc(&lv.x64, n));
    CHK(h->alloc(&lv.y64, n));
    CHK(h->alloc(&lv.r64, n));
    if (mixed) {
        CHK(h->alloc(&lv.b32, n));
        CHK(h->alloc(&lv.x32, n));
        CHK(h->alloc(&lv.y32, n));
        CHK(h->alloc(&lv.r32, n));
    }
    return XDG_OK;
}

// Galerkin level l -> l+1 for a dense transfer: the integer pattern and the
// list of fine blocks contributing to every coarse block (ascending fine-block
// order) are built once on the host; the products run in numeric_setup.
static int galerkin_symbolic(xdg_handle* h, Level& f, Level& c, const int32_t* parent) {
    const int nf = f.n_rows, ncr = c.n_rows;
    struct Item { int64_t key; int fb, i, l; };
    std::vector<Item> it;
    it.reserve(f.nnzb);
    for (int i = 0; i < nf; ++i)
        for (int b = f.h_rp[i]; b < f.h_rp[i + 1]; ++b) {
            const int l = f.h_ci[b];
            it.push_back({(int64_t)parent[i] * ncr + parent[l], b, i, l});
        }
    std::stable_sort(it.begin(), it.end(), [](const Item& a, const Item& b) { return a.key < b.key; });
    std::vector<int> cptr, cfb(it.size()), crow(it.size()), ccol(it.size());
    f.h_fb2cb.assign(f.nnzb, -1);
    c.h_rp.assign(ncr + 1, 0);
    c.h_ci.clear();
    for (size_t k = 0; k < it.size(); ++k) {
        if (k == 0 || it[k].key != it[k - 1].key) {
            cptr.push_back((int)k);
            const int row = (int)(it[k].key / ncr), col = (int)(it[k].key % ncr);
            c.h_ci.push_back(col);
            c.h_rp[row + 1]++;
        }
        cfb[k] = it[k].fb;
        f.h_fb2cb[it[k].fb] = (int)cptr.size() - 1;
        crow[k] = it[k].i;
        ccol[k] = it[k].l;
    }
    // the products index the table of distinct transfer blocks
    std::vector<int> rrow(it.size()), rcol(it.size());
    for (size_t k = 0; k < it.size(); ++k) {
        rrow[k] = f.h_ridx[crow[k]];
        rcol[k] = f.h_ridx[ccol[k]];
    }
    cptr.push_back((int)it.size());
    for (int i = 0; i < ncr; ++i) c.h_rp[i + 1] += c.h_rp[i];
    c.nnzb = (int)c.h_ci.size();
    CHK(check_pattern(ncr, c.nnzb, c.h_rp.data(), c.h_ci.data(), "coarse level"));
    CHK(h->upload(&c.rp, c.h_rp.data(), c.h_rp.size()));
    CHK(h->upload(&c.ci, c.h_ci.data(), c.h_ci.size()));
    CHK(h->upload(&f.g_ptr, cptr.data(), cptr.size()));
    CHK(h->upload(&f.g_fb, cfb.data(), cfb.size()));
    CHK(h->upload(&f.g_row, rrow.data(), rrow.size()));
    CHK(h->upload(&f.g_col, rcol.data(), rcol.size()));
    CHK(h->alloc(&c.A64, (size_t)c.nnzb * c.np * c.np));
    if (c.np * c.np > 32) {
        // fine-row groups inside every coarse block's contribution list
        std::vector<int> gstart, grow, cbg(c.nnzb + 1, 0);
        for (int cb = 0; cb < c.nnzb; ++cb) {
            cbg[cb] = (int)gstart.size();
            for (int k = cptr[cb]; k < cptr[cb + 1]; ++k)
                if (k == cptr[cb] || crow[k] != crow[k - 1]) {
                    gstart.push_back(k);
                    grow.push_back(rrow[k]);
                }
        }
        cbg[c.nnzb] = (int)gstart.size();
        f.n_grp = (int)gstart.size();
        gstart.push_back((int)it.size());
        CHK(h->upload(&f.g_gstart, gstart.data(), gstart.size()));
        CHK(h->upload(&f.g_grow, grow.data(), grow.size()));
        CHK(h->upload(&f.g_cbg, cbg.data(), cbg.size()));
        CHK(h->alloc(&f.g_U, (size_t)f.n_grp * f.np * c.np));
    }
    return XDG_OK;
}

// Pattern of (M R) for the post sweep after an aggregation coarse correction:
// per fine row the distinct parents of its columns (ascending), and for every
// such block the row's fine blocks that sum into it (ascending).
static int ar_symbolic(xdg_handle* h, Level& f, const int32_t* parent) {
    std::vector<int> arp(f.n_rows + 1, 0), arc, lptr(1, 0), lb;
    std::vector<std::pair<int, int>> jb;
    for (int i = 0; i < f.n_rows; ++i) {
        jb.clear();
        for (int b = f.h_rp[i]; b < f.h_rp[i + 1]; ++b) jb.push_back({parent[f.h_ci[b]], b});
        std::stable_sort(jb.begin(), jb.end(),
                         [](const std::pair<int, int>& a, const std::pair<int, int>& b) {
                             return a.first < b.first;
                         });
        for (size_t q = 0; q < jb.size(); ++q) {
            if (q == 0 || jb[q].first != jb[q - 1].first) {
                if (q) lptr.push_back((int)lb.size());
                arc.push_back(jb[q].first);
            }
            lb.push_back(jb[q].second);
        }
        if (!jb.empty()) lptr.push_back((int)lb.size());
        arp[i + 1] = (int)arc.size();
    }
    f.n_ar = (int)arc.size();
    CHK(h->upload(&f.arp, arp.data(), arp.size()));
    CHK(h->upload(&f.arc, arc.data(), arc.size()));
    CHK(h->upload(&f.ar_lptr, lptr.data(), lptr.size()));
    CHK(h->upload(&f.ar_lb, lb.data(), lb.size()));
    const size_t n = (size_t)f.n_ar * f.np * f.npc;
    if (h->mixed) CHK(h->alloc(&f.AR32, n));
    else CHK(h->alloc(&f.AR64, n));
    return XDG_OK;
}

// (M R) blocks of every level that has them, from the FP64 level matrices
static void ar_numeric(xdg_handle* h, hipStream_t s) {
    for (auto& f : h->L) {
        if (f.AR64)
            launch_ar_product<double>(s, f.n_ar, f.np, f.npc, f.ar_lptr, f.ar_lb, f.ci, f.ridx,
                                      f.A64, f.R64, f.AR64);
        if (f.AR32)
            launch_ar_product<float>(s, f.n_ar, f.np, f.npc, f.ar_lptr, f.ar_lb, f.ci, f.ridx,
                                     f.A64, f.R64, f.AR32);
    }
}

static int invert_cells(xdg_handle* h, Level& lv, hipStream_t s) {
    HIPCHK(hipMemsetAsync(lv.D64, 0, lv.dsize * sizeof(double), s));
    launch_gather_cells(s, lv.n_cells, lv.np, lv.cp, lv.rp, lv.ci, lv.A64, lv.doff, lv.D64,
                        nullptr);
    launch_gj_batched(s, lv.n_cells, lv.doff, lv.cp, lv.np, lv.max_nc, lv.D64, h->d_err,
                      nullptr);
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

static int invert_coarsest(xdg_handle* h, Level& lv) {
    const int nt = h->cld / kCoarseNB;
    HIPCHK(hipMemsetAsync(h->Cinv, 0, (size_t)h->cld * h->cld * sizeof(double), h->s));
    launch_bsr_to_dense(h->s, lv.n_rows, lv.np, lv.rp, lv.ci, lv.A64, h->cld, h->cld, h->Cinv);
    for (int K = 0; K < nt; ++K)
        launch_coarse_gj_step(h->s, nt, K, h->cld, h->Cinv, h->Pbuf, h->d_err);
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

// the level's derived FP64 copies from its full FP64 blocks: the symmetric
// level's upper blocks and the leading columns (FP32 ones: convert_level32)
static void sym_refresh(Level& lv, hipStream_t s) {
    if (lv.sym)
        launch_gather_blocks<double, double>(s, lv.nnzb_u, lv.np * lv.np, lv.ufull, lv.A64,
                                             lv.As64);
    if (lv.AP64) launch_leading_columns<double>(s, lv.nnzb, lv.np, lv.npc, lv.A64, lv.AP64);
}

// FP32 copies of a level's operator and cell inverses (mixed precision)
static void convert_level32(Level& lv, hipStream_t s) {
    if (lv.sym)
        launch_gather_blocks<double, float>(s, lv.nnzb_u, lv.np * lv.np, lv.ufull, lv.A64,
                                            lv.As32);
    else
        launch_convert<double, float>(s, (int64_t)lv.nnzb * lv.np * lv.np, lv.A64, lv.A32);
    if (lv.AP32) launch_leading_columns<float>(s, lv.nnzb, lv.np, lv.npc, lv.A64, lv.AP32);
    launch_convert<double, float>(s, lv.dsize, lv.D64, lv.D32);
}

// Numeric phase of the set-up from level-0 values `raw` (device, row-major
// blocks): layout change, Galerkin chain, cell-block and coarsest inverses,
// FP32 copies.  Errors of the inversions are reported through d_err.
//
// The coarsest inverse (a chain of small launches) is the critical path, so
// the handle's stream runs only the Galerkin chain down to it and the
// inverse; when level 1 is a p-truncation its blocks are the leading corners
// of the caller's row-major blocks, and the chain starts at once.  The chain's
// products are latency-bound and slow down several times beside a streaming
// kernel, so the side stream starts once they are done: it changes level 0's
// layout (column-major blocks, symmetric upper blocks, leading columns),
// inverts the cell blocks of every level, forms the M R products and the FP32
// copies while the coarsest inverse runs.  Both streams are joined before
// anything reads the result.
static int numeric_setup(xdg_handle* h, const double* raw) {
    hipStream_t s = h->s, s2 = h->s2;
    const int nl = (int)h->L.size();
    HIPCHK(hipMemsetAsync(h->d_err, 0, sizeof(int), s));
    Level& L0 = h->L[0];
    const bool from_raw = nl > 1 && L0.t_kind == XDG_T_PTRUNC;
    if (!from_raw)                           // the chain (or the inverse) reads L0.A64
        launch_transpose_blocks<double>(s, L0.nnzb, L0.np, raw, L0.A64);
    for (int t = 0; t + 1 < nl; ++t) {
        Level& f = h->L[t];
        Level& c = h->L[t + 1];
        if (f.t_kind == XDG_T_PTRUNC)
            launch_extract_leading(s, f.nnzb, f.np, c.np, t == 0 ? raw : f.A64, c.A64, t == 0);
        else if (f.g_U)
            launch_galerkin_wide(s, f.n_grp, c.nnzb, f.np, c.np, f.g_gstart, f.g_grow, f.g_cbg,
                                 f.g_fb, f.g_col, f.A64, f.R64, f.g_U, c.A64);
        else
            launch_galerkin_dense(s, c.nnzb, f.np, c.np, f.g_ptr, f.g_fb, f.g_row, f.g_col,
                                  f.A64, f.R64, c.A64, nullptr);
    }
    HIPCHK(hipEventRecord(h->ev_fork, s));
    HIPCHK(hipStreamWaitEvent(s2, h->ev_fork, 0));
    if (from_raw) launch_transpose_blocks<double>(s2, L0.nnzb, L0.np, raw, L0.A64);
    sym_refresh(L0, s2);
    for (int l = 0; l + 1 < nl; ++l) CHK(invert_cells(h, h->L[l], s2));
    ar_numeric(h, s2);
    if (h->mixed)
        for (int l = 0; l + 1 < nl; ++l) convert_level32(h->L[l], s2);
    HIPCHK(hipEventRecord(h->ev_join, s2));
    CHK(invert_coarsest(h, h->L[nl - 1]));
    HIPCHK(hipStreamWaitEvent(s, h->ev_join, 0));
    if (h->nrhs == kNrhs) CHK(mrhs_numeric(h));
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

static int check_setup_error(xdg_handle* h) {
    int herr = 0;
    HIPCHK(hipMemcpyAsync(&herr, h->d_err, sizeof(int), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    if (herr) return fail(XDG_ENOTSPD, "non-positive pivot in a cell block or the coarsest "
                                       "matrix (not SPD)");
    return XDG_OK;
}

// ---------------------------------------------------------------------------
// Level operators on the level's storage

template <typename T>
void xdg::level_spmv(xdg_handle* h, Level& lv, int mode, const T* x, const T* b, T* y, int npc,
                     T* yfull) {
    const bool rev = lv.next_dir();
    if (lv.sym)
        launch_spmv_sym<T>(h->s, mode, lv.n_rows, P<T>::sym(lv), x, b, y, npc, rev, yfull);
    else
        launch_spmv<T>(h->s, mode, lv.n_rows, lv.np, lv.rp, lv.ci, P<T>::A(lv), x, b, y, npc,
                       rev, yfull);
}
template void xdg::level_spmv<double>(xdg_handle*, Level&, int, const double*, const double*,
                                      double*, int, double*);
template void xdg::level_spmv<float>(xdg_handle*, Level&, int, const float*, const float*,
                                     float*, int, float*);

void xdg::level_spmv_dot(xdg_handle* h, Level& lv, const double* x, double* y, double* out) {
    const bool rev = lv.next_dir();
    const bool fits = (int64_t)(lv.n_rows + 1) / 2 <= (int64_t)kPartDoubles;
    if (fits && lv.sym) {
        launch_spmv_dot_sym(h->s, lv.n_rows, P<double>::sym(lv), x, y, h->part, out, rev);
        return;
    }
    if (fits && launch_spmv_dot(h->s, lv.n_rows, lv.np, lv.rp, lv.ci, lv.A64, x, y, h->part,
                                out, rev))
        return;
    if (lv.sym)
        launch_spmv_sym<double>(h->s, SPMV_AX, lv.n_rows, P<double>::sym(lv), x, nullptr, y, 0,
                                rev);
    else
        launch_spmv<double>(h->s, SPMV_AX, lv.n_rows, lv.np, lv.rp, lv.ci, lv.A64, x, nullptr, y,
                            0, rev);
    launch_dot(h->s, lv.len(), x, y, h->part, out);
}

template <typename T>
void xdg::level_jacobi(xdg_handle* h, Level& lv, bool first, const T* b, const T* xin,
                       T* xout) {
    const bool rev = lv.next_dir();
    const T om = (T)h->opt.omega;
    if (lv.sym && !first)
        launch_jacobi_sym<T>(h->s, lv.n_cells, lv.cp, P<T>::sym(lv), lv.doff, P<T>::D(lv), b, xin,
                             xout, om, rev);
    else
        launch_jacobi<T>(h->s, first, lv.n_cells, lv.np, lv.cp, lv.rp, lv.ci, P<T>::A(lv),
                         lv.doff, P<T>::D(lv), b, xin, xout, om, rev);
}
template void xdg::level_jacobi<double>(xdg_handle*, Level&, bool, const double*, const double*,
                                        double*);
template void xdg::level_jacobi<float>(xdg_handle*, Level&, bool, const float*, const float*,
                                       float*);

// ---------------------------------------------------------------------------
// V-cycle (templated on the storage precision of levels above the coarsest)

template <typename T>
static void smooth_from_zero(xdg_handle* h, Level& lv, int sweeps) {
    T* b = P<T>::b(lv);
    T*& x = P<T>::x(lv);
    T*& y = P<T>::y(lv);
    if (sweeps <= 0) {
        launch_fill_zero<T>(h->s, lv.len(), x);
        return;
    }
    xdg::level_jacobi<T>(h, lv, true, b, nullptr, x);
    for (int k = 1; k < sweeps; ++k) {
        xdg::level_jacobi<T>(h, lv, false, b, x, y);
        std::swap(x, y);
    }
}

void xdg::smooth_from_zero_fp64(xdg_handle* h, Level& lv, int sweeps) {
    smooth_from_zero<double>(h, lv, sweeps);
}

// out != nullptr: the last sweep writes there instead (x keeps the previous
// iterate)
template <typename T>
static void smooth_more(xdg_handle* h, Level& lv, int sweeps, T* out = nullptr) {
    T* b = P<T>::b(lv);
    T*& x = P<T>::x(lv);
    T*& y = P<T>::y(lv);
    for (int k = 0; k < sweeps; ++k) {
        if (out && k == sweeps - 1) {
            xdg::level_jacobi<T>(h, lv, false, b, x, out);
            return;
        }
        xdg::level_jacobi<T>(h, lv, false, b, x, y);
        std::swap(x, y);
    }
    if (out) (void)hipMemcpyAsync(out, x, lv.len() * sizeof(T), hipMemcpyDeviceToDevice, h->s);
}

template <typename T>
static void coarse_solve(xdg_handle* h, Level& lv);

template <>
void coarse_solve<double>(xdg_handle* h, Level& lv) {
    launch_coarse_gemv(h->s, h->cn, h->cld, h->Cinv, lv.b64, lv.x64);
}
template <>
void coarse_solve<float>(xdg_handle* h, Level& lv) {
    launch_convert<float, double>(h->s, lv.len(), lv.b32, lv.b64);
    launch_coarse_gemv(h->s, h->cn, h->cld, h->Cinv, lv.b64, lv.x64);
    launch_convert<double, float>(h->s, lv.len(), lv.x64, lv.x32);
}

// input: P<T>::b(L[l]); output: P<T>::x(L[l]), or `out` when given
template <typename T>
static void vcycle(xdg_handle* h, int l, T* out = nullptr) {
    Level& f = h->L[l];
    if (l == (int)h->L.size() - 1) {
        coarse_solve<T>(h, f);
        if (out)
            (void)hipMemcpyAsync(out, P<T>::x(f), f.len() * sizeof(T), hipMemcpyDeviceToDevice,
                                 h->s);
        return;
    }
    Level& c = h->L[l + 1];
    bool learned = false;
    if constexpr (std::is_same<T, double>::value) learned = l == 0 && xdg::learned_active(h);
    bool x1_done = false;
    if constexpr (std::is_same<T, double>::value) {
        x1_done = l == 0 && h->x1_ready;
        if (l == 0) h->x1_ready = false;
    }
    const int nu_pre = xdg::sweeps_pre(h, l), nu_post = xdg::sweeps_post(h, l);
    if (learned) {
        xdg::learned_first_sweep(h, f);
        smooth_more<T>(h, f, nu_pre - 1);
    } else if (x1_done) {
        f.next_dir();                    // the fused sweep counts as the pass
        smooth_more<T>(h, f, nu_pre - 1);
    } else {
        smooth_from_zero<T>(h, f, nu_pre);
    }
    // first post sweep from the kept residual and the coarse correction
    // (M P from the leading columns, or M R for an aggregation), where the
    // level stores them
    const bool cc = f.t_kind == XDG_T_PTRUNC && P<T>::AP(f) && nu_post >= 1;
    const bool ccd = f.t_kind == XDG_T_DENSE && P<T>::AR(f) && nu_post >= 1;
    if (f.t_kind == XDG_T_PTRUNC) {
        xdg::level_spmv<T>(h, f, SPMV_RESID_TRUNC, P<T>::x(f), P<T>::b(f), P<T>::b(c), c.np,
                           cc ? P<T>::r(f) : nullptr);
    } else {
        xdg::level_spmv<T>(h, f, SPMV_RESID, P<T>::x(f), P<T>::b(f), P<T>::r(f), 0);
        launch_restrict_dense<T>(h->s, c.n_rows, f.n_rows, f.np, c.np, f.chp, f.chi, f.ridx,
                                 P<T>::R(f), P<T>::r(f), P<T>::b(c), P<T>::y(f));
    }
    vcycle<T>(h, l + 1);
    if (cc || ccd) {
        T*& x = P<T>::x(f);
        T*& y = P<T>::y(f);
        const bool last = nu_post == 1;
        T* dst = last && out ? out : y;
        if (cc)
            launch_jacobi_cc<T>(h->s, f.n_cells, f.np, c.np, f.cp, f.rp, f.ci, P<T>::AP(f),
                                f.doff, P<T>::D(f), P<T>::r(f), x, P<T>::x(c), dst,
                                (T)h->opt.omega, f.next_dir());
        else
            launch_jacobi_cc_g<T>(h->s, f.n_cells, f.np, c.np, f.cp, f.arp, f.arc, P<T>::AR(f),
                                  f.doff, P<T>::D(f), P<T>::r(f), x, P<T>::x(c), f.parent,
                                  f.ridx, P<T>::R(f), dst, (T)h->opt.omega);
        if (last && out) return;
        std::swap(x, y);
        smooth_more<T>(h, f, nu_post - 1, out);
        return;
    }
    if (f.t_kind == XDG_T_PTRUNC)
        launch_prolong_trunc<T>(h->s, f.n_rows, f.np, c.np, P<T>::x(c), P<T>::x(f));
    else
        launch_prolong_dense<T>(h->s, f.n_rows, f.np, c.np, f.parent, f.ridx, P<T>::R(f), P<T>::x(c),
                                P<T>::x(f));
    smooth_more<T>(h, f, nu_post, out);
}

// every public call starts its streaming passes in ascending order (and with
// no first sweep carried over from an earlier solve)
static void reset_dirs(xdg_handle* h) {
    for (auto& lv : h->L) lv.rev_next = false;
    h->x1_ready = false;
}

// z = B r for FP64 vectors, using the handle's precision for the cycle
static int apply_precond(xdg_handle* h, const double* r, double* z) {
    Level& f = h->L[0];
    const int64_t n = f.len();
    if (h->mixed) {
        launch_convert<double, float>(h->s, n, r, f.b32);
        vcycle<float>(h, 0);
        launch_convert<float, double>(h->s, n, f.x32, z);
    } else if (r == z) {
        HIPCHK(hipMemcpyAsync(f.b64, r, n * sizeof(double), hipMemcpyDeviceToDevice, h->s));
        vcycle<double>(h, 0);
        HIPCHK(hipMemcpyAsync(z, f.x64, n * sizeof(double), hipMemcpyDeviceToDevice, h->s));
    } else {
        // the cycle reads level 0's right-hand side from r (only read there)
        // and its last sweep writes z
        double* own_b = f.b64;
        f.b64 = const_cast<double*>(r);
        vcycle<double>(h, 0, z);
        f.b64 = own_b;
    }
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

// ---------------------------------------------------------------------------
// V-cycle without allocation: the level work vectors live in a fixed device
// array.  Device code names it; host code uses only its device address,
// looked up once per device when a handle is created there.

namespace {
constexpr int64_t kScratchDoubles = int64_t(1) << 22;   // 32 MiB per device
constexpr int kMaxDevices = 64;
__device__ __align__(256) double scratch[kScratchDoubles];
double* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

int scratch_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(XDG_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return XDG_OK;
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(XDG_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch[dev] = static_cast<double*>(p);
    return XDG_OK;
}

// the work vectors of one level that the V-cycle touches
struct CyclePtrs {
    double *b64 = nullptr, *x64 = nullptr, *y64 = nullptr, *r64 = nullptr;
    float *b32 = nullptr, *x32 = nullptr, *y32 = nullptr, *r32 = nullptr;
};
constexpr int kMaxCycleLevels = 32;

// Lays the V-cycle's work vectors out in 256-byte aligned pieces from base
// (base = nullptr: only counts) and returns the doubles used.  Every level
// holds b, x, y and, above a dense transfer or where the first post sweep
// uses the kept residual, r in the cycle's precision; the
// coarsest level holds b, x (and b64, x64 for the FP32 cycle's FP64 solve).
int64_t carve_cycle(const xdg_handle* h, double* base, CyclePtrs* out) {
    int64_t used = 0;
    auto take = [&](int64_t n, int64_t word) -> char* {
        char* p = base ? reinterpret_cast<char*>(base + used) : nullptr;
        used += ((n * word + 255) / 256) * 32;
        return p;
    };
    const int nl = (int)h->L.size();
    for (int l = 0; l < nl; ++l) {
        const Level& lv = h->L[l];
        const int64_t n = lv.len();
        const bool last = l == nl - 1;
        CyclePtrs c;
        if (h->mixed) {
            c.b32 = reinterpret_cast<float*>(take(n, 4));
            c.x32 = reinterpret_cast<float*>(take(n, 4));
            if (!last) c.y32 = reinterpret_cast<float*>(take(n, 4));
            if (!last && (lv.t_kind == XDG_T_DENSE || lv.AP32))
                c.r32 = reinterpret_cast<float*>(take(n, 4));
            if (last) {
                c.b64 = reinterpret_cast<double*>(take(n, 8));
                c.x64 = reinterpret_cast<double*>(take(n, 8));
            }
        } else {
            c.b64 = reinterpret_cast<double*>(take(n, 8));
            c.x64 = reinterpret_cast<double*>(take(n, 8));
            if (!last) c.y64 = reinterpret_cast<double*>(take(n, 8));
            if (!last && (lv.t_kind == XDG_T_DENSE || lv.AP64))
                c.r64 = reinterpret_cast<double*>(take(n, 8));
        }
        if (out) out[l] = c;
    }
    return used;
}

void swap_cycle_ptrs(Level& lv, CyclePtrs& c) {
    std::swap(lv.b64, c.b64);
    std::swap(lv.x64, c.x64);
    std::swap(lv.y64, c.y64);
    std::swap(lv.r64, c.r64);
    std::swap(lv.b32, c.b32);
    std::swap(lv.x32, c.x32);
    std::swap(lv.y32, c.y32);
    std::swap(lv.r32, c.r32);
}
}  // namespace

extern "C" int xdg_vcycle_noalloc(xdg_handle* h, const double* r, double* z) {
    if (!h || !r || !z) return fail(XDG_EINVAL, "xdg_vcycle_noalloc: NULL argument");
    if (h->nrhs != 1 || h->opt.smoother != XDG_JACOBI)
        return fail(XDG_EINVAL, "xdg_vcycle_noalloc: single-column handles with the block-Jacobi "
                                "smoother only");
    if ((int)h->L.size() > kMaxCycleLevels)
        return fail(XDG_EINVAL, "xdg_vcycle_noalloc: more than 32 levels");
    if (h->dev < 0 || h->dev >= kMaxDevices || !g_scratch[h->dev])
        return fail(XDG_EINVAL, "xdg_vcycle_noalloc: no scratch address for the handle's device");
    const int64_t need = carve_cycle(h, nullptr, nullptr);
    if (need > kScratchDoubles)
        return fail(XDG_EINVAL, "xdg_vcycle_noalloc: the cycle needs " + std::to_string(need) +
                                    " doubles of work space, the fixed array holds " +
                                    std::to_string(kScratchDoubles));
    CyclePtrs ptrs[kMaxCycleLevels];
    carve_cycle(h, g_scratch[h->dev], ptrs);
    const int nl = (int)h->L.size();
    for (int l = 0; l < nl; ++l) swap_cycle_ptrs(h->L[l], ptrs[l]);     // scratch in
    reset_dirs(h);
    const int rc = apply_precond(h, r, z);
    for (int l = 0; l < nl; ++l) swap_cycle_ptrs(h->L[l], ptrs[l]);     // handle's back
    return rc;
}

// ---------------------------------------------------------------------------
// public API

extern "C" const char* xdg_last_error(void) { return xdg::last_error_text().c_str(); }

extern "C" void xdg_destroy(xdg_handle* h) {
    if (!h) return;
    if (h->s) (void)hipStreamSynchronize(h->s);
    if (h->s2) {
        (void)hipStreamSynchronize(h->s2);
        (void)hipStreamDestroy(h->s2);
    }
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    if (h->ev_scal) (void)hipEventDestroy(h->ev_scal);
    for (void* p : h->allocs) (void)hipFree(p);
    if (h->h_scal) (void)hipHostFree(h->h_scal);
    if (h->h_stage) (void)hipHostFree(h->h_stage);
    delete h;
}

// Row lists of the symmetric storage (SymRows): the upper blocks of every
// row (their indices among all blocks in ufull) and, for every lower block
// (i, j), the index of the stored (j, i).  False if some (i, j) has no (j, i).
// Every row holds its diagonal block (checked before).
struct SymLists {
    std::vector<int> urp, uci, ufull, lrp, lci, lidx;
};
static bool sym_lists(int n, const int32_t* rp, const int32_t* ci, SymLists& o) {
    o.urp.assign(n + 1, 0);
    o.lrp.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        for (int b = rp[i]; b < rp[i + 1]; ++b)
            if (ci[b] >= i) {
                o.uci.push_back(ci[b]);
                o.ufull.push_back(b);
            }
        o.urp[i + 1] = (int)o.uci.size();
    }
    for (int i = 0; i < n; ++i) {
        for (int b = rp[i]; b < rp[i + 1]; ++b) {
            const int j = ci[b];
            if (j >= i) continue;
            const auto first = o.uci.begin() + o.urp[j], last = o.uci.begin() + o.urp[j + 1];
            const auto it = std::lower_bound(first, last, i);     // columns sorted per row
            if (it == last || *it != i) return false;
            o.lci.push_back(j);
            o.lidx.push_back((int)(it - o.uci.begin()));
        }
        o.lrp[i + 1] = (int)o.lci.size();
    }
    // every lower block has its distinct stored mirror; the counts match only
    // if every off-diagonal upper block (one diagonal block per row) has one too
    return o.lci.size() + (size_t)n == o.uci.size();
}

static int create_impl(xdg_handle* h, const xdg_matrix* A0, int32_t n_levels,
                       const xdg_transfer* T, const xdg_options* opt) {
    // -- validation -----------------------------------------------------
    if (!A0 || !opt || n_levels < 1 || (n_levels > 1 && !T))
        return fail(XDG_EINVAL, "xdg_create: NULL argument or n_levels < 1");
    if (A0->n_rows < 1 || A0->np < 1 || A0->np > 64 || A0->nnzb < A0->n_rows || !A0->val)
        return fail(XDG_EINVAL, "xdg_create: bad matrix sizes");
    CHK(check_pattern(A0->n_rows, A0->nnzb, A0->row_ptr, A0->col_idx, "level-0 matrix"));
    CHK(check_cells(A0->n_rows, A0->np, A0->n_cells, A0->cell_ptr, "level-0 cells"));
    if (!finite_all(A0->val, (size_t)A0->nnzb * A0->np * A0->np))
        return fail(XDG_EINVAL, "xdg_create: non-finite matrix entry");
    if (!(opt->omega > 0.0 && opt->omega < 2.0) || opt->nu_pre < 0 || opt->nu_post < 0 ||
        opt->maxit < 1 || !(opt->rtol > 0.0) || (opt->nrhs != 1 && opt->nrhs != kNrhs) ||
        (opt->krylov != XDG_CG && opt->krylov != XDG_FGMRES && opt->krylov != XDG_ORTHOMG) ||
        (opt->precision != XDG_FP64 && opt->precision != XDG_MIXED))
        return fail(XDG_EINVAL, "xdg_create: invalid options");
    CHK(xdg::learned_validate(opt, A0->np));
    if (opt->krylov == XDG_FGMRES && (opt->restart < 1 || opt->restart > 64))
        return fail(XDG_EINVAL, "xdg_create: FGMRES restart must be in [1, 64]");
    if (opt->krylov == XDG_ORTHOMG &&
        (opt->restart < 3 || opt->restart > 64 || opt->precision != XDG_FP64 ||
         opt->nrhs != 1 || opt->smoother != XDG_JACOBI))
        return fail(XDG_EINVAL, "xdg_create: the orthonormalisation multigrid needs restart in "
                                "[3, 64], XDG_FP64, nrhs = 1 and block Jacobi");
    if (opt->krylov == XDG_CG && opt->nu_pre != opt->nu_post)
        return fail(XDG_EINVAL, "xdg_create: CG needs nu_pre == nu_post (symmetric V-cycle)");
    if (opt->nrhs == kNrhs) CHK(mrhs_validate(opt, A0->np, T, n_levels));
    if (opt->symmetric != 0 && opt->symmetric != 1)
        return fail(XDG_EINVAL, "xdg_create: symmetric must be 0 or 1");
    if (opt->nu_coarse < 0) return fail(XDG_EINVAL, "xdg_create: nu_coarse must be >= 0");
    SymLists sl;
    const bool use_sym = opt->symmetric == 1 && opt->nrhs == 1 && A0->np == kSymNp;
    if (use_sym && !sym_lists(A0->n_rows, A0->row_ptr, A0->col_idx, sl))
        return fail(XDG_EINVAL, "xdg_create: symmetric storage needs a symmetric block pattern "
                                "(a block (i, j) without (j, i)); set symmetric = 0");
    int nr = A0->n_rows, npf = A0->np;
    for (int t = 0; t < n_levels - 1; ++t) {
        const xdg_transfer& tr = T[t];
        const std::string w = "transfer " + std::to_string(t);
        if (tr.np_c < 1 || tr.np_c > 64 || tr.n_rows_c < 1)
            return fail(XDG_EINVAL, w + ": bad coarse sizes");
        if (tr.kind == XDG_T_PTRUNC) {
            if (tr.np_c > npf || tr.n_rows_c != nr)
                return fail(XDG_EINVAL, w + ": p-truncation needs np_c <= np_f, same rows");
        } else if (tr.kind == XDG_T_DENSE) {
            if (!tr.parent || !tr.R) return fail(XDG_EINVAL, w + ": NULL parent/R");
            if (tr.np_c > kMaxDenseCoarse)
                return fail(XDG_EINVAL, w + ": dense transfer with more than " +
                                            std::to_string(kMaxDenseCoarse) + " coarse modes");
            std::vector<int> cnt(tr.n_rows_c, 0);
            for (int i = 0; i < nr; ++i) {
                if (tr.parent[i] < 0 || tr.parent[i] >= tr.n_rows_c)
                    return fail(XDG_EINVAL, w + ": parent out of range");
                cnt[tr.parent[i]]++;
            }
            for (int c = 0; c < tr.n_rows_c; ++c)
                if (!cnt[c]) return fail(XDG_EINVAL, w + ": coarse row without children");
            if (!finite_all(tr.R, (size_t)nr * npf * tr.np_c))
                return fail(XDG_EINVAL, w + ": non-finite R");
        } else {
            return fail(XDG_EINVAL, w + ": unknown kind");
        }
        CHK(check_cells(tr.n_rows_c, tr.np_c, tr.n_cells_c, tr.cell_ptr_c,
                        (w + " coarse cells").c_str()));
        nr = tr.n_rows_c;
        npf = tr.np_c;
    }
    if ((int64_t)nr * npf > 16384)
        return fail(XDG_EINVAL, "xdg_create: coarsest level too large for the dense solve");

    // device work starts here (validation above touches no device)
    HIPCHK(hipGetDevice(&h->dev));
    CHK(scratch_setup(h->dev));
    h->opt = *opt;
    h->mixed = opt->precision == XDG_MIXED;
    h->nrhs = opt->nrhs;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // side stream of the set-up (default priority) and its fork / join events
    HIPCHK(hipStreamCreateWithFlags(&h->s2, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&h->ev_scal, hipEventDisableTiming));
    CHK(h->alloc(&h->d_err, 1));

    // -- symbolic phase: patterns, transfers, allocations ----------------------
    h->L.resize(n_levels);
    Level& L0 = h->L[0];
    L0.n_rows = A0->n_rows;
    L0.np = A0->np;
    L0.nnzb = A0->nnzb;
    L0.h_rp.assign(A0->row_ptr, A0->row_ptr + L0.n_rows + 1);
    L0.h_ci.assign(A0->col_idx, A0->col_idx + L0.nnzb);
    CHK(h->upload(&L0.rp, L0.h_rp.data(), L0.h_rp.size()));
    CHK(h->upload(&L0.ci, L0.h_ci.data(), L0.h_ci.size()));
    CHK(h->alloc(&L0.A64, (size_t)L0.nnzb * L0.np * L0.np));
    CHK(setup_cells(h, L0, A0->cell_ptr, A0->n_cells));
    if (use_sym) {
        L0.sym = true;
        L0.nnzb_u = (int64_t)sl.uci.size();
        CHK(h->upload(&L0.urp, sl.urp.data(), sl.urp.size()));
        CHK(h->upload(&L0.uci, sl.uci.data(), sl.uci.size()));
        CHK(h->upload(&L0.ufull, sl.ufull.data(), sl.ufull.size()));
        CHK(h->upload(&L0.lrp, sl.lrp.data(), sl.lrp.size()));
        CHK(h->upload(&L0.lci, sl.lci.data(), sl.lci.size()));
        CHK(h->upload(&L0.lidx, sl.lidx.data(), sl.lidx.size()));
        CHK(h->alloc(&L0.As64, (size_t)L0.nnzb_u * L0.np * L0.np));
        if (h->mixed) CHK(h->alloc(&L0.As32, (size_t)L0.nnzb_u * L0.np * L0.np));
    }
    for (int t = 0; t < n_levels - 1; ++t) {
        Level& f = h->L[t];
        Level& c = h->L[t + 1];
        const xdg_transfer& tr = T[t];
        f.t_kind = tr.kind;
        f.npc = tr.np_c;
        f.n_c = tr.n_rows_c;
        c.n_rows = tr.n_rows_c;
        c.np = tr.np_c;
        if (tr.kind == XDG_T_PTRUNC) {
            c.nnzb = f.nnzb;
            c.h_rp = f.h_rp;
            c.h_ci = f.h_ci;
            CHK(h->upload(&c.rp, c.h_rp.data(), c.h_rp.size()));
            CHK(h->upload(&c.ci, c.h_ci.data(), c.h_ci.size()));
            CHK(h->alloc(&c.A64, (size_t)c.nnzb * c.np * c.np));
        } else {
            CHK(h->upload(&f.parent, tr.parent, f.n_rows));
            {
                // store every distinct R_i once (equal bit for bit)
                const size_t bs = (size_t)f.np * c.np;
                std::unordered_map<uint64_t, std::vector<int>> seen;
                std::vector<double> table;
                f.h_ridx.assign(f.n_rows, -1);
                for (int i = 0; i < f.n_rows; ++i) {
                    const double* Ri = tr.R + (size_t)i * bs;
                    uint64_t hsh = 1469598103934665603ull;       // FNV-1a over the bytes
                    const unsigned char* by = reinterpret_cast<const unsigned char*>(Ri);
                    for (size_t q = 0; q < bs * sizeof(double); ++q)
                        hsh = (hsh ^ by[q]) * 1099511628211ull;
                    int id = -1;
                    for (int cand : seen[hsh])
                        if (std::memcmp(table.data() + (size_t)cand * bs, Ri,
                                        bs * sizeof(double)) == 0) {
                            id = cand;
                            break;
                        }
                    if (id < 0) {
                        id = f.n_rblocks++;
                        seen[hsh].push_back(id);
                        table.insert(table.end(), Ri, Ri + bs);
                    }
                    f.h_ridx[i] = id;
                }
                CHK(h->upload(&f.R64, table.data(), table.size()));
                CHK(h->upload(&f.ridx, f.h_ridx.data(), f.h_ridx.size()));
            }
            // children lists (ascending fine index)
            std::vector<int> chp(c.n_rows + 1, 0), chi(f.n_rows);
            for (int i = 0; i < f.n_rows; ++i) chp[tr.parent[i] + 1]++;
            for (int k = 0; k < c.n_rows; ++k) chp[k + 1] += chp[k];
            std::vector<int> fill(chp.begin(), chp.end() - 1);
            for (int i = 0; i < f.n_rows; ++i) chi[fill[tr.parent[i]]++] = i;
            CHK(h->upload(&f.chp, chp.data(), chp.size()));
            CHK(h->upload(&f.chi, chi.data(), chi.size()));
            CHK(galerkin_symbolic(h, f, c, tr.parent));
            if (h->nrhs == 1 && cc_dense_supported(f.np, c.np)) CHK(ar_symbolic(h, f, tr.parent));
            if (h->mixed || h->nrhs == kNrhs) {
                const int64_t nrr = (int64_t)f.n_rblocks * f.np * c.np;
                CHK(h->alloc(&f.R32, nrr));
                launch_convert<double, float>(h->s, nrr, f.R64, f.R32);
            }
        }
        CHK(setup_cells(h, c, tr.cell_ptr_c, tr.n_cells_c));
    }
    for (int l = 0; l + 1 < n_levels; ++l) {
        Level& lv = h->L[l];
        CHK(h->alloc(&lv.D64, lv.dsize));
        // leading columns for the post sweep after a p-coarse correction: the
        // single-column cycle at level 0
        if (l == 0 && h->nrhs == 1 && lv.t_kind == XDG_T_PTRUNC && cc_supported(lv.np, lv.npc)) {
            const size_t nap = (size_t)lv.nnzb * lv.np * lv.npc;
            if (h->mixed) CHK(h->alloc(&lv.AP32, nap));
            else CHK(h->alloc(&lv.AP64, nap));
        }
        if (h->mixed) {
            if (!lv.sym) CHK(h->alloc(&lv.A32, (size_t)lv.nnzb * lv.np * lv.np));
            CHK(h->alloc(&lv.D32, lv.dsize));
        }
    }
    {
        Level& lc = h->L[n_levels - 1];
        h->cn = lc.n_rows * lc.np;
        h->cld = ((h->cn + kCoarseNB - 1) / kCoarseNB) * kCoarseNB;
        CHK(h->alloc(&h->Cinv, (size_t)h->cld * h->cld));
        CHK(h->alloc(&h->Pbuf, 2 * kCoarseNB * kCoarseNB));
    }
    for (auto& lv : h->L) CHK(setup_vectors(h, lv, h->mixed));
    const int64_t n0 = L0.len();
    CHK(h->alloc(&h->scal, 4096));
    CHK(h->alloc(&h->part, kPartDoubles));
    HIPCHK(hipHostMalloc((void**)&h->h_scal, 4096 * sizeof(double), hipHostMallocDefault));
    CHK(h->alloc(&h->r, n0));
    CHK(h->alloc(&h->z, n0));
    CHK(h->alloc(&h->p, n0));
    CHK(h->alloc(&h->q, n0));
    CHK(h->alloc(&h->w, n0));
    if (opt->krylov == XDG_FGMRES && h->nrhs == 1) {
        CHK(h->alloc(&h->V, (size_t)(opt->restart + 1) * n0));
        CHK(h->alloc(&h->Z, (size_t)opt->restart * n0));
    }
    if (h->nrhs == kNrhs) CHK(mrhs_allocate(h));
    if (opt->krylov == XDG_ORTHOMG) CHK(xdg::orthomg_allocate(h));

    // -- numeric phase ------------------------------------------------------
    {
        const size_t nv = (size_t)L0.nnzb * L0.np * L0.np;
        double* raw;
        CHK(h->upload(&raw, A0->val, nv));
        HIPCHK(hipEventRecord(e0, h->s));
        CHK(numeric_setup(h, raw));
        HIPCHK(hipEventRecord(e1, h->s));
        HIPCHK(hipEventSynchronize(e1));
        h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), (void*)raw));
        HIPCHK(hipFree(raw));
    }
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    h->setup_ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    CHK(check_setup_error(h));
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

extern "C" int xdg_create(const xdg_matrix* A0, int32_t n_levels, const xdg_transfer* T,
                          const xdg_options* opt, void* hip_stream, xdg_handle** out) {
    if (!out) return fail(XDG_EINVAL, "xdg_create: out is NULL");
    *out = nullptr;
    xdg_handle* h = new xdg_handle();
    h->s = (hipStream_t)hip_stream;
    const int rc = create_impl(h, A0, n_levels, T, opt);
    if (rc < 0) {
        const std::string msg = xdg::last_error_text();
        xdg_destroy(h);
        fail(0, msg);
        return rc;
    }
    *out = h;
    return XDG_OK;
}

static int check_level(xdg_handle* h, int level, bool need_transfer) {
    if (!h) return fail(XDG_EINVAL, "NULL handle");
    const int nl = (int)h->L.size();
    if (level < 0 || level >= nl - (need_transfer ? 1 : 0))
        return fail(XDG_EINVAL, "level out of range");
    return XDG_OK;
}

extern "C" int xdg_level_info(xdg_handle* h, int32_t level, int32_t* n_rows, int32_t* np,
                              int32_t* nnzb) {
    CHK(check_level(h, level, false));
    const Level& lv = h->L[level];
    if (n_rows) *n_rows = lv.n_rows;
    if (np) *np = lv.np;
    if (nnzb) *nnzb = lv.nnzb;
    return XDG_OK;
}

extern "C" int xdg_spmv(xdg_handle* h, int32_t level, const double* x, double* y) {
    CHK(check_level(h, level, false));
    if (!x || !y) return fail(XDG_EINVAL, "xdg_spmv: NULL vector");
    Level& lv = h->L[level];
    if (h->nrhs == kNrhs) {
        // 16 columns [row][mode][16]: the FP64 matrix-core product of level 0
        // (the only level with packed FP64 blocks)
        if (level != 0)
            return fail(XDG_EINVAL, "xdg_spmv: a 16-column handle has the FP64 product on "
                                    "level 0 only (xdg_spmm with XDG_MIXED for coarser levels)");
        return mrhs_spmm(h, 0, XDG_FP64, x, y);
    }
    xdg::level_spmv<double>(h, lv, SPMV_AX, x, nullptr, y, 0);
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

extern "C" int xdg_smooth(xdg_handle* h, int32_t level, const double* b, double* x,
                          int32_t sweeps) {
    CHK(check_level(h, level, true));
    if (!b || !x || sweeps < 0) return fail(XDG_EINVAL, "xdg_smooth: bad argument");
    if (h->nrhs == kNrhs) return mrhs_smooth(h, level, b, x, sweeps);
    Level& lv = h->L[level];
    reset_dirs(h);
    for (int k = 0; k < sweeps; ++k) {
        xdg::level_jacobi<double>(h, lv, false, b, x, lv.y64);
        HIPCHK(hipMemcpyAsync(x, lv.y64, lv.len() * sizeof(double), hipMemcpyDeviceToDevice,
                              h->s));
    }
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

extern "C" int xdg_restrict(xdg_handle* h, int32_t level, const double* rf, double* rc) {
    CHK(check_level(h, level, true));
    if (!rf || !rc) return fail(XDG_EINVAL, "xdg_restrict: NULL vector");
    Level& f = h->L[level];
    Level& c = h->L[level + 1];
    if (h->nrhs == kNrhs) {
        if (f.t_kind == XDG_T_PTRUNC)
            launch_restrict_trunc_m<double>(h->s, f.n_rows, f.np, c.np, rf, rc);
        else
            launch_restrict_dense_m<double>(h->s, c.n_rows, f.np, c.np, f.chp, f.chi, f.ridx, f.R64, rf,
                                            rc);
    } else if (f.t_kind == XDG_T_PTRUNC)
        launch_restrict_trunc<double>(h->s, f.n_rows, f.np, c.np, rf, rc);
    else
        launch_restrict_dense<double>(h->s, c.n_rows, f.n_rows, f.np, c.np, f.chp, f.chi,
                                      f.ridx, f.R64, rf, rc, f.y64);
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

extern "C" int xdg_prolong(xdg_handle* h, int32_t level, const double* xc, double* xf) {
    CHK(check_level(h, level, true));
    if (!xc || !xf) return fail(XDG_EINVAL, "xdg_prolong: NULL vector");
    Level& f = h->L[level];
    Level& c = h->L[level + 1];
    if (h->nrhs == kNrhs) {
        if (f.t_kind == XDG_T_PTRUNC)
            launch_prolong_trunc_m<double>(h->s, f.n_rows, f.np, c.np, xc, xf);
        else
            launch_prolong_dense_m<double>(h->s, f.n_rows, f.np, c.np, f.parent, f.ridx, f.R64, xc,
                                           xf);
    } else if (f.t_kind == XDG_T_PTRUNC)
        launch_prolong_trunc<double>(h->s, f.n_rows, f.np, c.np, xc, xf);
    else
        launch_prolong_dense<double>(h->s, f.n_rows, f.np, c.np, f.parent, f.ridx, f.R64, xc,
                                     xf);
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

extern "C" int xdg_vcycle(xdg_handle* h, const double* r, double* z) {
    if (!h || !r || !z) return fail(XDG_EINVAL, "xdg_vcycle: NULL argument");
    if (h->nrhs == kNrhs) return mrhs_vcycle(h, r, z);
    reset_dirs(h);
    return apply_precond(h, r, z);
}

// -- Krylov solvers -------------------------------------------------------------

enum { S_BB = 0, S_RR = 1, S_PQ = 2, S_RZ0 = 3, S_RZ1 = 4, S_H = 8 };

static int read_scalars(xdg_handle* h, int first, int count) {
    HIPCHK(hipMemcpyAsync(h->h_scal + first, h->scal + first, count * sizeof(double),
                          hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    return XDG_OK;
}

static int true_relres(xdg_handle* h, const double* b, const double* x, double* out) {
    Level& f = h->L[0];
    xdg::level_spmv<double>(h, f, SPMV_RESID, x, b, h->w, 0);
    launch_dot(h->s, f.len(), h->w, h->w, h->part, h->scal + S_RR);
    launch_dot(h->s, f.len(), b, b, h->part, h->scal + S_BB);
    CHK(read_scalars(h, S_BB, 2));
    // b = 0: the solution is 0 and the residual is reported as an absolute norm
    const double nb = std::sqrt(h->h_scal[S_BB]);
    *out = nb > 0.0 ? std::sqrt(h->h_scal[S_RR]) / nb : std::sqrt(h->h_scal[S_RR]);
    return XDG_OK;
}

// Preconditioned CG.  With the FP32 V-cycle (precision XDG_MIXED) the
// preconditioner is symmetric only up to FP32 rounding, so the flexible
// variant is used (Notay's FCG with one stored direction): alpha = p.r / p.q
// and the new direction is made A-orthogonal to the previous one,
// beta = -z.q_old / p_old.q_old; in exact arithmetic with a fixed symmetric
// preconditioner it is PCG.
// the fused update's workgroup partials fit the reduction buffer
static bool n_cells_ok(const Level& f) {
    return (int64_t)(f.n_cells + 3) / 4 <= (int64_t)kPartDoubles;
}

// The host reads r . r and p . q of every iteration to test convergence.
// While the previous residual is more than kAheadFactor times the tolerance
// (CG's residual does not fall that much in one iteration here), the next
// direction's work -- preconditioner, r . z, new p; it writes neither x nor
// r -- is enqueued before the host waits for those scalars, so the device
// works on through the host's round trip.  Should the test pass after all,
// that work is simply not used.  Closer to the tolerance the host waits first.
constexpr double kAheadFactor = 10.0;

static int solve_cg(xdg_handle* h, const double* b, double* x, double* hist, int cap,
                    int* iters) {
    Level& f = h->L[0];
    const int64_t n = f.len();
    hipStream_t s = h->s;
    xdg::level_spmv<double>(h, f, SPMV_RESID, x, b, h->r, 0);
    launch_dot(s, n, b, b, h->part, h->scal + S_BB);
    launch_dot(s, n, h->r, h->r, h->part, h->scal + S_RR);
    CHK(read_scalars(h, S_BB, 2));
    const double nb = std::sqrt(h->h_scal[S_BB]);
    if (!std::isfinite(nb)) return fail(XDG_EINVAL, "xdg_solve: non-finite right-hand side");
    if (!std::isfinite(h->h_scal[S_RR]))
        return fail(XDG_EINVAL, "xdg_solve: non-finite initial guess");
    if (nb == 0.0) {
        HIPCHK(hipMemsetAsync(x, 0, n * sizeof(double), s));
        *iters = 0;
        if (cap > 0) hist[0] = 0.0;
        return XDG_OK;
    }
    double rel = std::sqrt(h->h_scal[S_RR]) / nb;
    if (cap > 0) hist[0] = rel;
    *iters = 0;
    if (rel <= h->opt.rtol) return XDG_OK;
    const bool flex = h->mixed;
    CHK(apply_precond(h, h->r, h->z));
    HIPCHK(hipMemcpyAsync(h->p, h->z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    int cur = S_RZ0, nxt = S_RZ1;
    if (!flex) launch_dot(s, n, h->r, h->z, h->part, h->scal + cur);
    // z = B r and the next direction p
    auto next_direction = [&]() -> int {
        CHK(apply_precond(h, h->r, h->z));
        if (flex) {
            launch_dot(s, n, h->z, h->q, h->part, h->scal + nxt);
            launch_fcg_update_p(s, n, h->scal, nxt, S_PQ, h->z, h->p);
        } else {
            launch_dot(s, n, h->r, h->z, h->part, h->scal + nxt);
            launch_cg_update_p(s, n, h->scal, nxt, cur, h->z, h->p);
            std::swap(cur, nxt);
        }
        return XDG_OK;
    };
    for (int k = 1; k <= h->opt.maxit; ++k) {
        // q = A p with p . q formed in the product's epilogue where the block
        // size allows, and r . r formed in the update of x and r
        xdg::level_spmv_dot(h, f, h->p, h->q, h->scal + S_PQ);
        if (flex) launch_dot(s, n, h->p, h->r, h->part, h->scal + cur);   // alpha numerator
        // the update fused with the next cycle's first level-0 sweep where the
        // cycle would start with it (FP64 block Jacobi, pre-sweeps, a level
        // below); if r converges the sweep was not needed
        const bool fuse = !flex && h->opt.smoother == XDG_JACOBI && h->opt.nu_pre >= 1 &&
                          h->L.size() > 1 && n_cells_ok(f) &&
                          launch_cg_update_first(s, f.n_cells, f.np, f.cp, f.doff, f.D64, h->scal,
                                                 cur, S_PQ, S_RR, h->p, h->q, x, h->r, f.x64,
                                                 h->opt.omega, h->part);
        if (!fuse)
            launch_cg_update_xr_dot(s, n, h->scal, cur, S_PQ, S_RR, h->p, h->q, x, h->r,
                                    h->part);
        h->x1_ready = fuse;
        HIPCHK(hipMemcpyAsync(h->h_scal + S_RR, h->scal + S_RR, 2 * sizeof(double),
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(h->ev_scal, s));
        const bool ahead = k < h->opt.maxit && rel > kAheadFactor * h->opt.rtol;
        if (ahead) CHK(next_direction());
        HIPCHK(hipEventSynchronize(h->ev_scal));
        HIPCHK(hipGetLastError());
        *iters = k;
        if (!(h->h_scal[S_PQ] > 0.0))
            return fail(XDG_EBREAKDOWN, "CG breakdown: p^T A p <= 0");
        rel = std::sqrt(h->h_scal[S_RR]) / nb;
        if (k < cap) hist[k] = rel;
        if (rel <= h->opt.rtol) return XDG_OK;
        if (!ahead) CHK(next_direction());
    }
    return XDG_ENOCONV;
}

// Flexible GMRES(m) with classical Gram-Schmidt applied twice; Arnoldi vectors,
// inner products and the true residual at every restart in FP64; the
// preconditioner runs in the handle's precision.
static int solve_fgmres(xdg_handle* h, const double* b, double* x, double* hist, int cap,
                        int* iters) {
    Level& f = h->L[0];
    const int64_t n = f.len();
    const int m = h->opt.restart;
    hipStream_t s = h->s;
    launch_dot(s, n, b, b, h->part, h->scal + S_BB);
    CHK(read_scalars(h, S_BB, 1));
    const double nb = std::sqrt(h->h_scal[S_BB]);
    if (!std::isfinite(nb)) return fail(XDG_EINVAL, "xdg_solve: non-finite right-hand side");
    *iters = 0;
    if (nb == 0.0) {
        HIPCHK(hipMemsetAsync(x, 0, n * sizeof(double), s));
        if (cap > 0) hist[0] = 0.0;
        return XDG_OK;
    }
    std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    h->learned_off = false;
    int k = 0;
    bool first = true;
    for (;;) {
        // true FP64 residual (the refinement step)
        xdg::level_spmv<double>(h, f, SPMV_RESID, x, b, h->r, 0);
        launch_dot(s, n, h->r, h->r, h->part, h->scal + S_RR);
        CHK(read_scalars(h, S_RR, 1));
        const double beta = std::sqrt(h->h_scal[S_RR]);
        if (!std::isfinite(beta)) return fail(XDG_EINVAL, "xdg_solve: non-finite residual");
        const double rel = beta / nb;
        if (k < cap) hist[k] = rel;       // replaces the estimate of the last inner step
        if (rel <= h->opt.rtol) return XDG_OK;
        if (k >= h->opt.maxit) return XDG_ENOCONV;
        if (!first && !(beta > 0.0)) return fail(XDG_EBREAKDOWN, "FGMRES: zero residual norm");
        first = false;
        h->h_scal[S_H] = beta;
        HIPCHK(hipMemcpyAsync(h->scal + S_H, h->h_scal + S_H, sizeof(double),
                              hipMemcpyHostToDevice, s));
        launch_div_scalar(s, n, h->scal, S_H, h->r, h->V);
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int j = 0, jdone = 0;
        for (j = 0; j < m && k < h->opt.maxit; ++j) {
            double* vj = h->V + (int64_t)j * n;
            double* zj = h->Z + (int64_t)j * n;
            double* vn = h->V + (int64_t)(j + 1) * n;
            CHK(apply_precond(h, vj, zj));
            xdg::level_spmv<double>(h, f, SPMV_AX, zj, nullptr, vn, 0);
            // CGS2
            launch_multidot(s, n, j + 1, h->V, vn, h->part, h->scal + S_H);
            launch_multi_axpy_neg(s, n, j + 1, h->V, h->scal + S_H, vn);
            launch_multidot(s, n, j + 1, h->V, vn, h->part, h->scal + S_H + 64);
            launch_multi_axpy_neg(s, n, j + 1, h->V, h->scal + S_H + 64, vn);
            launch_dot(s, n, vn, vn, h->part, h->scal + S_H + 128);
            CHK(read_scalars(h, S_H, 129));
            for (int i = 0; i <= j; ++i)
                H[i * m + j] = h->h_scal[S_H + i] + h->h_scal[S_H + 64 + i];
            const double hn = std::sqrt(h->h_scal[S_H + 128]);
            H[(j + 1) * m + j] = hn;
            h->h_scal[S_H + 192] = hn;
            HIPCHK(hipMemcpyAsync(h->scal + S_H + 192, h->h_scal + S_H + 192, sizeof(double),
                                  hipMemcpyHostToDevice, s));
            if (hn > 0.0) launch_div_scalar(s, n, h->scal, S_H + 192, vn, vn);
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
                H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
                H[i * m + j] = t;
            }
            const double den = std::hypot(H[j * m + j], H[(j + 1) * m + j]);
            if (!(den > 0.0)) return fail(XDG_EBREAKDOWN, "FGMRES: Arnoldi breakdown");
            cs[j] = H[j * m + j] / den;
            sn[j] = H[(j + 1) * m + j] / den;
            H[j * m + j] = den;
            H[(j + 1) * m + j] = 0.0;
            const double gprev = std::fabs(g[j]);
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            // residual-decrease test of the learned smoother: a step that
            // leaves the residual estimate almost unchanged switches it off
            if (xdg::learned_active(h) && std::fabs(g[j + 1]) > xdg::kLearnedStall * gprev) {
                h->learned_off = true;
                h->learned_fallbacks += 1;
            }
            ++k;
            jdone = j + 1;
            if (k < cap) hist[k] = std::fabs(g[j + 1]) / nb;
            *iters = k;
            if (std::fabs(g[j + 1]) / nb <= h->opt.rtol || hn == 0.0) break;
        }
        // y = H^{-1} g (upper triangular), x += Z y
        for (int i = jdone - 1; i >= 0; --i) {
            double t = g[i];
            for (int l = i + 1; l < jdone; ++l) t -= H[i * m + l] * y[l];
            y[i] = t / H[i * m + i];
        }
        std::memcpy(h->h_scal + S_H, y.data(), jdone * sizeof(double));
        HIPCHK(hipMemcpyAsync(h->scal + S_H, h->h_scal + S_H, jdone * sizeof(double),
                              hipMemcpyHostToDevice, s));
        launch_multi_axpy(s, n, jdone, h->Z, h->scal + S_H, x);
        HIPCHK(hipGetLastError());
    }
}

extern "C" int xdg_solve(xdg_handle* h, const double* b, double* x, double* hist,
                         int32_t hist_cap, int32_t* iters, double* final_relres) {
    if (!h || !b || !x || !iters || !final_relres || (hist_cap > 0 && !hist))
        return fail(XDG_EINVAL, "xdg_solve: NULL argument");
    *iters = 0;
    int it = 0;
    reset_dirs(h);
    if (h->nrhs == kNrhs) {
        const int rcm = mrhs_solve(h, b, x, hist, hist_cap, &it, final_relres);
        *iters = it;
        if (rcm == XDG_ENOCONV) fail(0, "xdg_solve: iteration limit reached");
        return rcm;
    }
    int rc = h->opt.krylov == XDG_CG       ? solve_cg(h, b, x, hist, hist_cap, &it)
             : h->opt.krylov == XDG_FGMRES ? solve_fgmres(h, b, x, hist, hist_cap, &it)
                                           : xdg::solve_orthomg(h, b, x, hist, hist_cap, &it);
    *iters = it;
    if (rc < 0) {
        // work the solver enqueued ahead of its last test may still be running
        (void)hipStreamSynchronize(h->s);
        return rc;
    }
    CHK(true_relres(h, b, x, final_relres));
    if (rc == XDG_ENOCONV) fail(0, "xdg_solve: iteration limit reached");
    return rc;
}

extern "C" int xdg_get_level_matrix(xdg_handle* h, int32_t level, int32_t* row_ptr,
                                    int32_t* col_idx, double* val) {
    CHK(check_level(h, level, false));
    if (!row_ptr || !col_idx || !val) return fail(XDG_EINVAL, "NULL output");
    Level& lv = h->L[level];
    std::copy(lv.h_rp.begin(), lv.h_rp.end(), row_ptr);
    std::copy(lv.h_ci.begin(), lv.h_ci.end(), col_idx);
    const int np = lv.np;
    std::vector<double> cm((size_t)lv.nnzb * np * np);
    HIPCHK(hipMemcpyAsync(cm.data(), lv.A64, cm.size() * sizeof(double), hipMemcpyDeviceToHost,
                          h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    for (int64_t b = 0; b < lv.nnzb; ++b)
        for (int r = 0; r < np; ++r)
            for (int c = 0; c < np; ++c)
                val[b * np * np + r * np + c] = cm[b * np * np + c * np + r];
    return XDG_OK;
}

extern "C" int xdg_get_cell_inverse(xdg_handle* h, int32_t level, int32_t cell, double* out,
                                    int32_t cap, int32_t* n) {
    CHK(check_level(h, level, false));
    if (!out || !n) return fail(XDG_EINVAL, "NULL output");
    if (level == (int)h->L.size() - 1) {
        if (cell != 0) return fail(XDG_EINVAL, "coarsest level has one block");
        *n = h->cn;
        if ((int64_t)h->cn * h->cn > cap) return fail(XDG_EINVAL, "output too small");
        HIPCHK(hipMemcpy2DAsync(out, h->cn * sizeof(double), h->Cinv, h->cld * sizeof(double),
                                h->cn * sizeof(double), h->cn, hipMemcpyDeviceToHost, h->s));
        HIPCHK(hipStreamSynchronize(h->s));
        return XDG_OK;
    }
    Level& lv = h->L[level];
    if (cell < 0 || cell >= lv.n_cells) return fail(XDG_EINVAL, "cell out of range");
    const int nc = (lv.h_cp[cell + 1] - lv.h_cp[cell]) * lv.np;
    *n = nc;
    if ((int64_t)nc * nc > cap) return fail(XDG_EINVAL, "output too small");
    std::vector<double> cm((size_t)nc * nc);
    HIPCHK(hipMemcpyAsync(cm.data(), lv.D64 + lv.h_doff[cell], cm.size() * sizeof(double),
                          hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    for (int r = 0; r < nc; ++r)
        for (int c = 0; c < nc; ++c) out[r * nc + c] = cm[(size_t)c * nc + r];
    return XDG_OK;
}

extern "C" int xdg_set_projection(xdg_handle* h, const xdg_projection* P) {
    if (!h || !P) return fail(XDG_EINVAL, "xdg_set_projection: NULL argument");
    if (h->nrhs != 1) return fail(XDG_EINVAL, "xdg_set_projection: single-column handles only");
    const Level& L0 = h->L[0];
    if (P->n_rows != L0.n_rows || P->np != L0.np || P->n_cols < 1 || P->nnzb < 1 ||
        !P->row_ptr || !P->col_idx || !P->val)
        return fail(XDG_EINVAL, "xdg_set_projection: sizes do not match level 0");
    if (P->row_ptr[0] != 0 || P->row_ptr[P->n_rows] != P->nnzb)
        return fail(XDG_EINVAL, "xdg_set_projection: row_ptr does not span [0, nnzb]");
    for (int i = 0; i < P->n_rows; ++i) {
        if (P->row_ptr[i + 1] < P->row_ptr[i])
            return fail(XDG_EINVAL, "xdg_set_projection: row_ptr decreases");
        for (int b = P->row_ptr[i]; b < P->row_ptr[i + 1]; ++b) {
            if (P->col_idx[b] < 0 || P->col_idx[b] >= P->n_cols)
                return fail(XDG_EINVAL, "xdg_set_projection: column index out of range");
            if (b > P->row_ptr[i] && P->col_idx[b] <= P->col_idx[b - 1])
                return fail(XDG_EINVAL, "xdg_set_projection: columns not strictly sorted");
        }
    }
    const size_t nv = (size_t)P->nnzb * P->np * P->np;
    if (!finite_all(P->val, nv)) return fail(XDG_EINVAL, "xdg_set_projection: non-finite entry");
    h->release(h->proj_rp);
    h->release(h->proj_ci);
    h->release(h->proj_A);
    h->proj_rp = h->proj_ci = nullptr;
    h->proj_A = nullptr;
    h->proj_rows = h->proj_cols = h->proj_nnzb = 0;
    CHK(h->upload(&h->proj_rp, P->row_ptr, (size_t)P->n_rows + 1));
    CHK(h->upload(&h->proj_ci, P->col_idx, (size_t)P->nnzb));
    CHK(h->alloc(&h->proj_A, nv));
    double* raw = nullptr;
    CHK(h->upload(&raw, P->val, nv));
    launch_transpose_blocks<double>(h->s, P->nnzb, P->np, raw, h->proj_A);
    HIPCHK(hipStreamSynchronize(h->s));
    h->release(raw);
    HIPCHK(hipGetLastError());
    h->proj_rows = P->n_rows;
    h->proj_cols = P->n_cols;
    h->proj_nnzb = P->nnzb;
    return XDG_OK;
}

extern "C" int xdg_project(xdg_handle* h, const double* x_old, double* x_new) {
    if (!h || !x_old || !x_new) return fail(XDG_EINVAL, "xdg_project: NULL argument");
    if (!h->proj_A) return fail(XDG_EINVAL, "xdg_project: no operator (xdg_set_projection)");
    const Level& L0 = h->L[0];
    launch_spmv<double>(h->s, SPMV_AX, h->proj_rows, L0.np, h->proj_rp, h->proj_ci, h->proj_A,
                        x_old, nullptr, x_new, 0);
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

extern "C" int xdg_update_matrix(xdg_handle* h, const double* val_dev) {
    if (!h || !val_dev) return fail(XDG_EINVAL, "xdg_update_matrix: NULL argument");
    CHK(numeric_setup(h, val_dev));
    return check_setup_error(h);
}

// Partial numeric set-up: the level-0 values changed only in the block rows
// and block columns of the listed smoother cells.  Affected sets, level by
// level: the level-0 blocks in those rows and their transposed blocks; a
// p-truncated level keeps the block indices; an aggregation level takes the
// coarse blocks the affected fine blocks contribute to; a cell is re-inverted
// when one of its diagonal-cell blocks is affected.  The same kernels as the
// full set-up run on the listed blocks and cells, so the result equals the
// full set-up's.  Host work is proportional to the affected sets (the maps
// below are built once per handle).
static int update_prepare(xdg_handle* h) {
    if (h->h_stage) return XDG_OK;
    int64_t total = 0;
    for (auto& lv : h->L) {
        lv.h_rob.resize(lv.nnzb);
        for (int i = 0; i < lv.n_rows; ++i)
            for (int b = lv.h_rp[i]; b < lv.h_rp[i + 1]; ++b) lv.h_rob[b] = i;
        lv.h_cor.assign(lv.n_rows, -1);
        for (int c = 0; c < lv.n_cells; ++c)
            for (int r = lv.h_cp[c]; r < lv.h_cp[c + 1]; ++r) lv.h_cor[r] = c;
        lv.h_bmark.assign(lv.nnzb, 0);
        lv.h_cmark.assign(std::max(lv.n_cells, 1), 0);
        total += lv.nnzb + lv.n_cells;
    }
    Level& L0 = h->L[0];
    L0.h_btr.assign(L0.nnzb, -1);
    for (int b = 0; b < L0.nnzb; ++b) {
        const int i = L0.h_rob[b], l = L0.h_ci[b];
        for (int e = L0.h_rp[l]; e < L0.h_rp[l + 1]; ++e)
            if (L0.h_ci[e] == i) L0.h_btr[b] = e;
        if (L0.h_btr[b] < 0)
            return fail(XDG_EINVAL, "xdg_update_cells: the level-0 pattern is not symmetric");
    }
    HIPCHK(hipHostMalloc((void**)&h->h_stage, std::max<int64_t>(total, 1) * sizeof(int),
                         hipHostMallocDefault));
    CHK(h->alloc(&h->d_stage, (size_t)std::max<int64_t>(total, 1)));
    h->stage_len = total;
    return XDG_OK;
}

extern "C" int xdg_update_cells(xdg_handle* h, const double* val_dev, int32_t n,
                                const int32_t* cells) {
    if (!h || !val_dev || n < 1 || !cells)
        return fail(XDG_EINVAL, "xdg_update_cells: NULL argument or n < 1");
    if (h->nrhs != 1)
        return fail(XDG_EINVAL, "xdg_update_cells: single-column handles only (use "
                                "xdg_update_matrix)");
    Level& L0 = h->L[0];
    for (int k = 0; k < n; ++k)
        if (cells[k] < 0 || cells[k] >= L0.n_cells)
            return fail(XDG_EINVAL, "xdg_update_cells: cell index out of range");
    CHK(update_prepare(h));
    {   // repeated cells
        std::vector<int32_t> sorted(cells, cells + n);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return fail(XDG_EINVAL, "xdg_update_cells: repeated cell");
    }
    const int nl = (int)h->L.size();
    // host lists, level by level, written straight into the pinned stage
    int* stage = h->h_stage;
    int64_t used = 0;
    std::vector<int64_t> boff(nl), bcnt(nl), coff(nl), ccnt(nl);
    std::vector<int> cur, nxt;
    for (int c = 0; c < n; ++c)
        for (int r = L0.h_cp[cells[c]]; r < L0.h_cp[cells[c] + 1]; ++r)
            for (int b = L0.h_rp[r]; b < L0.h_rp[r + 1]; ++b)
                for (int e : {b, L0.h_btr[b]})
                    if (!L0.h_bmark[e]) {
                        L0.h_bmark[e] = 1;
                        cur.push_back(e);
                    }
    for (int t = 0; t < nl; ++t) {
        Level& lv = h->L[t];
        boff[t] = used;
        bcnt[t] = (int64_t)cur.size();
        for (int b : cur) stage[used++] = b;
        coff[t] = used;
        ccnt[t] = 0;
        if (t + 1 < nl) {
            for (int b : cur) {
                const int c = lv.h_cor[lv.h_rob[b]];
                if (c == lv.h_cor[lv.h_ci[b]] && !lv.h_cmark[c]) {
                    lv.h_cmark[c] = 1;
                    stage[used++] = c;
                    ccnt[t]++;
                }
            }
            for (int64_t k = 0; k < ccnt[t]; ++k) lv.h_cmark[stage[coff[t] + k]] = 0;
            Level& cl = h->L[t + 1];
            nxt.clear();
            for (int b : cur) {
                const int cb = lv.t_kind == XDG_T_PTRUNC ? b : lv.h_fb2cb[b];
                if (!cl.h_bmark[cb]) {
                    cl.h_bmark[cb] = 1;
                    nxt.push_back(cb);
                }
            }
        }
        for (int b : cur) lv.h_bmark[b] = 0;
        cur.swap(nxt);
    }
    hipStream_t s = h->s;
    HIPCHK(hipMemsetAsync(h->d_err, 0, sizeof(int), s));
    if (used > 0)
        HIPCHK(hipMemcpyAsync(h->d_stage, stage, used * sizeof(int), hipMemcpyHostToDevice, s));
    for (int t = 0; t < nl; ++t) {
        Level& lv = h->L[t];
        const int* bl = h->d_stage + boff[t];
        if (t == 0) {
            launch_transpose_list(s, (int)bcnt[t], bl, lv.np, val_dev, lv.A64);
        } else {
            Level& f = h->L[t - 1];
            if (f.t_kind == XDG_T_PTRUNC)
                launch_extract_list(s, (int)bcnt[t], bl, f.np, lv.np, f.A64, lv.A64);
            else if (f.g_U)     // wide level: the whole product, as in the full set-up
                launch_galerkin_wide(s, f.n_grp, lv.nnzb, f.np, lv.np, f.g_gstart, f.g_grow,
                                     f.g_cbg, f.g_fb, f.g_col, f.A64, f.R64, f.g_U, lv.A64);
            else
                launch_galerkin_dense(s, (int)bcnt[t], f.np, lv.np, f.g_ptr, f.g_fb, f.g_row,
                                      f.g_col, f.A64, f.R64, lv.A64, bl);
        }
    }
    // level 0's symmetric copies, the listed cells' inversions and the FP32
    // copies on the side stream while the coarsest inverse is rebuilt, as in
    // the full set-up
    HIPCHK(hipEventRecord(h->ev_fork, s));
    HIPCHK(hipStreamWaitEvent(h->s2, h->ev_fork, 0));
    sym_refresh(h->L[0], h->s2);
    for (int t = 0; t + 1 < nl; ++t) {
        if (ccnt[t] == 0) continue;
        Level& lv = h->L[t];
        const int* cl = h->d_stage + coff[t];
        launch_gather_cells(h->s2, (int)ccnt[t], lv.np, lv.cp, lv.rp, lv.ci, lv.A64, lv.doff,
                            lv.D64, cl);
        launch_gj_batched(h->s2, (int)ccnt[t], lv.doff, lv.cp, lv.np, lv.max_nc, lv.D64,
                          h->d_err, cl);
    }
    ar_numeric(h, h->s2);
    if (h->mixed)
        for (int l = 0; l + 1 < nl; ++l) convert_level32(h->L[l], h->s2);
    HIPCHK(hipEventRecord(h->ev_join, h->s2));
    CHK(invert_coarsest(h, h->L[nl - 1]));
    HIPCHK(hipStreamWaitEvent(s, h->ev_join, 0));
    HIPCHK(hipGetLastError());
    return check_setup_error(h);   // synchronises: the stage may be reused afterwards
}

extern "C" int xdg_set_tolerance(xdg_handle* h, double rtol, int32_t maxit) {
    if (!h) return fail(XDG_EINVAL, "xdg_set_tolerance: NULL handle");
    if (!(rtol > 0.0) || maxit < 1) return fail(XDG_EINVAL, "xdg_set_tolerance: bad rtol or maxit");
    h->opt.rtol = rtol;
    h->opt.maxit = maxit;
    return XDG_OK;
}

extern "C" int xdg_setup_time(xdg_handle* h, double* ms) {
    if (!h || !ms) return fail(XDG_EINVAL, "NULL argument");
    *ms = h->setup_ms;
    return XDG_OK;
}
