// Sixteen right-hand sides at once: FP32 MFMA V-cycle as the preconditioner
// of sixteen independent flexible GMRES(m) iterations that share every
// operator application.  The Arnoldi matvec and the residual at every restart
// use the FP64 matrix on FP64 MFMA; inner products accumulate in FP64; the
// Krylov vectors V, Z are stored in FP32.  Each column keeps its own
// Hessenberg matrix, Givens rotations and stopping state on the host.
#include "xdg_handle.h"

using namespace xdg;

namespace {

// device scalar layout (doubles)
constexpr int M_BB = 0, M_RR = 16, M_HN = 32, M_SC = 48, M_H1 = 64, M_H2 = 64 + 64 * 16,
              M_CO = 64 + 2 * 64 * 16, M_END = 64 + 3 * 64 * 16;

int rd(xdg_handle* h, int first, int count) {
    HIPCHK(hipMemcpyAsync(h->h_scal + first, h->scal + first, count * sizeof(double),
                          hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    return XDG_OK;
}

int wr(xdg_handle* h, int first, int count) {
    HIPCHK(hipMemcpyAsync(h->scal + first, h->h_scal + first, count * sizeof(double),
                          hipMemcpyHostToDevice, h->s));
    return XDG_OK;
}

void sweeps_m(xdg_handle* h, Level& lv, bool from_zero, int n) {
    const float om = (float)h->opt.omega;
    int k = 0;
    if (from_zero) {
        if (n <= 0) {
            (void)hipMemsetAsync(lv.xm, 0, lv.len() * kNrhs * sizeof(float), h->s);
            return;
        }
        launch_jacobi_mrhs(h->s, true, lv.n_cells, lv.np, lv.cp, lv.rp, lv.ci, lv.Ap32, lv.doff,
                           lv.Dp32, lv.bm, nullptr, lv.xm, om);
        k = 1;
    }
    for (; k < n; ++k) {
        launch_jacobi_mrhs(h->s, false, lv.n_cells, lv.np, lv.cp, lv.rp, lv.ci, lv.Ap32, lv.doff,
                           lv.Dp32, lv.bm, lv.xm, lv.ym, om);
        std::swap(lv.xm, lv.ym);
    }
}

// input L[l].bm, output L[l].xm (FP32, 16 columns)
void vcycle_m(xdg_handle* h, int l) {
    Level& f = h->L[l];
    const int64_t n16 = f.len() * kNrhs;
    if (l == (int)h->L.size() - 1) {
        launch_convert<float, double>(h->s, n16, f.bm, f.bm64);
        launch_coarse_gemm16(h->s, h->cn, h->cld, h->Cinv, f.bm64, f.xm64);
        launch_convert<double, float>(h->s, n16, f.xm64, f.xm);
        return;
    }
    Level& c = h->L[l + 1];
    sweeps_m(h, f, true, xdg::sweeps_pre(h, l));
    if (f.t_kind == XDG_T_PTRUNC) {
        launch_spmm<float, float, float>(h->s, SPMV_RESID_TRUNC, f.n_rows, f.np, f.rp, f.ci,
                                         f.Ap32, f.xm, f.bm, c.bm, c.np);
    } else {
        launch_spmm<float, float, float>(h->s, SPMV_RESID, f.n_rows, f.np, f.rp, f.ci, f.Ap32,
                                         f.xm, f.bm, f.rm, 0);
        launch_restrict_dense_m<float>(h->s, c.n_rows, f.np, c.np, f.chp, f.chi, f.ridx, f.R32, f.rm,
                                       c.bm);
    }
    vcycle_m(h, l + 1);
    if (f.t_kind == XDG_T_PTRUNC)
        launch_prolong_trunc_m<float>(h->s, f.n_rows, f.np, c.np, c.xm, f.xm);
    else
        launch_prolong_dense_m<float>(h->s, f.n_rows, f.np, c.np, f.parent, f.ridx, f.R32, c.xm,
                                      f.xm);
    sweeps_m(h, f, false, xdg::sweeps_post(h, l));
}

// z = B v on 16 FP32 columns
int precond_m(xdg_handle* h, const float* v, float* z) {
    Level& f = h->L[0];
    float* keep = f.bm;
    f.bm = const_cast<float*>(v);
    vcycle_m(h, 0);
    f.bm = keep;
    HIPCHK(hipMemcpyAsync(z, f.xm, f.len() * kNrhs * sizeof(float), hipMemcpyDeviceToDevice,
                          h->s));
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

}  // namespace

namespace xdg {

int mrhs_validate(const xdg_options* opt, int np0, const xdg_transfer* T, int n_levels) {
    if (opt->krylov != XDG_FGMRES || opt->precision != XDG_MIXED)
        return fail(XDG_EINVAL, "16 right-hand sides need krylov XDG_FGMRES and XDG_MIXED");
    if (!mrhs_np_supported(np0)) return fail(XDG_EINVAL, "16 right-hand sides: unsupported np");
    for (int t = 0; t < n_levels - 1; ++t)
        if (!mrhs_np_supported(T[t].np_c))
            return fail(XDG_EINVAL, "16 right-hand sides: unsupported coarse np");
    return XDG_OK;
}

int mrhs_allocate(xdg_handle* h) {
    const int nl = (int)h->L.size();
    for (int l = 0; l < nl; ++l) {
        Level& lv = h->L[l];
        const int64_t n16 = lv.len() * kNrhs;
        CHK(h->alloc(&lv.bm, n16));
        CHK(h->alloc(&lv.xm, n16));
        CHK(h->alloc(&lv.ym, n16));
        CHK(h->alloc(&lv.rm, n16));
        if (l + 1 < nl) {
            CHK(h->alloc(&lv.Ap32, (size_t)lv.nnzb * lv.np * lv.np));
            CHK(h->alloc(&lv.Dp32, lv.dsize));
        } else {
            CHK(h->alloc(&lv.bm64, n16));
            CHK(h->alloc(&lv.xm64, n16));
        }
    }
    Level& L0 = h->L[0];
    CHK(h->alloc(&L0.Ap64, (size_t)L0.nnzb * L0.np * L0.np));
    const int64_t n16 = L0.len() * kNrhs;
    const int m = h->opt.restart;
    CHK(h->alloc(&h->Vm, (size_t)(m + 1) * n16));
    CHK(h->alloc(&h->Zm, (size_t)m * n16));
    CHK(h->alloc(&h->Wm, n16));
    CHK(h->alloc(&h->Rm, n16));
    return XDG_OK;
}

// packed copies of the freshly computed FP64 levels and inverses
int mrhs_numeric(xdg_handle* h) {
    const int nl = (int)h->L.size();
    for (int l = 0; l + 1 < nl; ++l) {
        Level& lv = h->L[l];
        launch_pack_blocks<float>(h->s, lv.nnzb, lv.np, lv.A64, lv.Ap32);
        launch_pack_cells(h->s, lv.n_cells, lv.np, lv.cp, lv.doff, lv.D64, lv.Dp32);
    }
    Level& L0 = h->L[0];
    launch_pack_blocks<double>(h->s, L0.nnzb, L0.np, L0.A64, L0.Ap64);
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

int mrhs_spmm(xdg_handle* h, int level, int precision, const double* X, double* Y) {
    Level& lv = h->L[level];
    const int64_t n16 = lv.len() * kNrhs;
    if (precision == XDG_FP64) {
        if (level != 0) return fail(XDG_EINVAL, "xdg_spmm: FP64 product on level 0 only");
        launch_spmm<double, double, double>(h->s, SPMV_AX, lv.n_rows, lv.np, lv.rp, lv.ci,
                                            lv.Ap64, X, nullptr, Y, 0);
    } else {
        if (level == (int)h->L.size() - 1)
            return fail(XDG_EINVAL, "xdg_spmm: no FP32 copy of the coarsest level");
        launch_convert<double, float>(h->s, n16, X, lv.rm);
        launch_spmm<float, float, float>(h->s, SPMV_AX, lv.n_rows, lv.np, lv.rp, lv.ci,
                                         lv.Ap32, lv.rm, nullptr, lv.ym, 0);
        launch_convert<float, double>(h->s, n16, lv.ym, Y);
    }
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

int mrhs_smooth(xdg_handle* h, int level, const double* B, double* X, int sweeps) {
    Level& lv = h->L[level];
    const int64_t n16 = lv.len() * kNrhs;
    launch_convert<double, float>(h->s, n16, B, lv.bm);
    launch_convert<double, float>(h->s, n16, X, lv.xm);
    sweeps_m(h, lv, false, sweeps);
    launch_convert<float, double>(h->s, n16, lv.xm, X);
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

int mrhs_vcycle(xdg_handle* h, const double* R, double* Z) {
    Level& f = h->L[0];
    const int64_t n16 = f.len() * kNrhs;
    launch_convert<double, float>(h->s, n16, R, f.bm);
    vcycle_m(h, 0);
    launch_convert<float, double>(h->s, n16, f.xm, Z);
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

int mrhs_solve(xdg_handle* h, const double* B, double* X, double* hist, int cap, int* iters,
               double* final_relres) {
    Level& f = h->L[0];
    const int64_t n16 = f.len() * kNrhs;
    const int m = h->opt.restart;
    hipStream_t s = h->s;
    const double rtol = h->opt.rtol;
    auto residual = [&](double* rel_out, double* beta_out, double* nb) -> int {
        launch_spmm<double, double, double>(s, SPMV_RESID, f.n_rows, f.np, f.rp, f.ci, f.Ap64, X,
                                            B, h->Rm, 0);
        launch_multidot16<double>(s, n16, 1, h->Rm, h->Rm, h->part, h->scal + M_RR);
        CHK(rd(h, M_RR, 16));
        double mx = 0.0;
        for (int c = 0; c < kNrhs; ++c) {
            beta_out[c] = std::sqrt(h->h_scal[M_RR + c]);
            if (!std::isfinite(beta_out[c]))
                return fail(XDG_EINVAL, "xdg_solve: non-finite residual");
            rel_out[c] = nb[c] > 0.0 ? beta_out[c] / nb[c] : 0.0;
            mx = std::max(mx, rel_out[c]);
        }
        *final_relres = mx;
        return XDG_OK;
    };
    launch_multidot16<double>(s, n16, 1, B, B, h->part, h->scal + M_BB);
    CHK(rd(h, M_BB, 16));
    double nb[kNrhs], beta[kNrhs], rel[kNrhs];
    for (int c = 0; c < kNrhs; ++c) {
        nb[c] = std::sqrt(h->h_scal[M_BB + c]);
        if (!std::isfinite(nb[c])) return fail(XDG_EINVAL, "xdg_solve: non-finite right-hand side");
    }
    // a zero right-hand side column has the solution zero (whatever x0 held)
    bool any_zero = false;
    for (int c = 0; c < kNrhs; ++c) {
        h->h_scal[M_SC + c] = nb[c] > 0.0 ? 1.0 : 0.0;
        any_zero |= !(nb[c] > 0.0);
    }
    if (any_zero) {
        CHK(wr(h, M_SC, 16));
        launch_zero_cols16(s, n16, h->scal + M_SC, X);
    }
    std::vector<double> H((size_t)kNrhs * (m + 1) * m), cs((size_t)kNrhs * m),
        sn((size_t)kNrhs * m), g((size_t)kNrhs * (m + 1));
    int jdone[kNrhs];
    bool live[kNrhs];
    int k = 0;
    *iters = 0;
    for (;;) {
        CHK(residual(rel, beta, nb));
        double mx = 0.0;
        for (int c = 0; c < kNrhs; ++c) mx = std::max(mx, rel[c]);
        if (k < cap) hist[k] = mx;
        if (mx <= rtol) return XDG_OK;
        if (k >= h->opt.maxit) return XDG_ENOCONV;
        for (int c = 0; c < kNrhs; ++c) {
            live[c] = rel[c] > rtol && beta[c] > 0.0;
            h->h_scal[M_SC + c] = live[c] ? 1.0 / beta[c] : 0.0;
            jdone[c] = 0;
            std::fill(g.begin() + (size_t)c * (m + 1), g.begin() + (size_t)(c + 1) * (m + 1), 0.0);
            g[(size_t)c * (m + 1)] = live[c] ? beta[c] : 0.0;
        }
        std::fill(H.begin(), H.end(), 0.0);
        for (int c = 0; c < kNrhs; ++c)
            if (!live[c]) g[(size_t)c * (m + 1)] = nb[c] * rel[c];   // frozen: keep its residual
        CHK(wr(h, M_SC, 16));
        launch_scale16<float>(s, n16, h->Rm, h->scal + M_SC, h->Vm);
        int jmax = 0;
        for (int j = 0; j < m && k < h->opt.maxit; ++j) {
            float* vj = h->Vm + (int64_t)j * n16;
            float* zj = h->Zm + (int64_t)j * n16;
            float* vn = h->Vm + (int64_t)(j + 1) * n16;
            CHK(precond_m(h, vj, zj));
            launch_spmm<double, float, double>(s, SPMV_AX, f.n_rows, f.np, f.rp, f.ci, f.Ap64, zj,
                                               nullptr, h->Wm, 0);
            launch_multidot16<float>(s, n16, j + 1, h->Vm, h->Wm, h->part, h->scal + M_H1);
            launch_multi_axpy16<float, double>(s, true, n16, j + 1, h->Vm, h->scal + M_H1, h->Wm);
            launch_multidot16<float>(s, n16, j + 1, h->Vm, h->Wm, h->part, h->scal + M_H2);
            launch_multi_axpy16<float, double>(s, true, n16, j + 1, h->Vm, h->scal + M_H2, h->Wm);
            launch_multidot16<double>(s, n16, 1, h->Wm, h->Wm, h->part, h->scal + M_HN);
            CHK(rd(h, M_HN, M_H2 + (j + 1) * 16 - M_HN));
            double est = 0.0;
            for (int c = 0; c < kNrhs; ++c) {
                const double hn = std::sqrt(h->h_scal[M_HN + c]);
                h->h_scal[M_SC + c] = 0.0;
                if (!live[c]) continue;
                double* Hc = H.data() + (size_t)c * (m + 1) * m;
                double* csc = cs.data() + (size_t)c * m;
                double* snc = sn.data() + (size_t)c * m;
                double* gc = g.data() + (size_t)c * (m + 1);
                for (int i = 0; i <= j; ++i)
                    Hc[i * m + j] = h->h_scal[M_H1 + i * 16 + c] + h->h_scal[M_H2 + i * 16 + c];
                Hc[(j + 1) * m + j] = hn;
                for (int i = 0; i < j; ++i) {
                    const double t = csc[i] * Hc[i * m + j] + snc[i] * Hc[(i + 1) * m + j];
                    Hc[(i + 1) * m + j] = -snc[i] * Hc[i * m + j] + csc[i] * Hc[(i + 1) * m + j];
                    Hc[i * m + j] = t;
                }
                const double den = std::hypot(Hc[j * m + j], Hc[(j + 1) * m + j]);
                if (!(den > 0.0)) {         // nothing left to reduce in this column
                    live[c] = false;
                    continue;
                }
                csc[j] = Hc[j * m + j] / den;
                snc[j] = Hc[(j + 1) * m + j] / den;
                Hc[j * m + j] = den;
                Hc[(j + 1) * m + j] = 0.0;
                gc[j + 1] = -snc[j] * gc[j];
                gc[j] = csc[j] * gc[j];
                jdone[c] = j + 1;
                const double e = std::fabs(gc[j + 1]) / nb[c];
                if (e <= rtol || hn == 0.0) live[c] = false;
                else h->h_scal[M_SC + c] = 1.0 / hn;
            }
            for (int c = 0; c < kNrhs; ++c)
                if (nb[c] > 0.0)
                    est = std::max(est, std::fabs(g[(size_t)c * (m + 1) + jdone[c]]) / nb[c]);
            ++k;
            *iters = k;
            jmax = j + 1;
            if (k < cap) hist[k] = est;
            bool any = false;
            for (int c = 0; c < kNrhs; ++c) any |= live[c];
            if (!any) break;
            CHK(wr(h, M_SC, 16));
            launch_scale16<float>(s, n16, h->Wm, h->scal + M_SC, vn);
        }
        // per column y = H^{-1} g, then X += sum_i y_i Z_i
        for (int i = 0; i < jmax; ++i)
            for (int c = 0; c < kNrhs; ++c) h->h_scal[M_CO + i * 16 + c] = 0.0;
        for (int c = 0; c < kNrhs; ++c) {
            const int jd = jdone[c];
            const double* Hc = H.data() + (size_t)c * (m + 1) * m;
            const double* gc = g.data() + (size_t)c * (m + 1);
            std::vector<double> y(jd);
            for (int i = jd - 1; i >= 0; --i) {
                double t = gc[i];
                for (int q = i + 1; q < jd; ++q) t -= Hc[i * m + q] * y[q];
                y[i] = t / Hc[i * m + i];
            }
            for (int i = 0; i < jd; ++i) h->h_scal[M_CO + i * 16 + c] = y[i];
        }
        if (jmax > 0) {
            CHK(wr(h, M_CO, jmax * 16));
            launch_multi_axpy16<float, double>(s, false, n16, jmax, h->Zm, h->scal + M_CO, X);
        }
        HIPCHK(hipGetLastError());
    }
}

}  // namespace xdg

extern "C" int xdg_spmm(xdg_handle* h, int32_t level, int32_t precision, const double* X,
                        double* Y) {
    if (!h || !X || !Y) return fail(XDG_EINVAL, "xdg_spmm: NULL argument");
    if (h->nrhs != kNrhs) return fail(XDG_EINVAL, "xdg_spmm: handle built for one column");
    if (level < 0 || level >= (int)h->L.size()) return fail(XDG_EINVAL, "level out of range");
    return mrhs_spmm(h, level, precision, X, Y);
}
