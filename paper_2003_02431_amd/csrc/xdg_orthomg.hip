// The paper's orthonormalisation multigrid as a solver (Section 3.3,
// Algorithms ResMinimi and OrthoMG): after the pre-smoother, after the
// coarse-grid correction and after the post-smoother the new direction z is
// added to the level's family Z, its image w = M z is made orthonormal to
// W = M Z (classical Gram-Schmidt, twice; z takes the same combination) and
// the iterate moves by (w . r) z, the least-residual point over the family.
// The coarse correction is one such cycle on the level below (x0 = 0), the
// coarsest level is solved directly; the top level loops until the relative
// residual reaches rtol and restarts its family (x0 := x) when `restart`
// directions would be exceeded.  The smoothers act on the current residual
// from zero (damped block Jacobi).
#include <hip/hip_runtime.h>

#include "xdg_handle.h"

namespace xdg {

namespace {

// device scalar slots (the Krylov solvers' slots end below 256)
constexpr int O_B1 = 1024, O_B2 = 1024 + 64, O_NRM = 1200, O_ALPHA = 1201, O_ONE = 1202,
              O_RR = 1203;

int om_rm(xdg_handle* h, int l, const double* z) {
    Level& lv = h->L[l];
    const int64_t n = lv.len();
    hipStream_t s = h->s;
    const int k = h->om_count[l];
    double* zk = h->omZ[l] + (int64_t)k * n;
    double* wk = h->omW[l] + (int64_t)k * n;
    HIPCHK(hipMemcpyAsync(zk, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    xdg::level_spmv<double>(h, lv, SPMV_AX, zk, nullptr, wk, 0);
    if (k > 0) {
        for (int pass = 0; pass < 2; ++pass) {
            double* beta = h->scal + (pass == 0 ? O_B1 : O_B2);
            launch_multidot(s, n, k, h->omW[l], wk, h->part, beta);
            launch_multi_axpy_neg(s, n, k, h->omW[l], beta, wk);
            launch_multi_axpy_neg(s, n, k, h->omZ[l], beta, zk);
        }
    }
    launch_dot(s, n, wk, wk, h->part, h->scal + O_NRM);
    launch_sqrt_scalar(s, h->scal, O_NRM);
    launch_div_scalar(s, n, h->scal, O_NRM, wk, wk);
    launch_div_scalar(s, n, h->scal, O_NRM, zk, zk);
    launch_dot(s, n, wk, h->omR[l], h->part, h->scal + O_ALPHA);
    // x += alpha z_k, r -= alpha w_k  (alpha = scal[O_ALPHA] / scal[O_ONE])
    launch_cg_update_xr(s, n, h->scal, O_ALPHA, O_ONE, zk, wk, h->omX[l], h->omR[l]);
    h->om_count[l] = k + 1;
    return XDG_OK;
}

int om_solve_level(xdg_handle* h, int l, const double* b);

// one pass of the loop body on level l (< coarsest): its x, r live in
// omX[l], omR[l], its family in omZ[l], omW[l]
int om_cycle(xdg_handle* h, int l) {
    Level& f = h->L[l];
    Level& c = h->L[l + 1];
    const int64_t n = f.len();
    hipStream_t s = h->s;
    // pre-smoother on the current residual
    HIPCHK(hipMemcpyAsync(f.b64, h->omR[l], n * sizeof(double), hipMemcpyDeviceToDevice, s));
    smooth_from_zero_fp64(h, f, h->opt.nu_pre);
    CHK(om_rm(h, l, f.x64));
    // coarse-grid correction: one cycle on the level below
    if (f.t_kind == XDG_T_PTRUNC)
        launch_restrict_trunc<double>(s, f.n_rows, f.np, c.np, h->omR[l], c.b64);
    else
        launch_restrict_dense<double>(s, c.n_rows, f.n_rows, f.np, c.np, f.chp, f.chi, f.ridx,
                                      f.R64, h->omR[l], c.b64, h->omT[l]);
    CHK(om_solve_level(h, l + 1, c.b64));
    HIPCHK(hipMemsetAsync(h->omT[l], 0, n * sizeof(double), s));
    if (f.t_kind == XDG_T_PTRUNC)
        launch_prolong_trunc<double>(s, f.n_rows, f.np, c.np, h->omX[l + 1], h->omT[l]);
    else
        launch_prolong_dense<double>(s, f.n_rows, f.np, c.np, f.parent, f.ridx, f.R64, h->omX[l + 1],
                                     h->omT[l]);
    CHK(om_rm(h, l, h->omT[l]));
    // post-smoother on the current residual
    HIPCHK(hipMemcpyAsync(f.b64, h->omR[l], n * sizeof(double), hipMemcpyDeviceToDevice, s));
    smooth_from_zero_fp64(h, f, h->opt.nu_post);
    CHK(om_rm(h, l, f.x64));
    return XDG_OK;
}

// omX[l] = OrthoMG(0, b) with one cycle; the direct solve on the coarsest
int om_solve_level(xdg_handle* h, int l, const double* b) {
    Level& lv = h->L[l];
    const int64_t n = lv.len();
    hipStream_t s = h->s;
    if (l == (int)h->L.size() - 1) {
        launch_coarse_gemv(s, h->cn, h->cld, h->Cinv, b, h->omX[l]);
        return XDG_OK;
    }
    HIPCHK(hipMemsetAsync(h->omX[l], 0, n * sizeof(double), s));
    HIPCHK(hipMemcpyAsync(h->omR[l], b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    h->om_count[l] = 0;
    return om_cycle(h, l);
}

}  // namespace

int orthomg_allocate(xdg_handle* h) {
    const int nl = (int)h->L.size();
    h->omZ.assign(nl, nullptr);
    h->omW.assign(nl, nullptr);
    h->omX.assign(nl, nullptr);
    h->omR.assign(nl, nullptr);
    h->omT.assign(nl, nullptr);
    h->om_count.assign(nl, 0);
    for (int l = 0; l < nl; ++l) {
        const int64_t n = h->L[l].len();
        CHK(h->alloc(&h->omX[l], n));
        if (l == nl - 1) break;
        const int cap = l == 0 ? h->opt.restart : 3;
        CHK(h->alloc(&h->omZ[l], (size_t)cap * n));
        CHK(h->alloc(&h->omW[l], (size_t)cap * n));
        CHK(h->alloc(&h->omR[l], n));
        CHK(h->alloc(&h->omT[l], n));
    }
    return XDG_OK;
}

int solve_orthomg(xdg_handle* h, const double* b, double* x, double* hist, int cap, int* iters) {
    Level& f = h->L[0];
    const int64_t n = f.len();
    const int nl = (int)h->L.size();
    hipStream_t s = h->s;
    *iters = 0;
    h->h_scal[O_ONE] = 1.0;
    HIPCHK(hipMemcpyAsync(h->scal + O_ONE, h->h_scal + O_ONE, sizeof(double),
                          hipMemcpyHostToDevice, s));
    launch_dot(s, n, b, b, h->part, h->scal + O_RR);
    HIPCHK(hipMemcpyAsync(h->h_scal + O_RR, h->scal + O_RR, sizeof(double),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double nb = std::sqrt(h->h_scal[O_RR]);
    if (!std::isfinite(nb)) return fail(XDG_EINVAL, "xdg_solve: non-finite right-hand side");
    if (nb == 0.0) {
        HIPCHK(hipMemsetAsync(x, 0, n * sizeof(double), s));
        if (cap > 0) hist[0] = 0.0;
        return XDG_OK;
    }
    if (nl == 1) {                     // a single level: the direct solve
        launch_coarse_gemv(s, h->cn, h->cld, h->Cinv, b, x);
        *iters = 1;
        if (cap > 1) hist[1] = 0.0;
        return XDG_OK;
    }
    // the top level works on the caller's x (restored on every return path)
    struct Restore {
        xdg_handle* h;
        double* p;
        ~Restore() { h->omX[0] = p; }
    } restore{h, h->omX[0]};
    h->omX[0] = x;
    int rc = XDG_ENOCONV;
    xdg::level_spmv<double>(h, f, SPMV_RESID, x, b, h->omR[0], 0);
    h->om_count[0] = 0;
    for (int k = 0;; ++k) {
        launch_dot(s, n, h->omR[0], h->omR[0], h->part, h->scal + O_RR);
        HIPCHK(hipMemcpyAsync(h->h_scal + O_RR, h->scal + O_RR, sizeof(double),
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(hipGetLastError());
        const double rel = std::sqrt(h->h_scal[O_RR]) / nb;
        if (!std::isfinite(rel)) return fail(XDG_EINVAL, "xdg_solve: non-finite residual");
        if (k < cap) hist[k] = rel;
        *iters = k;
        if (rel <= h->opt.rtol) {
            rc = XDG_OK;
            break;
        }
        if (k >= h->opt.maxit) break;
        if (h->om_count[0] + 3 > h->opt.restart) h->om_count[0] = 0;   // restart: x0 := x
        CHK(om_cycle(h, 0));
    }
    return rc;
}

}  // namespace xdg
