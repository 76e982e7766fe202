// Host code of the learned per-cell smoother: network parameters and Adam
// state on the device, the training loop, cell features, training pairs and
// the learned first sweep of the level-0 smoother.
#include <hip/hip_runtime.h>

#include "xdg_handle.h"

namespace xdg {

static int mlp_alloc(xdg_handle* h) {
    if (h->mlp_w) return XDG_OK;
    const int np = mlp_param_count();
    CHK(h->alloc(&h->mlp_w, np));
    CHK(h->alloc(&h->mlp_m, np));
    CHK(h->alloc(&h->mlp_v, np));
    CHK(h->alloc(&h->mlp_g, np));
    CHK(h->alloc(&h->mlp_part, (size_t)h->mlp_blocks * 4 * np));
    CHK(h->alloc(&h->mlp_ploss, (size_t)h->mlp_blocks * 4));
    CHK(h->alloc(&h->mlp_loss, 1));
    CHK(h->alloc(&h->d_nguard, 1));
    CHK(h->alloc(&h->mlp_wbf, mlp_packed_bf16_count()));
    HIPCHK(hipMemsetAsync(h->d_nguard, 0, sizeof(int), h->s));
    return XDG_OK;
}

static bool finite_f(const float* v, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

bool learned_active(xdg_handle* h) {
    return (h->opt.smoother == XDG_LEARNED || h->opt.smoother == XDG_LEARNED_BF16) &&
           h->learned_ready && !h->learned_off;
}

// First pre-smoothing sweep of level 0 from x = 0 with the network's proposal:
// the plain first sweep (x = omega D^{-1} b), then the per-cell correction
void learned_first_sweep(xdg_handle* h, Level& lv) {
    launch_jacobi<double>(h->s, true, lv.n_cells, lv.np, lv.cp, lv.rp, lv.ci, lv.A64, lv.doff,
                          lv.D64, lv.b64, nullptr, lv.x64, h->opt.omega);
    if (h->opt.smoother == XDG_LEARNED_BF16) {
        if (h->wbf_stale) {
            launch_pack_bf16(h->s, h->mlp_w, h->mlp_wbf);
            h->wbf_stale = false;
        }
        launch_learned_correct_bf16(h->s, lv.n_cells, lv.cp, h->row_species, h->cell_geom,
                                    h->mlp_wbf, h->mlp_w, h->guard, lv.x64, h->d_nguard);
        return;
    }
    launch_learned_correct(h->s, lv.n_cells, lv.cp, h->row_species, h->cell_geom, h->mlp_w,
                           h->guard, lv.x64, h->d_nguard);
}

// learned-smoother requirements on the handle's configuration
int learned_validate(const xdg_options* opt, int np0) {
    if (opt->smoother == XDG_JACOBI) return XDG_OK;
    if (opt->smoother != XDG_LEARNED && opt->smoother != XDG_LEARNED_BF16)
        return fail(XDG_EINVAL, "unknown smoother");
    if (np0 != 20 || opt->nrhs != 1 || opt->krylov != XDG_FGMRES ||
        opt->precision != XDG_FP64 || opt->nu_pre < 1)
        return fail(XDG_EINVAL,
                    "learned smoother needs np = 20, nrhs = 1, FGMRES, FP64 and nu_pre >= 1");
    return XDG_OK;
}

}  // namespace xdg

using namespace xdg;

extern "C" int32_t xdg_mlp_param_count(void) { return mlp_param_count(); }

extern "C" int xdg_mlp_set(xdg_handle* h, const float* params) {
    if (!h || !params) return fail(XDG_EINVAL, "xdg_mlp_set: NULL argument");
    const int np = mlp_param_count();
    CHK(mlp_alloc(h));
    HIPCHK(hipMemcpyAsync(h->mlp_w, params, np * sizeof(float), hipMemcpyHostToDevice, h->s));
    HIPCHK(hipMemsetAsync(h->mlp_m, 0, np * sizeof(float), h->s));
    HIPCHK(hipMemsetAsync(h->mlp_v, 0, np * sizeof(float), h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    h->mlp_step = 0;
    h->wbf_stale = true;
    h->learned_ready = h->row_species != nullptr;
    return XDG_OK;
}

extern "C" int xdg_mlp_get(xdg_handle* h, float* params) {
    if (!h || !params) return fail(XDG_EINVAL, "xdg_mlp_get: NULL argument");
    if (!h->mlp_w) return fail(XDG_EINVAL, "xdg_mlp_get: no network parameters set");
    HIPCHK(hipMemcpyAsync(params, h->mlp_w, mlp_param_count() * sizeof(float),
                          hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    return XDG_OK;
}

extern "C" int xdg_mlp_forward(xdg_handle* h, int32_t n, const float* X, float* Y) {
    if (!h || n < 0 || (n > 0 && (!X || !Y))) return fail(XDG_EINVAL, "xdg_mlp_forward: bad argument");
    if (!h->mlp_w) return fail(XDG_EINVAL, "xdg_mlp_forward: no network parameters set");
    if (n == 0) return XDG_OK;
    launch_mlp_forward(h->s, n, h->mlp_w, X, Y);
    HIPCHK(hipGetLastError());
    return XDG_OK;
}

extern "C" int xdg_mlp_gradient(xdg_handle* h, int32_t n, const float* X, const float* T,
                                float* grad, float* loss) {
    if (!h || n < 1 || !X || !T || !grad || !loss)
        return fail(XDG_EINVAL, "xdg_mlp_gradient: bad argument");
    if (!h->mlp_w) return fail(XDG_EINVAL, "xdg_mlp_gradient: no network parameters set");
    launch_mlp_grad(h->s, n, n, h->mlp_blocks, h->mlp_w, X, T, h->mlp_part, h->mlp_ploss, grad,
                    h->mlp_loss);
    HIPCHK(hipMemcpyAsync(loss, h->mlp_loss, sizeof(float), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    return XDG_OK;
}

extern "C" int xdg_mlp_train(xdg_handle* h, int32_t n, const float* X, const float* T,
                             int32_t batch, int32_t steps, float lr, float* loss_hist) {
    if (!h || !X || !T || batch < 1 || n < batch || steps < 0 || !(lr > 0.f))
        return fail(XDG_EINVAL, "xdg_mlp_train: bad argument");
    if (!h->mlp_w) return fail(XDG_EINVAL, "xdg_mlp_train: no network parameters set");
    const int nb = n / batch;
    const double b1 = 0.9, b2 = 0.999;
    for (int k = 0; k < steps; ++k) {
        const int64_t off = (int64_t)(k % nb) * batch;
        launch_mlp_grad(h->s, batch, batch, h->mlp_blocks, h->mlp_w, X + off * 45, T + off * 40,
                        h->mlp_part, h->mlp_ploss, h->mlp_g, h->mlp_loss);
        if (loss_hist)
            HIPCHK(hipMemcpyAsync(loss_hist + k, h->mlp_loss, sizeof(float),
                                  hipMemcpyDeviceToHost, h->s));
        const int64_t t = ++h->mlp_step;
        const float c1 = (float)(1.0 - std::pow(b1, (double)t));
        const float c2 = (float)(1.0 - std::pow(b2, (double)t));
        launch_adam(h->s, h->mlp_w, h->mlp_g, h->mlp_m, h->mlp_v, lr, (float)b1, (float)b2, c1, c2,
                    1e-8f);
    }
    if (steps > 0) h->wbf_stale = true;
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->s));
    return XDG_OK;
}

extern "C" int xdg_set_cell_features(xdg_handle* h, const int32_t* row_species,
                                     const float* cell_geom) {
    if (!h || !row_species || !cell_geom)
        return fail(XDG_EINVAL, "xdg_set_cell_features: NULL argument");
    Level& f = h->L[0];
    if (f.np != 20) return fail(XDG_EINVAL, "xdg_set_cell_features: needs np = 20 on level 0");
    for (int c = 0; c < f.n_cells; ++c) {
        const int r0 = f.h_cp[c], r1 = f.h_cp[c + 1];
        if (r1 - r0 < 1 || r1 - r0 > 2)
            return fail(XDG_EINVAL, "xdg_set_cell_features: a cell must hold 1 or 2 rows");
        for (int r = r0; r < r1; ++r)
            if (row_species[r] != 0 && row_species[r] != 1)
                return fail(XDG_EINVAL, "xdg_set_cell_features: species must be 0 or 1");
        if (r1 - r0 == 2 && row_species[r0] == row_species[r0 + 1])
            return fail(XDG_EINVAL, "xdg_set_cell_features: two rows of one species in a cell");
    }
    if (!finite_f(cell_geom, (size_t)f.n_cells * 5))
        return fail(XDG_EINVAL, "xdg_set_cell_features: non-finite geometry value");
    if (!h->row_species) {
        CHK(h->alloc(&h->row_species, f.n_rows));
        CHK(h->alloc(&h->cell_geom, (size_t)f.n_cells * 5));
    }
    HIPCHK(hipMemcpyAsync(h->row_species, row_species, f.n_rows * sizeof(int),
                          hipMemcpyHostToDevice, h->s));
    HIPCHK(hipMemcpyAsync(h->cell_geom, cell_geom, (size_t)f.n_cells * 5 * sizeof(float),
                          hipMemcpyHostToDevice, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    h->learned_ready = h->mlp_w != nullptr;
    return XDG_OK;
}

extern "C" int xdg_learned_pairs(xdg_handle* h, const double* b, const double* xk,
                                 const double* xs, int32_t cell0, int32_t cell_step, float clip,
                                 float* X, float* T, int32_t* n_out) {
    if (!h || !b || !xk || !xs || !X || !T || !n_out)
        return fail(XDG_EINVAL, "xdg_learned_pairs: NULL argument");
    if (!(clip >= 0.f) || !std::isfinite(clip))
        return fail(XDG_EINVAL, "xdg_learned_pairs: clip must be finite and >= 0");
    if (!h->row_species) return fail(XDG_EINVAL, "xdg_learned_pairs: no cell features set");
    Level& f = h->L[0];
    if (cell0 < 0 || cell0 >= f.n_cells || cell_step < 1)
        return fail(XDG_EINVAL, "xdg_learned_pairs: bad cell selection");
    const int n_sel = (f.n_cells - cell0 + cell_step - 1) / cell_step;
    // residual of the iterate, then features and targets of the selected cells
    xdg::level_spmv<double>(h, f, SPMV_RESID, xk, b, h->w, 0);
    launch_learned_features(h->s, n_sel, cell0, cell_step, f.cp, h->row_species, h->cell_geom,
                            f.doff, f.D64, h->w, xk, xs, h->opt.omega, clip, X, T);
    HIPCHK(hipGetLastError());
    *n_out = n_sel;
    return XDG_OK;
}

extern "C" int xdg_set_smoother(xdg_handle* h, int32_t smoother, float guard) {
    if (!h) return fail(XDG_EINVAL, "xdg_set_smoother: NULL handle");
    if (!(guard > 0.f) || !std::isfinite(guard))
        return fail(XDG_EINVAL, "xdg_set_smoother: guard must be positive and finite");
    xdg_options o = h->opt;
    o.smoother = smoother;
    CHK(learned_validate(&o, h->L[0].np));
    h->opt.smoother = smoother;
    h->guard = guard;
    return XDG_OK;
}

extern "C" int xdg_learned_stats(xdg_handle* h, int64_t* guarded_cells, int32_t* fallbacks) {
    if (!h || !guarded_cells || !fallbacks) return fail(XDG_EINVAL, "xdg_learned_stats: NULL argument");
    int g = 0;
    if (h->d_nguard) {
        HIPCHK(hipMemcpyAsync(&g, h->d_nguard, sizeof(int), hipMemcpyDeviceToHost, h->s));
        HIPCHK(hipStreamSynchronize(h->s));
    }
    *guarded_cells = g;
    *fallbacks = h->learned_fallbacks;
    return XDG_OK;
}
