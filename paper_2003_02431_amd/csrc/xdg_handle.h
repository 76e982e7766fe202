// Handle and level structures of libxdg shared by the single- and
// multi-right-hand-side host code (not part of the public C-ABI).
#pragma once
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "xdg.h"
#include "xdg_internal.h"

namespace xdg {
int fail(int code, const std::string& msg);
const std::string& last_error_text();
}  // namespace xdg
using xdg::fail;

#define HIPCHK(x)                                                                           \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess)                                                               \
            return fail(e_ == hipErrorOutOfMemory ? XDG_ENOMEM : XDG_EHIP,                  \
                        std::string(#x) + ": " + hipGetErrorString(e_));                    \
    } while (0)

#define CHK(x)                      \
    do {                            \
        int rc_ = (x);              \
        if (rc_ < 0) return rc_;    \
    } while (0)

namespace xdg {

struct Level {
    int n_rows = 0, np = 0, nnzb = 0, n_cells = 0, max_nc = 0;
    std::vector<int> h_rp, h_ci, h_cp;
    int *rp = nullptr, *ci = nullptr, *cp = nullptr;
    double* A64 = nullptr;
    float* A32 = nullptr;
    int64_t* doff = nullptr;
    int64_t dsize = 0;
    std::vector<int64_t> h_doff;
    double* D64 = nullptr;
    float* D32 = nullptr;
    // Galerkin contributions forming the next coarser level (dense transfers)
    int *g_ptr = nullptr, *g_fb = nullptr, *g_row = nullptr, *g_col = nullptr;
    std::vector<int> h_fb2cb;       // fine block -> the coarse block it contributes to
    // wide Galerkin (coarse blocks of more than 32 entries): fine-row groups of
    // the contribution lists, their fine row, the groups of every coarse block,
    // and the per-group products A R
    int n_grp = 0;
    int *g_gstart = nullptr, *g_grow = nullptr, *g_cbg = nullptr;
    double* g_U = nullptr;
    // partial update (built on first use): row of every block, cell of every
    // row, level 0: index of the transposed block (l, i) of block (i, l)
    std::vector<int> h_rob, h_cor, h_btr;
    std::vector<char> h_bmark, h_cmark;
    // transfer to the next coarser level
    int t_kind = -1, npc = 0, n_c = 0;
    int *parent = nullptr, *chp = nullptr, *chi = nullptr;
    // distinct transfer blocks R64 / R32 (the children of uncut aggregates
    // repeat 2^D blocks) and, per fine row, the index of its block
    int* ridx = nullptr;
    std::vector<int> h_ridx;
    int n_rblocks = 0;
    double* R64 = nullptr;
    float* R32 = nullptr;
    // work vectors
    double *b64 = nullptr, *x64 = nullptr, *y64 = nullptr, *r64 = nullptr;
    float *b32 = nullptr, *x32 = nullptr, *y32 = nullptr, *r32 = nullptr;
    // 16-column (multi-right-hand-side) data: packed FP32 blocks and inverses,
    // packed FP64 blocks (level 0), work vectors [row][mode][16]
    float *Ap32 = nullptr, *Dp32 = nullptr;
    double* Ap64 = nullptr;
    float *bm = nullptr, *xm = nullptr, *ym = nullptr, *rm = nullptr;
    double *bm64 = nullptr, *xm64 = nullptr;
    // symmetric storage (level 0 of single-column handles with kSymNp modes):
    // the diagonal and upper blocks As64 / As32 (ufull: their indices among
    // all blocks) and the row lists of SymRows
    bool sym = false;
    int64_t nnzb_u = 0;
    int *urp = nullptr, *uci = nullptr, *lrp = nullptr, *lci = nullptr, *lidx = nullptr;
    int* ufull = nullptr;
    double* As64 = nullptr;
    float* As32 = nullptr;
    // leading npc columns of every block (np x npc column-major, the level's
    // pattern) for the first post sweep after a p-coarse correction
    // (levels with a p-truncation below them and a kernel for the sizes)
    double* AP64 = nullptr;
    float* AP32 = nullptr;
    // (M R) for the first post sweep after an aggregation coarse correction
    // (small blocks): BSR pattern over the coarse columns, the fine blocks
    // summed into every block, values
    int n_ar = 0;
    int *arp = nullptr, *arc = nullptr, *ar_lptr = nullptr, *ar_lb = nullptr;
    double* AR64 = nullptr;
    float* AR32 = nullptr;
    // direction of the next streaming pass over this level's blocks
    // (alternates; reset at every public call so that results are repeatable)
    bool rev_next = false;
    bool next_dir() {
        const bool r = rev_next;
        rev_next = !r;
        return r;
    }
    int64_t len() const { return (int64_t)n_rows * np; }
};

template <typename T> struct P;
template <> struct P<double> {
    static double* A(Level& l) { return l.A64; }
    static double* D(Level& l) { return l.D64; }
    static double* R(Level& l) { return l.R64; }
    static double*& b(Level& l) { return l.b64; }
    static double*& x(Level& l) { return l.x64; }
    static double*& y(Level& l) { return l.y64; }
    static double*& r(Level& l) { return l.r64; }
    static double* AP(Level& l) { return l.AP64; }
    static double* AR(Level& l) { return l.AR64; }
    static SymRows<double> sym(Level& l) {
        SymRows<double> m;
        m.urp = l.urp; m.uci = l.uci; m.lrp = l.lrp; m.lci = l.lci; m.lidx = l.lidx;
        m.A = l.As64;
        return m;
    }
};
template <> struct P<float> {
    static float* A(Level& l) { return l.A32; }
    static float* D(Level& l) { return l.D32; }
    static float* R(Level& l) { return l.R32; }
    static float*& b(Level& l) { return l.b32; }
    static float*& x(Level& l) { return l.x32; }
    static float*& y(Level& l) { return l.y32; }
    static float*& r(Level& l) { return l.r32; }
    static float* AP(Level& l) { return l.AP32; }
    static float* AR(Level& l) { return l.AR32; }
    static SymRows<float> sym(Level& l) {
        SymRows<float> m;
        m.urp = l.urp; m.uci = l.uci; m.lrp = l.lrp; m.lci = l.lci; m.lidx = l.lidx;
        m.A = l.As32;
        return m;
    }
};

}  // namespace xdg

using xdg::Level;
using xdg::P;

struct xdg_handle {
    hipStream_t s = nullptr;
    hipStream_t s2 = nullptr;       // side stream of the numeric set-up
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_scal = nullptr;              // CG scalars copied to the host
    int dev = 0;                    // device current at xdg_create
    xdg_options opt{};
    std::vector<Level> L;
    int cn = 0, cld = 0;            // coarsest order, padded leading dimension
    double* Cinv = nullptr;
    int *h_stage = nullptr, *d_stage = nullptr;   // pinned / device lists of a partial update
    int64_t stage_len = 0;
    double* Pbuf = nullptr;         // pivot-tile inverses of the coarse inversion (two panels)
    double* scal = nullptr;         // device scalars
    double* part = nullptr;         // reduction partials
    double* h_scal = nullptr;       // pinned host mirror
    int* d_err = nullptr;
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *w = nullptr;
    double *V = nullptr, *Z = nullptr;
    std::vector<void*> allocs;
    double setup_ms = 0.0;
    bool mixed = false;
    int nrhs = 1;
    // 16-column Krylov space: FP32 V, Z [k][row][mode][16], FP64 W, R
    float *Vm = nullptr, *Zm = nullptr;
    double *Wm = nullptr, *Rm = nullptr;
    // learned smoother: network parameters, Adam moments, gradient buffers,
    // per-row species and per-cell geometry features of level 0
    float *mlp_w = nullptr, *mlp_m = nullptr, *mlp_v = nullptr, *mlp_g = nullptr;
    float *mlp_part = nullptr, *mlp_ploss = nullptr, *mlp_loss = nullptr;
    int mlp_blocks = 256;           // one 4-wave block per CU (register-bound)
    int64_t mlp_step = 0;
    int* row_species = nullptr;
    float* cell_geom = nullptr;
    int* d_nguard = nullptr;
    unsigned short* mlp_wbf = nullptr;   // bf16 MFMA operand tiles of the weights
    bool wbf_stale = true;               // parameters changed since the last packing
    // orthonormalisation multigrid: per level the family Z, W = M Z, the
    // iterate, its residual, a work vector, and the family size
    std::vector<double*> omZ, omW, omX, omR, omT;
    std::vector<int> om_count;
    // L2 re-projection from an earlier time level's space (xdg_set_projection):
    // pattern and column-major blocks on the device
    int proj_rows = 0, proj_cols = 0, proj_nnzb = 0;
    int *proj_rp = nullptr, *proj_ci = nullptr;
    double* proj_A = nullptr;
    float guard = 4.0f;             // |proposal| / |Jacobi step| above this: plain step
    // level 0's first pre-smoothing sweep of the next FP64 V-cycle already
    // done by the CG update (set by the solver, consumed by the cycle)
    bool x1_ready = false;
    bool learned_ready = false;     // weights and features present
    bool learned_off = false;       // solver-level fallback taken in this solve
    int learned_fallbacks = 0;      // solver-level fallbacks (all solves)

    template <typename T>
    int alloc(T** ptr, size_t n) {
        *ptr = nullptr;
        if (n == 0) n = 1;
        hipError_t e = hipMalloc((void**)ptr, n * sizeof(T));
        if (e != hipSuccess) {
            *ptr = nullptr;
            return fail(e == hipErrorOutOfMemory ? XDG_ENOMEM : XDG_EHIP,
                        std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        allocs.push_back((void*)*ptr);
        return XDG_OK;
    }
    // frees one allocation made by alloc()/upload() before the handle ends
    void release(void* p) {
        if (!p) return;
        auto it = std::find(allocs.begin(), allocs.end(), p);
        if (it != allocs.end()) allocs.erase(it);
        (void)hipFree(p);
    }
    template <typename T>
    int upload(T** ptr, const T* host, size_t n) {
        CHK(alloc(ptr, n));
        HIPCHK(hipMemcpyAsync(*ptr, host, n * sizeof(T), hipMemcpyHostToDevice, s));
        return XDG_OK;
    }
};


namespace xdg {
// multi-right-hand-side host code (xdg_mrhs.hip)
int mrhs_validate(const xdg_options* opt, int np0, const xdg_transfer* T, int n_levels);
int mrhs_allocate(xdg_handle* h);
int mrhs_numeric(xdg_handle* h);
int mrhs_spmm(xdg_handle* h, int level, int precision, const double* X, double* Y);
int mrhs_smooth(xdg_handle* h, int level, const double* B, double* X, int sweeps);
int mrhs_vcycle(xdg_handle* h, const double* R, double* Z);
int mrhs_solve(xdg_handle* h, const double* B, double* X, double* hist, int cap, int* iters,
               double* final_relres);
}  // namespace xdg

namespace xdg {
// block-Jacobi sweeps before / after the coarse correction on level l of the
// V-cycle (levels below the finest take nu_coarse when it is set)
inline int sweeps_pre(const xdg_handle* h, int l) {
    return l > 0 && h->opt.nu_coarse > 0 ? h->opt.nu_coarse : h->opt.nu_pre;
}
inline int sweeps_post(const xdg_handle* h, int l) {
    return l > 0 && h->opt.nu_coarse > 0 ? h->opt.nu_coarse : h->opt.nu_post;
}
// the level's operator on its storage (all blocks, or the symmetric upper
// blocks); every call flips the level's streaming direction
// (SPMV_RESID_TRUNC: yfull != nullptr also keeps the whole residual)
template <typename T>
void level_spmv(xdg_handle* h, Level& lv, int mode, const T* x, const T* b, T* y, int npc,
                T* yfull = nullptr);
// y = M x and *out = x . y on level 0 (fused where the block size allows)
void level_spmv_dot(xdg_handle* h, Level& lv, const double* x, double* y, double* out);
// one damped block-Jacobi sweep (first: x_in = 0, the matrix is not read)
template <typename T>
void level_jacobi(xdg_handle* h, Level& lv, bool first, const T* b, const T* xin, T* xout);
}  // namespace xdg

namespace xdg {
// orthonormalisation multigrid (xdg_orthomg.hip) and the FP64 smoother it uses
int orthomg_allocate(xdg_handle* h);
int solve_orthomg(xdg_handle* h, const double* b, double* x, double* hist, int cap, int* iters);
void smooth_from_zero_fp64(xdg_handle* h, Level& lv, int sweeps);
}  // namespace xdg

namespace xdg {
// learned smoother host code (xdg_mlp.hip)
constexpr double kLearnedStall = 0.99;    // FGMRES reduction factor that disables the network
int learned_validate(const xdg_options* opt, int np0);
bool learned_active(xdg_handle* h);
void learned_first_sweep(xdg_handle* h, Level& lv);
}  // namespace xdg
