// Internal launch interface of libxdg (not part of the public C-ABI).
//
// Device layouts (chosen for gfx950 wave64 access):
//   * BSR blocks are stored column-major inside each block:
//       A[b*np*np + c*np + r] = M[m(i, r), m(col_idx[b], c)]
//     so that for a fixed block column c the np entries of the column are
//     contiguous; a wavefront processes floor(64/np) columns per load, one
//     contiguous run of floor(64/np)*np elements.
//   * cell-block inverses D_c^{-1}: dense, column-major, n_c x n_c, n_c =
//     rows_in_cell * np, concatenated; doff[c] is the element offset.
//   * vectors: [block row][mode].
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace xdg {

constexpr int kMaxCell = 88;       // largest smoother cell block order (88^2 FP64 fit 64 KB LDS)
constexpr int kCoarseNB = 32;      // tile of the blocked coarse inversion
constexpr int kMaxTransferModes = 8;  // coarse modes held in registers by the restriction
constexpr int kMaxDenseCoarse = 35;   // coarse modes of a dense (aggregation) transfer

enum SpmvMode { SPMV_AX = 0, SPMV_RESID = 1, SPMV_RESID_TRUNC = 2, SPMV_AX_DOT = 3 };

// ---- level operators (k_level.hip) -------------------------------------
// rev: visit the block rows (cells) in descending order.  Consecutive
// streaming passes over one level alternate it, so that each pass starts
// where the previous one ended, on the blocks still held in the memory-side
// (Infinity) cache.  Results do not depend on it (rows and cells are
// independent), except the per-workgroup partials of launch_spmv_dot, which
// are added in launch order.
// yfull (SPMV_RESID_TRUNC, Np = 20 or 35): also keep the whole residual there
template <typename T>
void launch_spmv(hipStream_t s, int mode, int n_rows, int np, const int* rp, const int* ci,
                 const T* A, const T* x, const T* b, T* y, int npc, bool rev = false,
                 T* yfull = nullptr);
template <typename T>
void launch_jacobi(hipStream_t s, bool first, int n_cells, int np, const int* cell_ptr,
                   const int* rp, const int* ci, const T* A, const int64_t* doff, const T* D,
                   const T* b, const T* xin, T* xout, T omega, bool rev = false);
template <typename T>
void launch_restrict_trunc(hipStream_t s, int n_rows, int npf, int npc, const T* rf, T* rc);
template <typename T>
void launch_prolong_trunc(hipStream_t s, int n_rows, int npf, int npc, const T* xc, T* xf);
// rc = R^T rf over the children lists; coarse blocks of more than
// kMaxTransferModes modes go through tmp (n_f * npc entries: R_i^T rf_i per
// fine row, then the children sums)
// (transfer blocks: fine row i uses R + ridx[i] * npf * npc, a table of the
// distinct R_i blocks)
template <typename T>
void launch_restrict_dense(hipStream_t s, int n_c, int n_f, int npf, int npc,
                           const int* child_ptr, const int* child_idx, const int* ridx,
                           const T* R, const T* rf, T* rc, T* tmp);
template <typename T>
void launch_prolong_dense(hipStream_t s, int n_f, int npf, int npc, const int* parent,
                          const int* ridx, const T* R, const T* xc, T* xf);
void launch_coarse_gemv(hipStream_t s, int n, int ld, const double* Ainv, const double* r,
                        double* z);
bool launch_spmv_dot(hipStream_t s, int n_rows, int np, const int* rp, const int* ci,
                     const double* A, const double* x, double* y, double* partial, double* out,
                     bool rev = false);

// Symmetric level matrix kept as its diagonal and upper blocks (column >= row):
// row i's upper blocks are urp[i] .. urp[i+1]-1 (columns uci, column-major
// blocks A, row by row); its lower blocks (i, j), j < i, are listed in
// lrp[i] .. lrp[i+1]-1 with the column j (lci) and the index in A of the
// stored block (j, i) (lidx), whose transpose they are.  Kernels exist for
// kSymNp modes per block.
constexpr int kSymNp = 20;
template <typename T>
struct SymRows {
    const int *urp = nullptr, *uci = nullptr, *lrp = nullptr, *lci = nullptr, *lidx = nullptr;
    const T* A = nullptr;
};
template <typename T>
void launch_spmv_sym(hipStream_t s, int mode, int n_rows, const SymRows<T>& m, const T* x,
                     const T* b, T* y, int npc, bool rev, T* yfull = nullptr);
void launch_spmv_dot_sym(hipStream_t s, int n_rows, const SymRows<double>& m, const double* x,
                         double* y, double* partial, double* out, bool rev);
// x_in given (not the first sweep from zero)
template <typename T>
void launch_jacobi_sym(hipStream_t s, int n_cells, const int* cp, const SymRows<T>& m,
                       const int64_t* doff, const T* D, const T* b, const T* xin, T* xout,
                       T omega, bool rev);
// First post sweep after a p-coarse correction e (npc leading modes per row):
// x_out = x1 + P e + omega D^-1 (r1 - (M P) e), r1 = b - M x1 kept by the
// residual pass, AP the leading npc columns of every block (np x npc
// column-major, the level's pattern).  cc_supported: block sizes with the kernel.
bool cc_supported(int np, int npc);
template <typename T>
void launch_jacobi_cc(hipStream_t s, int n_cells, int np, int npc, const int* cp, const int* rp,
                      const int* ci, const T* AP, const int64_t* doff, const T* D, const T* r1,
                      const T* x1, const T* e, T* xout, T omega, bool rev);
// First post sweep after an aggregation coarse correction e (npc modes per
// coarse row): x_out = x1 + R e + omega D^-1 (r1 - (M R) e) on small blocks,
// (M R) in BSR form (row pointer arp, coarse columns arc, np x npc blocks,
// column-major); cc_dense_supported: block sizes with the kernel.
bool cc_dense_supported(int np, int npc);
template <typename T>
void launch_jacobi_cc_g(hipStream_t s, int n_cells, int np, int npc, const int* cp,
                        const int* arp, const int* arc, const T* AR, const int64_t* doff,
                        const T* D, const T* r1, const T* x1, const T* e, const int* parent,
                        const int* ridx, const T* R, T* xout, T omega);
// (M R) blocks: block k sums M_b R_j over the fine blocks b = lb[lptr[k] ..
// lptr[k+1]-1] (column j = ci[b], transfer block ridx[j] of the table R)
template <typename Tout>
void launch_ar_product(hipStream_t s, int64_t n_ar, int np, int npc, const int* lptr,
                       const int* lb, const int* ci, const int* ridx, const double* A,
                       const double* R, Tout* AR);
// CG update (x += alpha p, r -= alpha q) fused with the first sweep from zero
// of the next V-cycle on level 0 (x1 = omega D^-1 r) and scal[i_rr] = r . r;
// false (nothing launched) for block sizes without the kernel (np 20, 35)
bool launch_cg_update_first(hipStream_t s, int n_cells, int np, const int* cp,
                            const int64_t* doff, const double* D, const double* scal, int i_rz,
                            int i_pq, int i_rr, const double* p, const double* q, double* x,
                            double* r, double* x1, double omega, double* partial);
// AP[b] = the first np*npc entries of block b (its leading npc columns)
template <typename Tout>
void launch_leading_columns(hipStream_t s, int64_t nnzb, int np, int npc, const double* A,
                            Tout* AP);
// out[k] = in[idx[k]] for blocks of bs entries (converted to Tout)
template <typename Tin, typename Tout>
void launch_gather_blocks(hipStream_t s, int64_t n, int bs, const int* idx, const Tin* in,
                          Tout* out);

// ---- setup (k_setup.hip) -------------------------------------------------
template <typename T>
void launch_transpose_blocks(hipStream_t s, int64_t nnzb, int np, const double* in, T* out);
void launch_extract_leading(hipStream_t s, int64_t nnzb, int npf, int npc, const double* A,
                            double* Ac, bool row_major = false);
// list == nullptr: every coarse block / cell 0..n-1; else the n listed ones
void launch_galerkin_dense(hipStream_t s, int n_cblk, int npf, int npc, const int* cptr,
                           const int* cfb, const int* ci_row, const int* ci_col,
                           const double* A, const double* R, double* Ac, const int* list);
// the same product for coarse blocks of more than 32 entries, in two passes
// over the fine-row groups of every coarse block (U: n_grp * npf * npc)
void launch_galerkin_wide(hipStream_t s, int n_grp, int n_cblk, int npf, int npc,
                          const int* gstart, const int* grow, const int* cbg, const int* cfb,
                          const int* ccol, const double* A, const double* R, double* U,
                          double* Ac);
void launch_gather_cells(hipStream_t s, int n_cells, int np, const int* cell_ptr,
                         const int* rp, const int* ci, const double* A, const int64_t* doff,
                         double* D, const int* list);
void launch_gj_batched(hipStream_t s, int n_mats, const int64_t* doff, const int* cell_ptr,
                       int np, int max_n, double* D, int* err, const int* list);
// row-major -> column-major layout and leading-mode extraction of listed blocks
void launch_transpose_list(hipStream_t s, int n, const int* list, int np, const double* in,
                           double* out);
void launch_extract_list(hipStream_t s, int n, const int* list, int npf, int npc,
                         const double* A, double* Ac);
void launch_bsr_to_dense(hipStream_t s, int n_rows, int np, const int* rp, const int* ci,
                         const double* A, int ld, int npad, double* dense);
void launch_coarse_gj_step(hipStream_t s, int nt, int K, int ld, double* A, double* P,
                           int* err);
template <typename Tin, typename Tout>
void launch_convert(hipStream_t s, int64_t n, const Tin* in, Tout* out);

// ---- vector kernels (k_blas.hip) -----------------------------------------
constexpr int kDotBlocks = 512;
// 16-column multi-dot: blocks of its partial pass and the largest number of
// basis vectors (restart <= 64); the partial buffer holds both layouts
constexpr int kDot16Blocks = 2048;
constexpr int kMaxBasis16 = 64;
// doubles of the handle's reduction-partial buffer (holds every layout above
// and one partial per workgroup of the fused product-and-inner-product)
constexpr size_t kPartDoubles = (size_t)kDot16Blocks * kMaxBasis16 * 16;
void launch_dot(hipStream_t s, int64_t n, const double* a, const double* b, double* partial,
                double* out);
void launch_cg_update_xr(hipStream_t s, int64_t n, const double* scal, int i_rz, int i_pq,
                         const double* p, const double* q, double* x, double* r);
// the same update and scal[i_rr] = r . r of the new r (the partial grid and
// order of launch_dot: the same value bit for bit)
void launch_cg_update_xr_dot(hipStream_t s, int64_t n, double* scal, int i_rz, int i_pq,
                             int i_rr, const double* p, const double* q, double* x, double* r,
                             double* partial);
// *out = sum of partial[0 .. np-1] in a fixed order
void launch_dot_final(hipStream_t s, const double* partial, int np, double* out);
void launch_cg_update_p(hipStream_t s, int64_t n, const double* scal, int i_new, int i_old,
                        const double* z, double* p);
void launch_fcg_update_p(hipStream_t s, int64_t n, const double* scal, int i_zq, int i_pq,
                         const double* z, double* p);
void launch_axpy(hipStream_t s, int64_t n, double a, const double* x, double* y);
template <typename T>
void launch_fill_zero(hipStream_t s, int64_t n, T* x);
void launch_scale_copy(hipStream_t s, int64_t n, double a, const double* x, double* y);

}  // namespace xdg

namespace xdg {
// multi-vector kernels for FGMRES (k_blas.hip): V is [nv][n] contiguous
void launch_multidot(hipStream_t s, int64_t n, int nv, const double* V, const double* w,
                     double* partial, double* out);
// w -= sum_k coef[k] V[k]   (coef in device memory)
void launch_multi_axpy_neg(hipStream_t s, int64_t n, int nv, const double* V, const double* coef,
                           double* w);
// x += sum_k coef[k] V[k]
void launch_multi_axpy(hipStream_t s, int64_t n, int nv, const double* V, const double* coef,
                       double* x);
// y = x / scal[i]
void launch_div_scalar(hipStream_t s, int64_t n, const double* scal, int i, const double* x,
                       double* y);
void launch_sqrt_scalar(hipStream_t s, double* scal, int i);
}  // namespace xdg

namespace xdg {
// ---- 16-column (multi-right-hand-side) kernels (k_mrhs.hip) ---------------
constexpr int kNrhs = 16;
bool mrhs_np_supported(int np);
template <typename TA, typename TX, typename TY>
void launch_spmm(hipStream_t s, int mode, int n_rows, int np, const int* rp, const int* ci,
                 const TA* Ap, const TX* X, const TY* B, TY* Y, int npc);
void launch_jacobi_mrhs(hipStream_t s, bool first, int n_cells, int np, const int* cp,
                        const int* rp, const int* ci, const float* Ap, const int64_t* doff,
                        const float* Dp, const float* B, const float* Xin, float* Xout,
                        float omega);
template <typename Tout>
void launch_pack_blocks(hipStream_t s, int64_t nblocks, int n, const double* in, Tout* out);
void launch_pack_cells(hipStream_t s, int n_cells, int np, const int* cp, const int64_t* doff,
                       const double* in, float* out);
template <typename T>
void launch_restrict_trunc_m(hipStream_t s, int n_rows, int npf, int npc, const T* rf, T* rc);
template <typename T>
void launch_prolong_trunc_m(hipStream_t s, int n_rows, int npf, int npc, const T* xc, T* xf);
template <typename T>
void launch_restrict_dense_m(hipStream_t s, int n_c, int npf, int npc, const int* cptr,
                             const int* cidx, const int* ridx, const T* R, const T* rf, T* rc);
template <typename T>
void launch_prolong_dense_m(hipStream_t s, int n_f, int npf, int npc, const int* parent,
                            const int* ridx, const T* R, const T* xc, T* xf);
void launch_coarse_gemm16(hipStream_t s, int n, int ld, const double* Ainv, const double* r,
                          double* z);
template <typename TV>
void launch_multidot16(hipStream_t s, int64_t n16, int nv, const TV* V, const double* w,
                       double* partial, double* out);
template <typename TV, typename TW>
void launch_multi_axpy16(hipStream_t s, bool neg, int64_t n16, int nv, const TV* V,
                         const double* coef, TW* w);
template <typename TO>
void launch_scale16(hipStream_t s, int64_t n16, const double* w, const double* sc, TO* out);
void launch_zero_cols16(hipStream_t s, int64_t n16, const double* keep, double* x);
}  // namespace xdg

namespace xdg {
// ---- learned smoother network (k_mlp.hip) ---------------------------------
int mlp_param_count();
void launch_mlp_forward(hipStream_t s, int n, const float* params, const float* X, float* Y);
void launch_mlp_grad(hipStream_t s, int n, int n_total, int n_blocks, const float* params,
                     const float* X, const float* T, float* partial, float* partial_loss,
                     float* grad, float* loss);
void launch_adam(hipStream_t s, float* w, const float* g, float* m, float* v, float lr, float b1,
                 float b2, float c1, float c2, float eps);
// bf16 inference: weights packed into MFMA operand tiles
int mlp_packed_bf16_count();
void launch_pack_bf16(hipStream_t s, const float* params, unsigned short* out);
void launch_learned_correct_bf16(hipStream_t s, int n_cells, const int* cp, const int* row_species,
                                 const float* geom, const unsigned short* wpk,
                                 const float* params, float guard, double* x, int* nguard);
// x holds j = omega D^{-1} b (the plain first sweep); adds the learned part
void launch_learned_correct(hipStream_t s, int n_cells, const int* cp, const int* row_species,
                            const float* geom, const float* params, float guard, double* x,
                            int* nguard);
void launch_learned_features(hipStream_t s, int n_sel, int cell0, int cell_step, const int* cp,
                             const int* row_species, const float* geom, const int64_t* doff,
                             const double* D, const double* r, const double* xk,
                             const double* xs, double omega, float clip, float* Xf, float* Tf);
}  // namespace xdg
