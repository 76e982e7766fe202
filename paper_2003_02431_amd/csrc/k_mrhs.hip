// Multi-right-hand-side (16 columns) block products on MFMA.
//
// With 16 right-hand sides the block product Y_i = sum_l M_il X_l is a dense
// contraction (Np x Np times Np x 16 per block, 8 flop per matrix byte in
// FP32), so it runs on the matrix cores: v_mfma_f32_16x16x4f32 for the FP32
// V-cycle and v_mfma_f64_16x16x4f64 for the FP64 products of the outer Krylov
// method.  Lane layout of both instructions (checked on gfx950):
//   A (16 x 4): lane l holds A[l % 16][l / 16]
//   B (4 x 16): lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l, register r holds D[i][l % 16] with
//                i = 4 (l / 16) + r for the FP32 instruction and
//                i = (l / 16) + 4 r for the FP64 instruction.
//
// Packed block layout ("row-tiled column-major"): the rows of an n x n block
// are cut into tiles of 16 (the last one has nr = n - 16 m rows); tile m is
// stored column-major with leading dimension nr at offset 16 m n:
//   P[16 m n + nr c + (i - 16 m)] = M[i][c].
// The A operand of tile m, k-step kk is then one contiguous run of 4 nr values.
// Multi-column vectors are [block row][mode][16].
#include "xdg_internal.h"

namespace xdg {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int uniform_m(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <typename T> struct Mfma;
template <> struct Mfma<float> {
    using acc_t = f32x4;
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    using acc_t = f64x4;
    static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

__host__ __device__ constexpr int tile_rows(int n, int m) { return n - 16 * m < 16 ? n - 16 * m : 16; }

// Y[row] = sum_b A_b X_col(b) for one block row; acc[m] accumulates row tile m.
// TA: matrix and accumulation type, TX: type of the stored X.  All operands
// of a block are loaded before its MFMAs, and the next block's operands are
// in flight while the current block is multiplied (register double buffer;
// skipped when the buffer would cost too many registers).
template <typename TA, typename TX, int NP>
__device__ __forceinline__ void fetch_block(const TA* __restrict__ Ab, const TX* __restrict__ Xb,
                                            int li, int lk, TA (&xv)[(NP + 3) / 4],
                                            TA (&av)[(NP + 3) / 4][(NP + 15) / 16]) {
    constexpr int MT = (NP + 15) / 16, KT = (NP + 3) / 4;
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) {
        const int k = 4 * kk + lk;
        const bool kv = k < NP;
        xv[kk] = kv ? (TA)Xb[k * 16 + li] : TA(0);
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int nr = tile_rows(NP, m);
            av[kk][m] = (kv && li < nr) ? Ab[16 * m * NP + nr * k + li] : TA(0);
        }
    }
}

template <typename TA, typename TX, int NP>
__device__ __forceinline__ void row_mma(int b0, int nb, const int* __restrict__ ci,
                                        const TA* __restrict__ Ap, const TX* __restrict__ X,
                                        int lane, typename Mfma<TA>::acc_t (&acc)[(NP + 15) / 16]) {
    constexpr int MT = (NP + 15) / 16, KT = (NP + 3) / 4;
    constexpr bool PF = sizeof(TA) * KT * (MT + 1) <= 128;
    const int li = lane & 15, lk = lane >> 4;
    const int colreg = lane < nb ? ci[b0 + lane] : 0;
    auto colof = [&](int b) {
        return b < 64 ? __builtin_amdgcn_readlane(colreg, b) : uniform_m(ci[b0 + b]);
    };
    TA xa[KT], aa[KT][MT];
    if (nb <= 0) return;
    fetch_block<TA, TX, NP>(Ap + (int64_t)b0 * (NP * NP), X + (int64_t)colof(0) * (NP * 16), li, lk,
                            xa, aa);
    for (int b = 0; b < nb; ++b) {
        TA xn[KT], an[KT][MT];
        if (PF && b + 1 < nb)
            fetch_block<TA, TX, NP>(Ap + (int64_t)(b0 + b + 1) * (NP * NP),
                                    X + (int64_t)colof(b + 1) * (NP * 16), li, lk, xn, an);
#pragma unroll
        for (int kk = 0; kk < KT; ++kk)
#pragma unroll
            for (int m = 0; m < MT; ++m) acc[m] = Mfma<TA>::mma(aa[kk][m], xa[kk], acc[m]);
        if (b + 1 < nb) {
            if (!PF)
                fetch_block<TA, TX, NP>(Ap + (int64_t)(b0 + b + 1) * (NP * NP),
                                        X + (int64_t)colof(b + 1) * (NP * 16), li, lk, xn, an);
#pragma unroll
            for (int kk = 0; kk < KT; ++kk) {
                xa[kk] = xn[kk];
#pragma unroll
                for (int m = 0; m < MT; ++m) aa[kk][m] = an[kk][m];
            }
        }
    }
}

// MODE 0: Y = A X; 1: Y = B - A X; 2: Yc[row][a < npc] = (B - A X)[row][a]
template <typename TA, typename TX, typename TY, int NP, int MODE>
__global__ __launch_bounds__(256) void k_spmm_mfma(int n_rows, const int* __restrict__ rp,
                                                   const int* __restrict__ ci,
                                                   const TA* __restrict__ Ap,
                                                   const TX* __restrict__ X,
                                                   const TY* __restrict__ B, TY* __restrict__ Y,
                                                   int npc) {
    constexpr int MT = (NP + 15) / 16;
    const int lane = threadIdx.x & 63;
    const int row = uniform_m(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (row >= n_rows) return;
    const int b0 = uniform_m(rp[row]), nb = uniform_m(rp[row + 1]) - b0;
    typename Mfma<TA>::acc_t acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = typename Mfma<TA>::acc_t{0, 0, 0, 0};
    row_mma<TA, TX, NP>(b0, nb, ci, Ap, X, lane, acc);
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * m + Mfma<TA>::row(lk, r);
            if (i < NP) {
                const int64_t o = ((int64_t)row * NP + i) * 16 + li;
                if (MODE == 0) Y[o] = (TY)acc[m][r];
                else if (MODE == 1) Y[o] = B[o] - (TY)acc[m][r];
                else if (i < npc) Y[((int64_t)row * npc + i) * 16 + li] = B[o] - (TY)acc[m][r];
            }
        }
    }
}

// X_out[I_c] = X_in[I_c] + omega D_c^{-1} res for a cell block of compile-time
// order NC (packed row-tiled D, res [NC][16] in LDS): every D operand of the
// block is loaded before the MFMAs so the loads overlap.
template <int NC, bool FIRST>
__device__ __forceinline__ void cell_apply_mrhs(const float* __restrict__ D, const float* res,
                                                int lane, int64_t base,
                                                const float* __restrict__ Xin,
                                                float* __restrict__ Xout, float omega) {
    constexpr int MT = (NC + 15) / 16, KT = (NC + 3) / 4;
    const int li = lane & 15, lk = lane >> 4;
    float av[KT][MT], rv[KT];
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) {
        const int k = 4 * kk + lk;
        const bool kv = k < NC;
        rv[kk] = kv ? res[k * 16 + li] : 0.f;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int nr = tile_rows(NC, m);
            av[kk][m] = (kv && li < nr) ? D[16 * m * NC + nr * k + li] : 0.f;
        }
    }
    f32x4 acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < KT; ++kk)
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = Mfma<float>::mma(av[kk][m], rv[kk], acc[m]);
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * m + Mfma<float>::row(lk, r);
            if (i < NC) {
                const int64_t o = base + (int64_t)i * 16 + li;
                Xout[o] = (FIRST ? 0.f : Xin[o]) + omega * acc[m][r];
            }
        }
}

// One damped block-Jacobi sweep on 16 columns, FP32, MFMA for both the
// residual rows and the cell-block inverse (packed, order n_c):
//   X_out[I_c] = X_in[I_c] + omega D_c^{-1} (B - M X_in)[I_c]
template <int NP, bool FIRST>
__global__ __launch_bounds__(256) void k_jacobi_mrhs(int n_cells, const int* __restrict__ cell_ptr,
                                                     const int* __restrict__ rp,
                                                     const int* __restrict__ ci,
                                                     const float* __restrict__ Ap,
                                                     const int64_t* __restrict__ doff,
                                                     const float* __restrict__ Dp,
                                                     const float* __restrict__ B,
                                                     const float* __restrict__ Xin,
                                                     float* __restrict__ Xout, float omega) {
    constexpr int MT = (NP + 15) / 16;
    constexpr int MTD = (kMaxCell + 15) / 16;
    __shared__ float res[4][kMaxCell * 16];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int cell = uniform_m(blockIdx.x * 4 + w);
    if (cell >= n_cells) return;
    const int r0 = uniform_m(cell_ptr[cell]), r1 = uniform_m(cell_ptr[cell + 1]);
    const int nc = (r1 - r0) * NP;
    for (int row = r0; row < r1; ++row) {
        f32x4 acc[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = f32x4{0, 0, 0, 0};
        if (!FIRST) {
            const int b0 = uniform_m(rp[row]), nb = uniform_m(rp[row + 1]) - b0;
            row_mma<float, float, NP>(b0, nb, ci, Ap, Xin, lane, acc);
        }
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * m + Mfma<float>::row(lk, r);
                if (i < NP) {
                    const int il = (row - r0) * NP + i;
                    res[w][il * 16 + li] = B[((int64_t)row * NP + i) * 16 + li] - acc[m][r];
                }
            }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const float* D = Dp + doff[cell];
    const int64_t base = (int64_t)r0 * NP * 16;
    if (nc == NP) {
        cell_apply_mrhs<NP, FIRST>(D, res[w], lane, base, Xin, Xout, omega);
    } else if (nc == 2 * NP) {
        cell_apply_mrhs<2 * NP, FIRST>(D, res[w], lane, base, Xin, Xout, omega);
    } else {
        const int mtd = (nc + 15) / 16, ktd = (nc + 3) / 4;
        f32x4 acc[MTD];
#pragma unroll
        for (int m = 0; m < MTD; ++m) acc[m] = f32x4{0, 0, 0, 0};
        for (int kk = 0; kk < ktd; ++kk) {
            const int k = 4 * kk + lk;
            const bool kv = k < nc;
            const float rv = kv ? res[w][k * 16 + li] : 0.f;
#pragma unroll
            for (int m = 0; m < MTD; ++m) {
                if (m < mtd) {
                    const int nr = tile_rows(nc, m);
                    const float av = (kv && li < nr) ? D[16 * m * nc + nr * k + li] : 0.f;
                    acc[m] = Mfma<float>::mma(av, rv, acc[m]);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < MTD; ++m) {
            if (m < mtd) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 16 * m + Mfma<float>::row(lk, r);
                    if (i < nc) {
                        const int64_t o = base + (int64_t)i * 16 + li;
                        Xout[o] = (FIRST ? 0.f : Xin[o]) + omega * acc[m][r];
                    }
                }
            }
        }
    }
}

// pack column-major n x n blocks (all of order n) into the row-tiled layout
template <typename Tout>
__global__ void k_pack_blocks(int64_t nblocks, int n, const double* __restrict__ in,
                              Tout* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n2 = (int64_t)n * n;
    if (t >= nblocks * n2) return;
    const int64_t b = t / n2;
    const int e = (int)(t - b * n2);
    const int c = e / n, i = e - c * n;      // input column-major
    const int m = i / 16;
    const int nr = tile_rows(n, m);
    out[b * n2 + 16 * m * n + nr * c + (i - 16 * m)] = (Tout)in[t];
}

// pack the cell-block inverses (orders vary; offsets doff shared with the source)
__global__ void k_pack_cells(int n_cells, int np, const int* __restrict__ cell_ptr,
                             const int64_t* __restrict__ doff, const double* __restrict__ in,
                             float* __restrict__ out) {
    const int c = blockIdx.x;
    if (c >= n_cells) return;
    const int n = (cell_ptr[c + 1] - cell_ptr[c]) * np;
    const double* src = in + doff[c];
    float* dst = out + doff[c];
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int col = e / n, i = e - col * n;
        const int m = i / 16;
        dst[16 * m * n + tile_rows(n, m) * col + (i - 16 * m)] = (float)src[e];
    }
}

// ---- 16-column transfers, coarse solve and vector kernels ---------------
template <typename T>
__global__ void k_prolong_trunc_m(int n_rows, int npf, int npc, const T* __restrict__ xc,
                                  T* __restrict__ xf) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_rows * npc * 16) return;
    const int64_t i = t / (npc * 16);
    const int rem = (int)(t - i * npc * 16);
    xf[i * npf * 16 + rem] += xc[t];
}

// rc[i][m][k] = rf[i][m][k] for the leading npc modes (p-truncation)
template <typename T>
__global__ void k_restrict_trunc_m(int n_rows, int npf, int npc, const T* __restrict__ rf,
                                   T* __restrict__ rc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_rows * npc * 16) return;
    const int64_t i = t / (npc * 16);
    const int rem = (int)(t - i * npc * 16);
    rc[t] = rf[i * npf * 16 + rem];
}

// rc[c][m][k] = sum_{i in children(c)} sum_a R_i[a][m] rf[i][a][k]
template <typename T>
__global__ void k_restrict_dense_m(int n_c, int npf, int npc, const int* __restrict__ child_ptr,
                                   const int* __restrict__ child_idx,
                                   const int* __restrict__ ridx, const T* __restrict__ R,
                                   const T* __restrict__ rf, T* __restrict__ rc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_c * npc * 16) return;
    const int c = (int)(t / (npc * 16));
    const int rem = (int)(t - (int64_t)c * npc * 16);
    const int m = rem >> 4, k = rem & 15;
    T acc = 0;
    for (int q = child_ptr[c]; q < child_ptr[c + 1]; ++q) {
        const int i = child_idx[q];
        const T* Ri = R + (int64_t)ridx[i] * npf * npc;
        const T* ri = rf + (int64_t)i * npf * 16 + k;
        for (int a = 0; a < npf; ++a) acc += Ri[a * npc + m] * ri[a * 16];
    }
    rc[t] = acc;
}

// xf[i][a][k] += sum_m R_i[a][m] xc[parent(i)][m][k]
template <typename T>
__global__ void k_prolong_dense_m(int n_f, int npf, int npc, const int* __restrict__ parent,
                                  const int* __restrict__ ridx,
                                  const T* __restrict__ R, const T* __restrict__ xc,
                                  T* __restrict__ xf) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_f * npf * 16) return;
    const int i = (int)(t / (npf * 16));
    const int rem = (int)(t - (int64_t)i * npf * 16);
    const int a = rem >> 4, k = rem & 15;
    const T* Ri = R + ((int64_t)ridx[i] * npf + a) * npc;
    const T* xp = xc + (int64_t)parent[i] * npc * 16 + k;
    T acc = 0;
    for (int m = 0; m < npc; ++m) acc += Ri[m] * xp[m * 16];
    xf[t] += acc;
}

// z[row][k] = sum_j Ainv[row][j] r[j][k]; one wave per row, lane = (j group, k)
__global__ __launch_bounds__(256) void k_coarse_gemm16(int n, int ld, const double* __restrict__ Ainv,
                                                       const double* __restrict__ r,
                                                       double* __restrict__ z) {
    const int lane = threadIdx.x & 63;
    const int row = uniform_m(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (row >= n) return;
    const int k = lane & 15, jg = lane >> 4;
    const double* a = Ainv + (int64_t)row * ld;
    double acc = 0.0;
    for (int j = jg; j < n; j += 4) acc += a[j] * r[(int64_t)j * 16 + k];
    acc += __shfl_xor(acc, 16, 64);
    acc += __shfl_xor(acc, 32, 64);
    if (jg == 0) z[(int64_t)row * 16 + k] = acc;
}

// ---------------------------------------------------------------------------
static inline unsigned nb_(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename TA, typename TX, typename TY, int MODE>
static void spmm_np(hipStream_t s, int n_rows, int np, const int* rp, const int* ci, const TA* Ap,
                    const TX* X, const TY* B, TY* Y, int npc) {
    dim3 g(nb_(n_rows, 4)), blk(256);
    switch (np) {
#define XDG_NP(N) \
    case N: k_spmm_mfma<TA, TX, TY, N, MODE><<<g, blk, 0, s>>>(n_rows, rp, ci, Ap, X, B, Y, npc); break;
        XDG_NP(1) XDG_NP(3) XDG_NP(4) XDG_NP(6) XDG_NP(10) XDG_NP(20) XDG_NP(35)
#undef XDG_NP
        default: break;
    }
}

template <typename TA, typename TX, typename TY>
void launch_spmm(hipStream_t s, int mode, int n_rows, int np, const int* rp, const int* ci,
                 const TA* Ap, const TX* X, const TY* B, TY* Y, int npc) {
    if (mode == SPMV_AX) spmm_np<TA, TX, TY, 0>(s, n_rows, np, rp, ci, Ap, X, B, Y, npc);
    else if (mode == SPMV_RESID) spmm_np<TA, TX, TY, 1>(s, n_rows, np, rp, ci, Ap, X, B, Y, npc);
    else spmm_np<TA, TX, TY, 2>(s, n_rows, np, rp, ci, Ap, X, B, Y, npc);
}

bool mrhs_np_supported(int np) {
    return np == 1 || np == 3 || np == 4 || np == 6 || np == 10 || np == 20 || np == 35;
}

template <bool FIRST>
static void jac_m_np(hipStream_t s, int n_cells, int np, const int* cp, const int* rp,
                     const int* ci, const float* Ap, const int64_t* doff, const float* Dp,
                     const float* B, const float* Xin, float* Xout, float omega) {
    dim3 g(nb_(n_cells, 4)), blk(256);
    switch (np) {
#define XDG_NP(N)                                                                             \
    case N:                                                                                   \
        k_jacobi_mrhs<N, FIRST><<<g, blk, 0, s>>>(n_cells, cp, rp, ci, Ap, doff, Dp, B, Xin, \
                                                   Xout, omega);                              \
        break;
        XDG_NP(1) XDG_NP(3) XDG_NP(4) XDG_NP(6) XDG_NP(10) XDG_NP(20) XDG_NP(35)
#undef XDG_NP
        default: break;
    }
}

void launch_jacobi_mrhs(hipStream_t s, bool first, int n_cells, int np, const int* cp,
                        const int* rp, const int* ci, const float* Ap, const int64_t* doff,
                        const float* Dp, const float* B, const float* Xin, float* Xout,
                        float omega) {
    if (first) jac_m_np<true>(s, n_cells, np, cp, rp, ci, Ap, doff, Dp, B, Xin, Xout, omega);
    else jac_m_np<false>(s, n_cells, np, cp, rp, ci, Ap, doff, Dp, B, Xin, Xout, omega);
}

template <typename Tout>
void launch_pack_blocks(hipStream_t s, int64_t nblocks, int n, const double* in, Tout* out) {
    k_pack_blocks<Tout><<<nb_(nblocks * n * n, 256), 256, 0, s>>>(nblocks, n, in, out);
}
void launch_pack_cells(hipStream_t s, int n_cells, int np, const int* cp, const int64_t* doff,
                       const double* in, float* out) {
    k_pack_cells<<<n_cells, 256, 0, s>>>(n_cells, np, cp, doff, in, out);
}
template <typename T>
void launch_prolong_trunc_m(hipStream_t s, int n_rows, int npf, int npc, const T* xc, T* xf) {
    k_prolong_trunc_m<T><<<nb_((int64_t)n_rows * npc * 16, 256), 256, 0, s>>>(n_rows, npf, npc, xc, xf);
}
template <typename T>
void launch_restrict_trunc_m(hipStream_t s, int n_rows, int npf, int npc, const T* rf, T* rc) {
    k_restrict_trunc_m<T><<<nb_((int64_t)n_rows * npc * 16, 256), 256, 0, s>>>(n_rows, npf, npc, rf, rc);
}
template <typename T>
void launch_restrict_dense_m(hipStream_t s, int n_c, int npf, int npc, const int* cptr,
                             const int* cidx, const int* ridx, const T* R, const T* rf, T* rc) {
    k_restrict_dense_m<T><<<nb_((int64_t)n_c * npc * 16, 256), 256, 0, s>>>(n_c, npf, npc, cptr,
                                                                            cidx, ridx, R, rf,
                                                                            rc);
}
template <typename T>
void launch_prolong_dense_m(hipStream_t s, int n_f, int npf, int npc, const int* parent,
                            const int* ridx, const T* R, const T* xc, T* xf) {
    k_prolong_dense_m<T><<<nb_((int64_t)n_f * npf * 16, 256), 256, 0, s>>>(n_f, npf, npc, parent,
                                                                           ridx, R, xc, xf);
}
void launch_coarse_gemm16(hipStream_t s, int n, int ld, const double* Ainv, const double* r,
                          double* z) {
    k_coarse_gemm16<<<nb_(n, 4), 256, 0, s>>>(n, ld, Ainv, r, z);
}

template void launch_spmm<float, float, float>(hipStream_t, int, int, int, const int*, const int*,
                                               const float*, const float*, const float*, float*, int);
template void launch_spmm<double, float, double>(hipStream_t, int, int, int, const int*, const int*,
                                                 const double*, const float*, const double*,
                                                 double*, int);
template void launch_spmm<double, double, double>(hipStream_t, int, int, int, const int*,
                                                  const int*, const double*, const double*,
                                                  const double*, double*, int);
template void launch_pack_blocks<float>(hipStream_t, int64_t, int, const double*, float*);
template void launch_pack_blocks<double>(hipStream_t, int64_t, int, const double*, double*);
template void launch_prolong_trunc_m<float>(hipStream_t, int, int, int, const float*, float*);
template void launch_restrict_dense_m<float>(hipStream_t, int, int, int, const int*, const int*,
                                             const int*, const float*, const float*, float*);
template void launch_prolong_dense_m<float>(hipStream_t, int, int, int, const int*, const int*,
                                            const float*, const float*, float*);
// FP64 forms: the boundary's restriction / prolongation on 16-column vectors
template void launch_restrict_trunc_m<double>(hipStream_t, int, int, int, const double*, double*);
template void launch_prolong_trunc_m<double>(hipStream_t, int, int, int, const double*, double*);
template void launch_restrict_dense_m<double>(hipStream_t, int, int, int, const int*, const int*,
                                              const int*, const double*, const double*, double*);
template void launch_prolong_dense_m<double>(hipStream_t, int, int, int, const int*, const int*,
                                             const double*, const double*, double*);

}  // namespace xdg

namespace xdg {

// ---- 16-column vector kernels: column c of element e is e % 16 ------------
// partial[(k * gridDim + blk) * 16 + c] = sum over the block's slice of V_k * w
template <typename TV> struct Vec4;
template <> struct Vec4<float> {
    static __device__ __forceinline__ void load(const float* p, double (&v)[4]) {
        const float4 t = *reinterpret_cast<const float4*>(p);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    }
};
template <> struct Vec4<double> {
    static __device__ __forceinline__ void load(const double* p, double (&v)[4]) {
        const double2 t0 = *reinterpret_cast<const double2*>(p);
        const double2 t1 = *reinterpret_cast<const double2*>(p + 2);
        v[0] = t0.x; v[1] = t0.y; v[2] = t1.x; v[3] = t1.y;
    }
};

// partial[k][block][c] = sum over this block's elements e (column c = e % 16)
// of V_k[e] w[e].  Every thread takes 4 consecutive elements per step (16-byte
// loads; since the grid stride is a multiple of 16 a thread always sees the
// same 4 columns), and groups of kG basis vectors share one pass over w.
// Fixed-order sums: per thread ascending e, then a fixed block reduction.
template <typename TV>
__global__ __launch_bounds__(256) void k_multidot16_partial(int64_t n16, int nv,
                                                            const TV* __restrict__ V,
                                                            const double* __restrict__ w,
                                                            double* __restrict__ partial) {
    constexpr int kG = 8;
    __shared__ double sh[4][kG][16];
    const int64_t n4 = n16 >> 2;
    const int lane = threadIdx.x & 63, wv_id = threadIdx.x >> 6;
    for (int k0 = 0; k0 < nv; k0 += kG) {
        const int g = min(kG, nv - k0);
        double acc[kG][4];
#pragma unroll
        for (int q = 0; q < kG; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[q][i] = 0.0;
        for (int64_t e4 = (int64_t)blockIdx.x * 256 + threadIdx.x; e4 < n4;
             e4 += (int64_t)gridDim.x * 256) {
            double wv[4];
            Vec4<double>::load(w + 4 * e4, wv);
#pragma unroll
            for (int q = 0; q < kG; ++q)
                if (q < g) {
                    double vv[4];
                    Vec4<TV>::load(V + (int64_t)(k0 + q) * n16 + 4 * e4, vv);
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[q][i] += vv[i] * wv[i];
                }
        }
        // lanes with the same lane % 4 hold the same 4 columns: fixed xor tree
        // over the other lane bits, then lanes 0..3 hold the wave's sums
#pragma unroll
        for (int q = 0; q < kG; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                double v = acc[q][i];
                for (int off = 4; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
                if (lane < 4) sh[wv_id][q][4 * lane + i] = v;
            }
        __syncthreads();
        if (threadIdx.x < 16 * g) {
            const int q = threadIdx.x >> 4, c = threadIdx.x & 15;
            const double s = ((sh[0][q][c] + sh[1][q][c]) + sh[2][q][c]) + sh[3][q][c];
            partial[((int64_t)(k0 + q) * gridDim.x + blockIdx.x) * 16 + c] = s;
        }
        __syncthreads();
    }
}

// out[k][c] = sum over the nb block partials, in a fixed order: thread
// t = 16 j + c sums blocks j, j + 16, ... of column c, then thread c adds the
// 16 part sums in order
__global__ __launch_bounds__(256) void k_multidot16_final(int nv, int nb,
                                                          const double* __restrict__ partial,
                                                          double* __restrict__ out) {
    __shared__ double sh[256];
    const int k = blockIdx.x, c = threadIdx.x & 15, j = threadIdx.x >> 4;
    if (k >= nv) return;
    double s = 0.0;
    for (int b = j; b < nb; b += 16) s += partial[((int64_t)k * nb + b) * 16 + c];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < 16) {
        double t = 0.0;
        for (int q = 0; q < 16; ++q) t += sh[q * 16 + c];
        out[k * 16 + c] = t;
    }
}

// w[e] -/+= sum_k coef[k][e % 16] V_k[e]; 4 consecutive elements per thread
template <typename TV, typename TW, bool NEG>
__global__ void k_multi_axpy16(int64_t n16, int nv, const TV* __restrict__ V,
                               const double* __restrict__ coef, TW* __restrict__ w) {
    const int64_t e4 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (4 * e4 >= n16) return;
    const int c0 = (int)((4 * e4) & 15);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < nv; ++k) {
        double vv[4];
        Vec4<TV>::load(V + (int64_t)k * n16 + 4 * e4, vv);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] += coef[k * 16 + c0 + i] * vv[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t e = 4 * e4 + i;
        w[e] = NEG ? (TW)((double)w[e] - acc[i]) : (TW)((double)w[e] + acc[i]);
    }
}

// out[e] = w[e] * s[e % 16]
template <typename TO>
__global__ void k_scale16(int64_t n16, const double* __restrict__ w, const double* __restrict__ s,
                          TO* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n16) out[e] = (TO)(w[e] * s[e & 15]);
}

template <typename TV>
void launch_multidot16(hipStream_t s, int64_t n16, int nv, const TV* V, const double* w,
                       double* partial, double* out) {
    k_multidot16_partial<TV><<<kDot16Blocks, 256, 0, s>>>(n16, nv, V, w, partial);
    k_multidot16_final<<<nv, 256, 0, s>>>(nv, kDot16Blocks, partial, out);
}
template <typename TV, typename TW>
void launch_multi_axpy16(hipStream_t s, bool neg, int64_t n16, int nv, const TV* V,
                         const double* coef, TW* w) {
    if (neg) k_multi_axpy16<TV, TW, true><<<nb_(n16 / 4, 256), 256, 0, s>>>(n16, nv, V, coef, w);
    else k_multi_axpy16<TV, TW, false><<<nb_(n16 / 4, 256), 256, 0, s>>>(n16, nv, V, coef, w);
}
template <typename TO>
void launch_scale16(hipStream_t s, int64_t n16, const double* w, const double* sc, TO* out) {
    k_scale16<TO><<<nb_(n16, 256), 256, 0, s>>>(n16, w, sc, out);
}

template void launch_multidot16<float>(hipStream_t, int64_t, int, const float*, const double*,
                                       double*, double*);
template void launch_multidot16<double>(hipStream_t, int64_t, int, const double*, const double*,
                                        double*, double*);
template void launch_multi_axpy16<float, double>(hipStream_t, bool, int64_t, int, const float*,
                                                 const double*, double*);
template void launch_scale16<float>(hipStream_t, int64_t, const double*, const double*, float*);

// x[e] = 0 where keep[e % 16] == 0 (in place)
__global__ void k_zero_cols16(int64_t n16, const double* __restrict__ keep, double* x) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n16 && keep[e & 15] == 0.0) x[e] = 0.0;
}
void launch_zero_cols16(hipStream_t s, int64_t n16, const double* keep, double* x) {
    k_zero_cols16<<<nb_(n16, 256), 256, 0, s>>>(n16, keep, x);
}

}  // namespace xdg
