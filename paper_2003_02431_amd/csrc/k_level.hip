// Level operators on the block-sparse XDG matrix: SpMV (Eq. GenericMatrixSystem),
// fused residual + p-restriction, damped block-Jacobi sweep, and the transfers
// R^{X,lambda} / (R^{X,lambda})^T (Eq. XDGrestrictionMatrix).
//
// Work mapping: one wavefront per block row (SpMV) or per smoother cell block
// (Jacobi).  Lane l of a wave owns output mode r = l % np of column group
// g = l / np; the G = 64/np groups walk the block columns c = g, g+G, ... so
// every load instruction of the wave reads one contiguous run of G*np matrix
// entries (blocks are column-major on the device).  The G partial sums of a
// mode are combined with cross-lane shuffles in a fixed order.
#include "xdg_internal.h"

namespace xdg {

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Sum over the G column groups: result valid in lanes 0..np-1.
template <typename T>
__device__ __forceinline__ T group_sum(T acc, int np, int G) {
    T tot = acc;
    for (int k = 1; k < G; ++k) tot += __shfl_down(acc, k * np, 64);
    return tot;
}

// (M x) restricted to block row `row`: partial sums per lane (see group_sum).
// NP > 0 is the compile-time block size; NP == 0 uses np_rt.
template <typename T, int NP>
__device__ __forceinline__ T row_times_x(int beg, int end, const int* __restrict__ ci,
                                         const T* __restrict__ A, const T* __restrict__ x,
                                         int lane, int np_rt) {
    const int np = NP ? NP : np_rt;
    const int G = 64 / np;
    const int r = lane % np;
    const int g = lane / np;
    T acc = 0;
    if (g < G) {
        for (int blk = beg; blk < end; ++blk) {
            const int col = uniform(ci[blk]);
            const T* Ab = A + (int64_t)blk * (np * np) + r;
            const T* xb = x + (int64_t)col * np;
            if constexpr (NP > 0) {
#pragma unroll
                for (int c0 = 0; c0 < NP; c0 += 64 / NP) {
                    const int c = c0 + g;
                    if (c < NP) acc += Ab[c * NP] * xb[c];
                }
            } else {
                for (int c = g; c < np; c += G) acc += Ab[c * np] * xb[c];
            }
        }
    }
    return acc;
}

template <typename T, int NP, int MODE>
__global__ __launch_bounds__(256) void k_bsr_spmv(int n_rows, int np_rt, const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const T* __restrict__ A,
                                                  const T* __restrict__ x,
                                                  const T* __restrict__ b, T* __restrict__ y,
                                                  int npc) {
    const int np = NP ? NP : np_rt;
    const int lane = threadIdx.x & 63;
    const int row = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (row >= n_rows) return;
    const int beg = uniform(rp[row]), end = uniform(rp[row + 1]);
    T acc = row_times_x<T, NP>(beg, end, ci, A, x, lane, np);
    acc = group_sum(acc, np, 64 / np);
    if (lane < np) {
        const int64_t o = (int64_t)row * np + lane;
        if (MODE == SPMV_AX) {
            y[o] = acc;
        } else if (MODE == SPMV_RESID) {
            y[o] = b[o] - acc;
        } else if (lane < npc) {
            y[(int64_t)row * npc + lane] = b[o] - acc;
        }
    }
}

// One damped block-Jacobi sweep for every cell block c:
//   x_out[I_c] = x_in[I_c] + omega D_c^{-1} (b - M x_in)[I_c]
// FIRST: x_in == 0, so the residual is b and no matrix row is read.
template <typename T, int NP, bool FIRST>
__global__ __launch_bounds__(256) void k_jacobi(int n_cells, int np_rt, const int* __restrict__ cell_ptr,
                                                const int* __restrict__ rp,
                                                const int* __restrict__ ci,
                                                const T* __restrict__ A,
                                                const int64_t* __restrict__ doff,
                                                const T* __restrict__ D,
                                                const T* __restrict__ b,
                                                const T* __restrict__ xin,
                                                T* __restrict__ xout, T omega) {
    __shared__ T res[4][kMaxCell];
    const int np = NP ? NP : np_rt;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int cell = uniform(blockIdx.x * 4 + w);
    if (cell >= n_cells) return;
    const int r0 = uniform(cell_ptr[cell]), r1 = uniform(cell_ptr[cell + 1]);
    const int nc = (r1 - r0) * np;
    for (int row = r0; row < r1; ++row) {
        T acc = 0;
        if (!FIRST) {
            acc = row_times_x<T, NP>(uniform(rp[row]), uniform(rp[row + 1]), ci, A, xin, lane, np);
            acc = group_sum(acc, np, 64 / np);
        }
        if (lane < np) res[w][(row - r0) * np + lane] = b[(int64_t)row * np + lane] - acc;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const T* Dc = D + doff[cell];
    const int64_t base = (int64_t)r0 * np;
    if (nc <= 64) {
        const int G2 = 64 / nc;
        const int o = lane % nc, g2 = lane / nc;
        T acc = 0;
        if (g2 < G2)
            for (int c = g2; c < nc; c += G2) acc += Dc[(int64_t)c * nc + o] * res[w][c];
        acc = group_sum(acc, nc, G2);
        if (lane < nc) xout[base + lane] = (FIRST ? T(0) : xin[base + lane]) + omega * acc;
    } else {
        for (int o = lane; o < nc; o += 64) {
            T acc = 0;
            for (int c = 0; c < nc; ++c) acc += Dc[(int64_t)c * nc + o] * res[w][c];
            xout[base + o] = (FIRST ? T(0) : xin[base + o]) + omega * acc;
        }
    }
}

template <typename T>
__global__ void k_restrict_trunc(int n_rows, int npf, int npc, const T* __restrict__ rf,
                                 T* __restrict__ rc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_rows * npc) return;
    const int64_t i = t / npc;
    const int a = (int)(t - i * npc);
    rc[t] = rf[i * npf + a];
}

template <typename T>
__global__ void k_prolong_trunc(int n_rows, int npf, int npc, const T* __restrict__ xc,
                                T* __restrict__ xf) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_rows * npc) return;
    const int64_t i = t / npc;
    const int a = (int)(t - i * npc);
    xf[i * npf + a] += xc[t];
}

// rc[c][m] = sum_{i in children(c)} sum_a R_i[a][m] rf[i][a]   (children in
// ascending order: a fixed summation order, no atomics)
template <typename T>
__global__ void k_restrict_dense(int n_c, int npf, int npc, const int* __restrict__ child_ptr,
                                 const int* __restrict__ child_idx, const T* __restrict__ R,
                                 const T* __restrict__ rf, T* __restrict__ rc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_c * npc) return;
    const int c = (int)(t / npc);
    const int m = (int)(t - (int64_t)c * npc);
    T acc = 0;
    for (int k = child_ptr[c]; k < child_ptr[c + 1]; ++k) {
        const int i = child_idx[k];
        const T* Ri = R + (int64_t)i * npf * npc;
        const T* ri = rf + (int64_t)i * npf;
        for (int a = 0; a < npf; ++a) acc += Ri[a * npc + m] * ri[a];
    }
    rc[t] = acc;
}

// xf[i][a] += sum_m R_i[a][m] xc[parent(i)][m]
template <typename T>
__global__ void k_prolong_dense(int n_f, int npf, int npc, const int* __restrict__ parent,
                                const T* __restrict__ R, const T* __restrict__ xc,
                                T* __restrict__ xf) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_f * npf) return;
    const int i = (int)(t / npf);
    const int a = (int)(t - (int64_t)i * npf);
    const T* Ri = R + (int64_t)i * npf * npc + a * npc;
    const T* xp = xc + (int64_t)parent[i] * npc;
    T acc = 0;
    for (int m = 0; m < npc; ++m) acc += Ri[m] * xp[m];
    xf[t] += acc;
}

// z = Ainv r, Ainv dense row-major (leading dimension ld); one wave per row,
// fixed-order lane partials then a shuffle tree.
__global__ __launch_bounds__(256) void k_coarse_gemv(int n, int ld, const double* __restrict__ Ainv,
                                                     const double* __restrict__ r,
                                                     double* __restrict__ z) {
    const int lane = threadIdx.x & 63;
    const int row = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (row >= n) return;
    const double* a = Ainv + (int64_t)row * ld;
    double acc = 0.0;
    for (int j = lane; j < n; j += 64) acc += a[j] * r[j];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) z[row] = acc;
}

// ---------------------------------------------------------------------------
// launchers

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T, int MODE>
static void spmv_np(hipStream_t s, int n_rows, int np, const int* rp, const int* ci, const T* A,
                    const T* x, const T* b, T* y, int npc) {
    dim3 g(nblk(n_rows, 4)), blk(256);
    switch (np) {
#define XDG_NP(N) \
    case N: k_bsr_spmv<T, N, MODE><<<g, blk, 0, s>>>(n_rows, np, rp, ci, A, x, b, y, npc); break;
        XDG_NP(1) XDG_NP(3) XDG_NP(4) XDG_NP(6) XDG_NP(10) XDG_NP(20) XDG_NP(35)
#undef XDG_NP
        default: k_bsr_spmv<T, 0, MODE><<<g, blk, 0, s>>>(n_rows, np, rp, ci, A, x, b, y, npc);
    }
}

template <typename T>
void launch_spmv(hipStream_t s, int mode, int n_rows, int np, const int* rp, const int* ci,
                 const T* A, const T* x, const T* b, T* y, int npc) {
    if (mode == SPMV_AX) spmv_np<T, SPMV_AX>(s, n_rows, np, rp, ci, A, x, b, y, npc);
    else if (mode == SPMV_RESID) spmv_np<T, SPMV_RESID>(s, n_rows, np, rp, ci, A, x, b, y, npc);
    else spmv_np<T, SPMV_RESID_TRUNC>(s, n_rows, np, rp, ci, A, x, b, y, npc);
}

template <typename T, bool FIRST>
static void jacobi_np(hipStream_t s, int n_cells, int np, const int* cp, const int* rp,
                      const int* ci, const T* A, const int64_t* doff, const T* D, const T* b,
                      const T* xin, T* xout, T omega) {
    dim3 g(nblk(n_cells, 4)), blk(256);
    switch (np) {
#define XDG_NP(N)                                                                       \
    case N:                                                                             \
        k_jacobi<T, N, FIRST><<<g, blk, 0, s>>>(n_cells, np, cp, rp, ci, A, doff, D, b, \
                                                 xin, xout, omega);                     \
        break;
        XDG_NP(1) XDG_NP(3) XDG_NP(4) XDG_NP(6) XDG_NP(10) XDG_NP(20) XDG_NP(35)
#undef XDG_NP
        default:
            k_jacobi<T, 0, FIRST><<<g, blk, 0, s>>>(n_cells, np, cp, rp, ci, A, doff, D, b, xin,
                                                     xout, omega);
    }
}

template <typename T>
void launch_jacobi(hipStream_t s, bool first, int n_cells, int np, const int* cp, const int* rp,
                   const int* ci, const T* A, const int64_t* doff, const T* D, const T* b,
                   const T* xin, T* xout, T omega) {
    if (first) jacobi_np<T, true>(s, n_cells, np, cp, rp, ci, A, doff, D, b, xin, xout, omega);
    else jacobi_np<T, false>(s, n_cells, np, cp, rp, ci, A, doff, D, b, xin, xout, omega);
}

template <typename T>
void launch_restrict_trunc(hipStream_t s, int n_rows, int npf, int npc, const T* rf, T* rc) {
    k_restrict_trunc<T><<<nblk((int64_t)n_rows * npc, 256), 256, 0, s>>>(n_rows, npf, npc, rf, rc);
}
template <typename T>
void launch_prolong_trunc(hipStream_t s, int n_rows, int npf, int npc, const T* xc, T* xf) {
    k_prolong_trunc<T><<<nblk((int64_t)n_rows * npc, 256), 256, 0, s>>>(n_rows, npf, npc, xc, xf);
}
template <typename T>
void launch_restrict_dense(hipStream_t s, int n_c, int npf, int npc, const int* cptr,
                           const int* cidx, const T* R, const T* rf, T* rc) {
    k_restrict_dense<T><<<nblk((int64_t)n_c * npc, 256), 256, 0, s>>>(n_c, npf, npc, cptr, cidx,
                                                                      R, rf, rc);
}
template <typename T>
void launch_prolong_dense(hipStream_t s, int n_f, int npf, int npc, const int* parent,
                          const T* R, const T* xc, T* xf) {
    k_prolong_dense<T><<<nblk((int64_t)n_f * npf, 256), 256, 0, s>>>(n_f, npf, npc, parent, R,
                                                                     xc, xf);
}
void launch_coarse_gemv(hipStream_t s, int n, int ld, const double* Ainv, const double* r,
                        double* z) {
    k_coarse_gemv<<<nblk(n, 4), 256, 0, s>>>(n, ld, Ainv, r, z);
}

#define XDG_INST(T)                                                                           \
    template void launch_spmv<T>(hipStream_t, int, int, int, const int*, const int*, const T*, \
                                 const T*, const T*, T*, int);                                 \
    template void launch_jacobi<T>(hipStream_t, bool, int, int, const int*, const int*,        \
                                   const int*, const T*, const int64_t*, const T*, const T*,   \
                                   const T*, T*, T);                                           \
    template void launch_restrict_trunc<T>(hipStream_t, int, int, int, const T*, T*);          \
    template void launch_prolong_trunc<T>(hipStream_t, int, int, int, const T*, T*);           \
    template void launch_restrict_dense<T>(hipStream_t, int, int, int, const int*, const int*, \
                                           const T*, const T*, T*);                            \
    template void launch_prolong_dense<T>(hipStream_t, int, int, int, const int*, const T*,    \
                                          const T*, T*);
XDG_INST(double)
XDG_INST(float)
#undef XDG_INST

}  // namespace xdg
