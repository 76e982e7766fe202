// Hierarchy set-up on the device:
//   * block layout change (row-major input blocks -> column-major device blocks)
//   * Galerkin coarse operators M^{lambda+1} = R^T M^lambda R (Eq. XDGsysRestriction):
//     p-levels keep the leading np_c x np_c sub-block of every block (R_i = [I;0]);
//     aggregation levels sum R_i^T M_il R_l over the fine blocks (i,l) that map to
//     one coarse block, in ascending fine-block order (no atomics)
//   * cell-block diagonal D_c gathered from the BSR and inverted in FP64 by
//     Gauss-Jordan elimination (pivots are the Schur-complement diagonals of an
//     SPD matrix, so no pivoting; a non-positive pivot reports "not SPD")
//   * coarsest matrix densified and inverted by blocked Gauss-Jordan (32x32 tiles)
#include "xdg_internal.h"

namespace xdg {

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// row-major blocks in, column-major blocks out, staged through LDS so that
// both the reads and the writes are contiguous (bpg blocks per group, at
// most 32 KB of LDS)
static inline int transpose_bpg(int np) {
    return std::max(1, std::min(8, 32768 / (np * np * (int)sizeof(double))));
}
template <typename T>
__global__ __launch_bounds__(256) void k_transpose_blocks(int64_t nnzb, int np, int bpg,
                                                          const double* __restrict__ in,
                                                          T* __restrict__ out) {
    extern __shared__ double tile[];
    const int nb2 = np * np;
    const int64_t b0 = (int64_t)blockIdx.x * bpg;
    const int nb = (int)min<int64_t>(bpg, nnzb - b0);
    const int64_t base = b0 * nb2;
    for (int e = threadIdx.x; e < nb * nb2; e += blockDim.x) tile[e] = in[base + e];
    __syncthreads();
    for (int e = threadIdx.x; e < nb * nb2; e += blockDim.x) {
        const int b = e / nb2, f = e - b * nb2;
        const int c = f / np, r = f - c * np;          // output: column-major
        out[base + e] = (T)tile[b * nb2 + r * np + c];
    }
}

// the same two layout steps for a list of blocks (one group per listed block)
__global__ __launch_bounds__(256) void k_transpose_list(int n, const int* __restrict__ list,
                                                        int np, const double* __restrict__ in,
                                                        double* __restrict__ out) {
    extern __shared__ double tile[];
    if ((int)blockIdx.x >= n) return;
    const int nb2 = np * np;
    const int64_t base = (int64_t)list[blockIdx.x] * nb2;
    for (int e = threadIdx.x; e < nb2; e += blockDim.x) tile[e] = in[base + e];
    __syncthreads();
    for (int e = threadIdx.x; e < nb2; e += blockDim.x) {
        const int c = e / np, r = e - c * np;
        out[base + e] = tile[r * np + c];
    }
}

__global__ __launch_bounds__(256) void k_extract_list(int n, const int* __restrict__ list,
                                                      int npf, int npc,
                                                      const double* __restrict__ A,
                                                      double* __restrict__ Ac) {
    if ((int)blockIdx.x >= n) return;
    const int64_t b = list[blockIdx.x];
    const int nc2 = npc * npc;
    for (int e = threadIdx.x; e < nc2; e += blockDim.x) {
        const int c = e / npc, r = e - c * npc;
        Ac[b * nc2 + e] = A[b * npf * npf + (int64_t)c * npf + r];
    }
}

// Ac = the leading npc x npc corner of every block (column-major out); the
// blocks of A are column-major, or row-major (the caller's level-0 values)
// when row_major is set
__global__ void k_extract_leading(int64_t nnzb, int npf, int npc, const double* __restrict__ A,
                                  double* __restrict__ Ac, int row_major) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nc2 = (int64_t)npc * npc;
    if (t >= nnzb * nc2) return;
    const int64_t b = t / nc2;
    const int e = (int)(t - b * nc2);
    const int c = e / npc, r = e - c * npc;
    Ac[t] = A[b * npf * npf + (row_major ? (int64_t)r * npf + c : (int64_t)c * npf + r)];
}

// (M R)_k for the blocks k = (i, J) of the aggregation-level product: sum over
// the listed fine blocks b = (i, j), parent(j) = J, of M_b R_j (np x npc,
// column-major out; M_b column-major, R_j row-major), in list order.  One
// thread per entry.
template <typename Tout>
__global__ void k_ar_product(int64_t n_ar, int np, int npc, const int* __restrict__ lptr,
                             const int* __restrict__ lb, const int* __restrict__ ci,
                             const int* __restrict__ ridx, const double* __restrict__ A,
                             const double* __restrict__ R, Tout* __restrict__ AR) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int w = np * npc;
    if (t >= n_ar * w) return;
    const int64_t k = t / w;
    const int e = (int)(t - k * w);
    const int c = e / np, r = e - c * np;
    double acc = 0.0;
    for (int q = lptr[k]; q < lptr[k + 1]; ++q) {
        const int b = lb[q];
        const double* Ab = A + (int64_t)b * np * np + r;
        const double* Rj = R + (int64_t)ridx[ci[b]] * np * npc + c;
        for (int kk = 0; kk < np; ++kk) acc += Ab[kk * np] * Rj[kk * npc];
    }
    AR[t] = (Tout)acc;
}

template <typename Tout>
void launch_ar_product(hipStream_t s, int64_t n_ar, int np, int npc, const int* lptr,
                       const int* lb, const int* ci, const int* ridx, const double* A,
                       const double* R, Tout* AR) {
    if (n_ar > 0)
        k_ar_product<Tout><<<nblk(n_ar * np * npc, 256), 256, 0, s>>>(n_ar, np, npc, lptr, lb, ci,
                                                                      ridx, A, R, AR);
}
template void launch_ar_product<double>(hipStream_t, int64_t, int, int, const int*, const int*,
                                        const int*, const int*, const double*, const double*,
                                        double*);
template void launch_ar_product<float>(hipStream_t, int64_t, int, int, const int*, const int*,
                                       const int*, const int*, const double*, const double*,
                                       float*);

// AP[b] = the leading npc columns of block b (column-major: its first
// np*npc entries)
template <typename Tout>
__global__ void k_leading_columns(int64_t nnzb, int np, int npc, const double* __restrict__ A,
                                  Tout* __restrict__ AP) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int w = np * npc;
    if (t >= nnzb * w) return;
    const int64_t b = t / w;
    AP[t] = (Tout)A[b * np * np + (t - b * w)];
}

// out[k] = in[idx[k]] block by block (the upper blocks of a symmetric level)
template <typename Tin, typename Tout>
__global__ void k_gather_blocks(int64_t n, int bs, const int* __restrict__ idx,
                                const Tin* __restrict__ in, Tout* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * bs) return;
    const int64_t k = t / bs;
    const int e = (int)(t - k * bs);
    out[t] = (Tout)in[(int64_t)idx[k] * bs + e];
}

// one workgroup per coarse block; thread (m, m2) of the block computes
// sum_k sum_a sum_b R_i[a][m] A_fb[a][b] R_l[b][m2]
__global__ __launch_bounds__(64) void k_galerkin_dense(int n_cblk, int npf, int npc,
                                                       const int* __restrict__ cptr,
                                                       const int* __restrict__ cfb,
                                                       const int* __restrict__ crow,
                                                       const int* __restrict__ ccol,
                                                       const double* __restrict__ A,
                                                       const double* __restrict__ R,
                                                       double* __restrict__ Ac,
                                                       const int* __restrict__ list) {
    __shared__ double part[64];
    if ((int)blockIdx.x >= n_cblk) return;
    const int cb = list ? list[blockIdx.x] : (int)blockIdx.x;
    const int nc2 = npc * npc;
    const int k0 = cptr[cb], k1 = cptr[cb + 1];
    auto term = [&](int k, int m, int m2) {
        const double* Ab = A + (int64_t)cfb[k] * npf * npf;      // column-major
        const double* Ri = R + (int64_t)crow[k] * npf * npc;
        const double* Rl = R + (int64_t)ccol[k] * npf * npc;
        double acc = 0.0;
        for (int b = 0; b < npf; ++b) {
            double s = 0.0;
            for (int a = 0; a < npf; ++a) s += Ri[a * npc + m] * Ab[b * npf + a];
            acc += s * Rl[b * npc + m2];
        }
        return acc;
    };
    if (nc2 > 32) {
        for (int t = threadIdx.x; t < nc2; t += blockDim.x) {
            const int m2 = t / npc, m = t - m2 * npc;
            double acc = 0.0;
            for (int k = k0; k < k1; ++k) acc += term(k, m, m2);
            Ac[(int64_t)cb * nc2 + t] = acc;
        }
        return;
    }
    // small coarse blocks: G groups of nc2 threads take every G-th fine
    // contribution; the G partial sums are added in group order
    const int G = 64 / nc2;
    const int g = threadIdx.x / nc2, t = threadIdx.x - g * nc2;
    double acc = 0.0;
    if (g < G) {
        const int m2 = t / npc, m = t - m2 * npc;
        for (int k = k0 + g; k < k1; k += G) acc += term(k, m, m2);
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < nc2) {
        double sum = 0.0;
        for (int q = 0; q < G; ++q) sum += part[q * nc2 + threadIdx.x];
        Ac[(int64_t)cb * nc2 + threadIdx.x] = sum;
    }
}

// Wide Galerkin product in two passes (one wave per item, wave-private LDS,
// no workgroup barriers), for aggregation levels that keep the fine degree.
// The contributions of a coarse block (I, L) that share a fine row i form a
// group g;  pass 1:  U_g = sum over the group's fine blocks (i, l), in list
// order, of A_il R_l;  pass 2:  C_IL = sum over the groups of (I, L), in order,
// of R_i^T U_g.  Either pass streams each operand once per use.
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kWideQ = 20;     // outputs per lane: 64 * 20 >= 35 * 35

__global__ __launch_bounds__(256) void k_galerkin_u(int n_grp, int npf, int npc,
                                                    const int* __restrict__ gstart,
                                                    const int* __restrict__ cfb,
                                                    const int* __restrict__ ccol,
                                                    const double* __restrict__ A,
                                                    const double* __restrict__ R,
                                                    double* __restrict__ U) {
    extern __shared__ double lds[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nf2 = npf * npf, nfc = npf * npc;
    double* sA = lds + (size_t)w * (nf2 + nfc);     // column-major npf x npf
    double* sR = sA + nf2;                           // row-major npf x npc
    const int g = (int)blockIdx.x * (int)(blockDim.x >> 6) + w;
    if (g >= n_grp) return;
    double u[kWideQ];
#pragma unroll
    for (int q = 0; q < kWideQ; ++q) u[q] = 0.0;
    for (int k = gstart[g]; k < gstart[g + 1]; ++k) {
        const double* Ab = A + (int64_t)cfb[k] * nf2;
        const double* Rl = R + (int64_t)ccol[k] * nfc;
        for (int e = lane; e < nf2; e += 64) sA[e] = Ab[e];
        for (int e = lane; e < nfc; e += 64) sR[e] = Rl[e];
        wave_sync_lds();
#pragma unroll
        for (int q = 0; q < kWideQ; ++q) {
            const int t = lane + 64 * q;
            if (t < nfc) {
                const int a = t / npc, m2 = t - a * npc;
                double v = 0.0;
                for (int b = 0; b < npf; ++b) v += sA[b * npf + a] * sR[b * npc + m2];
                u[q] += v;
            }
        }
        wave_sync_lds();
    }
#pragma unroll
    for (int q = 0; q < kWideQ; ++q) {
        const int t = lane + 64 * q;
        if (t < nfc) U[(int64_t)g * nfc + t] = u[q];
    }
}

__global__ __launch_bounds__(256) void k_galerkin_c(int n_cblk, int npf, int npc,
                                                    const int* __restrict__ cbg,
                                                    const int* __restrict__ grow,
                                                    const double* __restrict__ R,
                                                    const double* __restrict__ U,
                                                    double* __restrict__ Ac) {
    extern __shared__ double lds[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nfc = npf * npc, nc2 = npc * npc;
    double* sRi = lds + (size_t)w * 2 * nfc;
    double* sU = sRi + nfc;
    const int cb = (int)blockIdx.x * (int)(blockDim.x >> 6) + w;
    if (cb >= n_cblk) return;
    double c[kWideQ];
#pragma unroll
    for (int q = 0; q < kWideQ; ++q) c[q] = 0.0;
    for (int g = cbg[cb]; g < cbg[cb + 1]; ++g) {
        const double* Ri = R + (int64_t)grow[g] * nfc;
        const double* Ug = U + (int64_t)g * nfc;
        for (int e = lane; e < nfc; e += 64) {
            sRi[e] = Ri[e];
            sU[e] = Ug[e];
        }
        wave_sync_lds();
#pragma unroll
        for (int q = 0; q < kWideQ; ++q) {
            const int t = lane + 64 * q;
            if (t < nc2) {
                const int m2 = t / npc, m = t - m2 * npc;
                double v = 0.0;
                for (int a = 0; a < npf; ++a) v += sRi[a * npc + m] * sU[a * npc + m2];
                c[q] += v;
            }
        }
        wave_sync_lds();
    }
#pragma unroll
    for (int q = 0; q < kWideQ; ++q) {
        const int t = lane + 64 * q;
        if (t < nc2) Ac[(int64_t)cb * nc2 + t] = c[q];
    }
}

// D_c (column-major n_c x n_c) from the blocks (i, l) with i, l in cell c;
// entries not covered by a block stay at the caller's zero fill.
__global__ __launch_bounds__(256) void k_gather_cells(int n_cells, int np,
                                                      const int* __restrict__ cell_ptr,
                                                      const int* __restrict__ rp,
                                                      const int* __restrict__ ci,
                                                      const double* __restrict__ A,
                                                      const int64_t* __restrict__ doff,
                                                      double* __restrict__ D,
                                                      const int* __restrict__ list) {
    if ((int)blockIdx.x >= n_cells) return;
    const int c = list ? list[blockIdx.x] : (int)blockIdx.x;
    const int r0 = cell_ptr[c], r1 = cell_ptr[c + 1];
    const int nc = (r1 - r0) * np;
    double* Dc = D + doff[c];        // zero-filled by the caller (whole array) or here (list)
    if (list) {
        for (int e = threadIdx.x; e < nc * nc; e += blockDim.x) Dc[e] = 0.0;
        __syncthreads();
    }
    const int np2 = np * np;
    for (int row = r0; row < r1; ++row) {
        for (int blk = rp[row]; blk < rp[row + 1]; ++blk) {
            const int col = ci[blk];
            if (col < r0 || col >= r1) continue;
            const double* Ab = A + (int64_t)blk * np2;
            for (int e = threadIdx.x; e < np2; e += blockDim.x) {
                const int cc = e / np, rr = e - cc * np;
                Dc[(int64_t)((col - r0) * np + cc) * nc + (row - r0) * np + rr] = Ab[e];
            }
        }
    }
}

// In-place Gauss-Jordan inverse of an n x n column-major matrix held in LDS.
__device__ void gj_lds(double* a, int n, int* err) {
    for (int k = 0; k < n; ++k) {
        __syncthreads();
        const double piv = a[k * n + k];
        if (!(piv > 0.0)) {
            if (threadIdx.x == 0) *err = 1;
        }
        const double ip = 1.0 / piv;
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
            const int j = e / n, i = e - j * n;
            if (i != k && j != k) a[e] -= a[k * n + i] * a[j * n + k] * ip;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
            if (e != k) {
                a[e * n + k] *= ip;           // row k
                a[k * n + e] = -a[k * n + e] * ip;   // column k
            }
        }
        if (threadIdx.x == 0) a[k * n + k] = ip;
    }
    __syncthreads();
}

// The same elimination for a compile-time order N and 256 threads (constant
// index arithmetic, a fixed number of elements per thread).
template <int N>
__device__ void gj_lds_fixed(double* a, int* err) {
    constexpr int kPer = (N * N + 255) / 256;
    static_assert(N <= 256, "one thread per row/column entry in the scaling step");
    for (int k = 0; k < N; ++k) {
        __syncthreads();
        const double piv = a[k * N + k];
        if (!(piv > 0.0) && threadIdx.x == 0) *err = 1;
        const double ip = 1.0 / piv;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = (int)threadIdx.x + 256 * q;
            if (N * N % 256 == 0 || e < N * N) {
                const int j = e / N, i = e - j * N;
                if (i != k && j != k) a[e] -= a[k * N + i] * a[j * N + k] * ip;
            }
        }
        __syncthreads();
        const int e = threadIdx.x;
        if (e < N && e != k) {
            a[e * N + k] *= ip;                 // row k
            a[k * N + e] = -a[k * N + e] * ip;  // column k
        }
        if (threadIdx.x == 0) a[k * N + k] = ip;
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_gj_batched(int n_mats, const int64_t* __restrict__ doff,
                                                    const int* __restrict__ cell_ptr, int np,
                                                    double* __restrict__ D, int* err,
                                                    const int* __restrict__ list) {
    extern __shared__ double sm[];
    if ((int)blockIdx.x >= n_mats) return;
    const int c = list ? list[blockIdx.x] : (int)blockIdx.x;
    const int n = (cell_ptr[c + 1] - cell_ptr[c]) * np;
    double* Dc = D + doff[c];
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) sm[e] = Dc[e];
    if (n == 20)
        gj_lds_fixed<20>(sm, err);
    else if (n == 40)
        gj_lds_fixed<40>(sm, err);
    else
        gj_lds(sm, n, err);
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) Dc[e] = sm[e];
}

// dense row-major (leading dimension ld) copy of the coarsest level, padded
// with the identity up to npad rows
__global__ void k_bsr_to_dense(int n_rows, int np, const int* __restrict__ rp,
                               const int* __restrict__ ci, const double* __restrict__ A, int ld,
                               int npad, double* __restrict__ dense) {
    const int row = blockIdx.x;
    const int n = n_rows * np;
    if (row < n_rows) {
        const int np2 = np * np;
        for (int blk = rp[row]; blk < rp[row + 1]; ++blk) {
            const int col = ci[blk];
            for (int e = threadIdx.x; e < np2; e += blockDim.x) {
                const int cc = e / np, rr = e - cc * np;
                dense[(int64_t)(row * np + rr) * ld + col * np + cc] = A[(int64_t)blk * np2 + e];
            }
        }
    } else {
        // padding rows: identity (the single extra workgroup)
        for (int i = n + threadIdx.x; i < npad; i += blockDim.x) dense[(int64_t)i * ld + i] = 1.0;
    }
}

// ---- blocked Gauss-Jordan on the dense coarsest matrix (row-major) --------
constexpr int NB = kCoarseNB;

__device__ __forceinline__ void load_tile(double (*t)[NB + 1], const double* A, int ld, int I,
                                          int J) {
    for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
        const int r = e / NB, c = e - r * NB;
        t[r][c] = A[(int64_t)(I * NB + r) * ld + J * NB + c];
    }
}

// P = inverse of the pivot tile A_KK (one block; measured faster than
// one-wave variants with the tile in LDS or in registers, whose single
// dependency chain per step leaves the wave idle)
__global__ __launch_bounds__(256) void k_cgj_pivot(int K, int ld, const double* __restrict__ A,
                                                   double* __restrict__ P, int* err) {
    __shared__ double a[NB * NB];
    for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
        const int r = e / NB, c = e - r * NB;
        a[c * NB + r] = A[(int64_t)(K * NB + r) * ld + K * NB + c];   // column-major in LDS
    }
    gj_lds_fixed<NB>(a, err);
    for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
        const int r = e / NB, c = e - r * NB;
        P[e] = a[c * NB + r];                                          // row-major out
    }
}

// row K: A_KJ <- P A_KJ for J != K
__global__ __launch_bounds__(256) void k_cgj_row(int nt, int K, int ld, double* __restrict__ A,
                                                 const double* __restrict__ P) {
    __shared__ double p[NB][NB + 1], t[NB][NB + 1];
    const int J = blockIdx.x + (blockIdx.x >= (unsigned)K ? 1 : 0);
    for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) p[e / NB][e % NB] = P[e];
    load_tile(t, A, ld, K, J);
    __syncthreads();
    for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
        const int r = e / NB, c = e - r * NB;
        double s = 0.0;
        for (int k = 0; k < NB; ++k) s += p[r][k] * t[k][c];
        A[(int64_t)(K * NB + r) * ld + J * NB + c] = s;
    }
}

// ---- 32 x 32 tile products on the FP64 matrix cores ------------------------
// v_mfma_f64_16x16x4f64, lane layout (checked on gfx950): A operand (16 x 4)
// lane l holds A[l % 16][l / 16]; B operand (4 x 16) lane l holds
// B[l / 16][l % 16]; result (16 x 16) lane l, register r holds
// D[l / 16 + 4 r][l % 16].  A 32 x 32 tile is 2 x 2 such blocks; one wave
// multiplies two tiles in 8 k-steps of 4.  Row kk of the B operand of a
// product lives in the same lane and register (r = kk % 4 of block row
// kk / 4) as the result of the previous product, so chained products need
// no data movement.
typedef double cgj_f64x4 __attribute__((ext_vector_type(4)));

struct TileAcc {
    cgj_f64x4 d[2][2];
};

// D element (i, j) of the tile held by `lane`, register r of block (mi, nj)
__device__ __forceinline__ int tile_d_row(int lane, int mi, int r) { return 16 * mi + (lane >> 4) + 4 * r; }
__device__ __forceinline__ int tile_d_col(int lane, int nj) { return 16 * nj + (lane & 15); }

// acc (+)= sgn * X Y with X, Y 32 x 32 row-major at leading dimensions ldx, ldy
__device__ __forceinline__ void tile_mma(const double* __restrict__ X, int ldx,
                                         const double* __restrict__ Y, int ldy, double sgn,
                                         int lane, TileAcc& acc) {
    const int li = lane & 15, lk = lane >> 4;
    double a[8][2], b[8][2];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            a[kk][m] = sgn * X[(int64_t)(16 * m + li) * ldx + 4 * kk + lk];
            b[kk][m] = Y[(int64_t)(4 * kk + lk) * ldy + 16 * m + li];
        }
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int nj = 0; nj < 2; ++nj)
                acc.d[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk][mi], b[kk][nj],
                                                                     acc.d[mi][nj], 0, 0, 0);
}

__device__ __forceinline__ void tile_load(const double* __restrict__ T, int ld, int lane,
                                          TileAcc& acc) {
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc.d[mi][nj][r] = T[(int64_t)tile_d_row(lane, mi, r) * ld + tile_d_col(lane, nj)];
}

__device__ __forceinline__ void tile_store(double* __restrict__ T, int ld, int lane,
                                           const TileAcc& acc, double sgn) {
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                T[(int64_t)tile_d_row(lane, mi, r) * ld + tile_d_col(lane, nj)] =
                    sgn * acc.d[mi][nj][r];
}

__device__ __forceinline__ void tile_zero(TileAcc& acc) {
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) acc.d[mi][nj] = cgj_f64x4{0.0, 0.0, 0.0, 0.0};
}

// A_IJ <- A_IJ - A_IK A_KJ for I, J != K (row K already updated).  One wave
// per tile, four tiles (2 x 2 of the tile grid without row and column K) per
// group.  When a next panel exists, the group holding the pivot tile
// A_{K+1,K+1} is dispatched first and, after its update, inverts that tile
// into Pn (the next panel's P), so the pivot inversion overlaps the rest of
// the update.
__global__ __launch_bounds__(256) void k_cgj_update(int nt, int K, int ld, double* __restrict__ A,
                                                    double* __restrict__ Pn, int* err) {
    __shared__ double a[NB * NB];
    const int m = nt - 1;                  // tiles per dimension without K
    const int G = (m + 1) / 2;             // groups per dimension
    const bool next = K + 1 < nt;
    int g = blockIdx.x;
    const int gs = (K / 2) * G + K / 2;    // group of reduced tile (K, K) = tile (K+1, K+1)
    if (next) g = g == 0 ? gs : (g == gs ? 0 : g);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int Ip = 2 * (g / G) + (w >> 1), Jp = 2 * (g % G) + (w & 1);
    const bool pivot_group = next && g == gs;
    if (Ip < m && Jp < m) {
        const int I = Ip + (Ip >= K ? 1 : 0), J = Jp + (Jp >= K ? 1 : 0);
        double* Cij = A + (int64_t)(I * NB) * ld + J * NB;
        TileAcc acc;
        tile_load(Cij, ld, lane, acc);
        tile_mma(A + (int64_t)(I * NB) * ld + K * NB, ld, A + (int64_t)(K * NB) * ld + J * NB, ld,
                 -1.0, lane, acc);
        tile_store(Cij, ld, lane, acc, 1.0);
        if (pivot_group && I == K + 1 && J == K + 1) {
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int nj = 0; nj < 2; ++nj)
#pragma unroll
                    for (int r = 0; r < 4; ++r)          // column-major in LDS
                        a[tile_d_col(lane, nj) * NB + tile_d_row(lane, mi, r)] = acc.d[mi][nj][r];
        }
    }
    if (pivot_group) {                     // uniform over the group
        gj_lds_fixed<NB>(a, err);          // starts with a barrier
        for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
            const int r = e / NB, cc = e - r * NB;
            Pn[e] = a[cc * NB + r];                                // row-major out
        }
    }
}

// column K: A_IK <- -A_IK P for I != K ; A_KK <- P
__global__ __launch_bounds__(256) void k_cgj_col(int nt, int K, int ld, double* __restrict__ A,
                                                 const double* __restrict__ P) {
    __shared__ double p[NB][NB + 1], t[NB][NB + 1];
    const int I = blockIdx.x;
    for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) p[e / NB][e % NB] = P[e];
    if (I == K) {
        for (int e = threadIdx.x; e < NB * NB; e += blockDim.x)
            A[(int64_t)(K * NB + e / NB) * ld + K * NB + e % NB] = P[e];
        return;
    }
    load_tile(t, A, ld, I, K);
    __syncthreads();
    for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
        const int r = e / NB, c = e - r * NB;
        double s = 0.0;
        for (int k = 0; k < NB; ++k) s += t[r][k] * p[k][c];
        A[(int64_t)(I * NB + r) * ld + K * NB + c] = -s;
    }
}

// column K (with P = inverse of panel K's pivot) and row K+1 (with Pn, the
// next pivot inverse) in one launch, one wave per tile: waves 0..nt-1 do
// column K (A_IK <- -A_IK P; A_KK <- P) except tile (K+1, K); waves nt.. do
// row K+1 (A_{K+1,J} <- Pn A_{K+1,J}), and the wave of tile (K+1, K) first
// applies the column-K step to it, then the row-(K+1) step -- the order of
// separate launches.  The two steps touch no other common tile.
__global__ __launch_bounds__(64) void k_cgj_colrow(int nt, int K, int ld, double* __restrict__ A,
                                                   const double* __restrict__ P,
                                                   const double* __restrict__ Pn) {
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    TileAcc acc;
    tile_zero(acc);
    if (w < nt) {                              // column K
        const int I = w;
        if (I == K + 1) return;
        double* T = A + (int64_t)(I * NB) * ld + K * NB;
        if (I == K) {
            for (int e = lane; e < NB * NB; e += 64) T[(int64_t)(e / NB) * ld + e % NB] = P[e];
            return;
        }
        tile_mma(T, ld, P, NB, 1.0, lane, acc);
        tile_store(T, ld, lane, acc, -1.0);
        return;
    }
    const int jj = w - nt;                     // row K+1, J != K+1
    const int J = jj + (jj >= K + 1 ? 1 : 0);
    double* T = A + (int64_t)((K + 1) * NB) * ld + J * NB;
    if (J == K) {
        // t = -A_{K+1,K} P, then A_{K+1,K} <- Pn t; t stays in registers as
        // the B operand of the second product
        tile_mma(T, ld, P, NB, -1.0, lane, acc);
        const int li = lane & 15;
        double a[8][2];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
                a[kk][mi] = Pn[(16 * mi + li) * NB + 4 * kk + (lane >> 4)];
        TileAcc out;
        tile_zero(out);
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int nj = 0; nj < 2; ++nj)
                    out.d[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                        a[kk][mi], acc.d[kk / 4][nj][kk % 4], out.d[mi][nj], 0, 0, 0);
        tile_store(T, ld, lane, out, 1.0);
        return;
    }
    tile_mma(Pn, NB, T, ld, 1.0, lane, acc);
    tile_store(T, ld, lane, acc, 1.0);
}

template <typename Tin, typename Tout>
__global__ void k_convert(int64_t n, const Tin* __restrict__ in, Tout* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = (Tout)in[t];
}

// ---------------------------------------------------------------------------
template <typename T>
void launch_transpose_blocks(hipStream_t s, int64_t nnzb, int np, const double* in, T* out) {
    const int bpg = transpose_bpg(np);
    const size_t lds = (size_t)bpg * np * np * sizeof(double);
    k_transpose_blocks<T><<<nblk(nnzb, bpg), 256, lds, s>>>(nnzb, np, bpg, in, out);
}
template <typename Tout>
void launch_leading_columns(hipStream_t s, int64_t nnzb, int np, int npc, const double* A,
                            Tout* AP) {
    if (nnzb > 0)
        k_leading_columns<Tout><<<nblk(nnzb * np * npc, 256), 256, 0, s>>>(nnzb, np, npc, A, AP);
}
template void launch_leading_columns<double>(hipStream_t, int64_t, int, int, const double*,
                                             double*);
template void launch_leading_columns<float>(hipStream_t, int64_t, int, int, const double*,
                                            float*);
template <typename Tin, typename Tout>
void launch_gather_blocks(hipStream_t s, int64_t n, int bs, const int* idx, const Tin* in,
                          Tout* out) {
    if (n > 0) k_gather_blocks<Tin, Tout><<<nblk(n * bs, 256), 256, 0, s>>>(n, bs, idx, in, out);
}
template void launch_gather_blocks<double, double>(hipStream_t, int64_t, int, const int*,
                                                   const double*, double*);
template void launch_gather_blocks<double, float>(hipStream_t, int64_t, int, const int*,
                                                  const double*, float*);
void launch_extract_leading(hipStream_t s, int64_t nnzb, int npf, int npc, const double* A,
                            double* Ac, bool row_major) {
    k_extract_leading<<<nblk(nnzb * npc * npc, 256), 256, 0, s>>>(nnzb, npf, npc, A, Ac,
                                                                   row_major ? 1 : 0);
}
void launch_galerkin_dense(hipStream_t s, int n_cblk, int npf, int npc, const int* cptr,
                           const int* cfb, const int* crow, const int* ccol, const double* A,
                           const double* R, double* Ac, const int* list) {
    if (n_cblk > 0)
        k_galerkin_dense<<<n_cblk, 64, 0, s>>>(n_cblk, npf, npc, cptr, cfb, crow, ccol, A, R, Ac,
                                               list);
}
void launch_galerkin_wide(hipStream_t s, int n_grp, int n_cblk, int npf, int npc,
                          const int* gstart, const int* grow, const int* cbg, const int* cfb,
                          const int* ccol, const double* A, const double* R, double* U,
                          double* Ac) {
    if (n_grp <= 0 || n_cblk <= 0) return;
    const size_t nf2 = (size_t)npf * npf, nfc = (size_t)npf * npc;
    // waves per workgroup: as many as 48 KB of LDS allows (at most 4)
    const size_t budget = 48 * 1024 / sizeof(double);
    const int w1 = (int)std::max<size_t>(1, std::min<size_t>(4, budget / (nf2 + nfc)));
    const int w2 = (int)std::max<size_t>(1, std::min<size_t>(4, budget / (2 * nfc)));
    k_galerkin_u<<<(n_grp + w1 - 1) / w1, 64 * w1, (size_t)w1 * (nf2 + nfc) * sizeof(double),
                   s>>>(n_grp, npf, npc, gstart, cfb, ccol, A, R, U);
    k_galerkin_c<<<(n_cblk + w2 - 1) / w2, 64 * w2, (size_t)w2 * 2 * nfc * sizeof(double),
                   s>>>(n_cblk, npf, npc, cbg, grow, R, U, Ac);
}
void launch_transpose_list(hipStream_t s, int n, const int* list, int np, const double* in,
                           double* out) {
    if (n > 0)
        k_transpose_list<<<n, 256, (size_t)np * np * sizeof(double), s>>>(n, list, np, in, out);
}
void launch_extract_list(hipStream_t s, int n, const int* list, int npf, int npc,
                         const double* A, double* Ac) {
    if (n > 0) k_extract_list<<<n, 256, 0, s>>>(n, list, npf, npc, A, Ac);
}
void launch_gather_cells(hipStream_t s, int n_cells, int np, const int* cell_ptr, const int* rp,
                         const int* ci, const double* A, const int64_t* doff, double* D,
                         const int* list) {
    if (n_cells > 0)
        k_gather_cells<<<n_cells, 256, 0, s>>>(n_cells, np, cell_ptr, rp, ci, A, doff, D, list);
}
void launch_gj_batched(hipStream_t s, int n_mats, const int64_t* doff, const int* cell_ptr,
                       int np, int max_n, double* D, int* err, const int* list) {
    const size_t lds = (size_t)max_n * max_n * sizeof(double);
    if (n_mats > 0) k_gj_batched<<<n_mats, 256, lds, s>>>(n_mats, doff, cell_ptr, np, D, err, list);
}
void launch_bsr_to_dense(hipStream_t s, int n_rows, int np, const int* rp, const int* ci,
                         const double* A, int ld, int npad, double* dense) {
    k_bsr_to_dense<<<n_rows + 1, 256, 0, s>>>(n_rows, np, rp, ci, A, ld, npad, dense);
}
void launch_coarse_gj_step(hipStream_t s, int nt, int K, int ld, double* A, double* P2, int* err) {
    // P2 holds two pivot inverses: panel K uses P2[K % 2]; the update of
    // panel K writes the inverse for panel K + 1 into the other half, and the
    // row step of panel K + 1 runs together with the column step of panel K
    double* P = P2 + (K & 1) * NB * NB;
    double* Pn = P2 + ((K + 1) & 1) * NB * NB;
    if (K == 0) {
        k_cgj_pivot<<<1, 256, 0, s>>>(K, ld, A, P, err);
        if (nt > 1) k_cgj_row<<<nt - 1, 256, 0, s>>>(nt, K, ld, A, P);
    }
    if (nt > 1) {
        const int G = nt / 2;              // ceil((nt - 1) / 2) groups of 2 x 2 tiles per dimension
        k_cgj_update<<<G * G, 256, 0, s>>>(nt, K, ld, A, Pn, err);
    }
    if (K + 1 < nt)
        k_cgj_colrow<<<2 * nt - 1, 64, 0, s>>>(nt, K, ld, A, P, Pn);
    else
        k_cgj_col<<<nt, 256, 0, s>>>(nt, K, ld, A, P);
}
template <typename Tin, typename Tout>
void launch_convert(hipStream_t s, int64_t n, const Tin* in, Tout* out) {
    k_convert<Tin, Tout><<<nblk(n, 256), 256, 0, s>>>(n, in, out);
}

template void launch_transpose_blocks<double>(hipStream_t, int64_t, int, const double*, double*);
template void launch_transpose_blocks<float>(hipStream_t, int64_t, int, const double*, float*);
template void launch_convert<double, float>(hipStream_t, int64_t, const double*, float*);
template void launch_convert<float, double>(hipStream_t, int64_t, const float*, double*);

}  // namespace xdg
