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

// ---------------------------------------------------------------------------
// Row streaming.  The blocks of one block row are contiguous on the device
// (column-major each), so the row is one stream of nb*np*np entries in which
// entry e belongs to block column xi = e / np and matrix row e % np.  Lane l
// owns VEC consecutive matrix rows (q = l % L, L = np/VEC lanes per column) of
// column group cl = l / L; one load step of the wave covers C = 64/L whole
// columns (C*np contiguous entries, 16-byte loads where the block size
// allows).  The column index of block k sits in lane k's register and is
// fetched with a cross-lane permute, so the only global loads in the loop are
// the matrix stream and the x gather.

// WIDE: four rows per lane wherever the block size allows (for FP64 two
// 16-byte loads per lane), so that every x value fetched serves four matrix
// entries -- half the gather instructions per streamed byte of two rows.
// Blocks of 16 modes and more use it (measured: SpMV and the Jacobi sweep at
// Np = 20 gain 4-7%); the small coarse blocks keep two rows per lane, where
// the longer cross-lane reduction of the wide form costs more than it saves.
template <typename T, int NP, bool WIDE = false>
struct RowCfg {
    static constexpr int VEC = (WIDE || sizeof(T) == 4)
                                   ? (NP % 4 == 0 ? 4 : (NP % 2 == 0 ? 2 : 1))
                                   : (NP % 2 == 0 ? 2 : 1);
    static constexpr int L = NP / VEC;     // lanes per column
    static constexpr int C = 64 / L;       // columns per load instruction
    static constexpr int CH = C * NP;      // entries per load instruction
};

template <typename T, int V> struct VecT;
template <> struct VecT<double, 1> { using t = double; };
template <> struct VecT<double, 2> { using t = double2; };
template <> struct VecT<float, 1> { using t = float; };
template <> struct VecT<float, 2> { using t = float2; };
template <> struct VecT<float, 4> { using t = float4; };

template <typename T, int V>
__device__ __forceinline__ void load_vec(const T* p, T (&a)[V]) {
    if constexpr (sizeof(T) == 8 && V == 4) {
        const double2 u = *reinterpret_cast<const double2*>(p);
        const double2 w = *reinterpret_cast<const double2*>(p + 2);
        a[0] = u.x;
        a[1] = u.y;
        a[2] = w.x;
        a[3] = w.y;
        return;
    } else {
    const typename VecT<T, V>::t v = *reinterpret_cast<const typename VecT<T, V>::t*>(p);
    if constexpr (V == 1) {
        a[0] = v;
    } else if constexpr (V == 2) {
        a[0] = v.x;
        a[1] = v.y;
    } else {
        a[0] = v.x;
        a[1] = v.y;
        a[2] = v.z;
        a[3] = v.w;
    }
    }
}

// acc[v] += sum over the row's stream; partial sums per lane (reduce with
// reduce_groups).  b0: first block of the row, nb: number of blocks.
template <typename T, int NP, bool WIDE = false>
__device__ __forceinline__ void row_stream(int b0, int nb, const int* __restrict__ ci,
                                           const T* __restrict__ A, const T* __restrict__ x,
                                           int lane, T (&acc)[RowCfg<T, NP, WIDE>::VEC]) {
    using R = RowCfg<T, NP, WIDE>;
    constexpr int V = R::VEC;
    const int q = lane % R::L;
    const int cl = lane / R::L;
    const bool act = cl < R::C;
    const int colreg = lane < nb ? ci[b0 + lane] : 0;
    const T* Ar = A + (int64_t)b0 * (NP * NP);
    const int E = nb * (NP * NP);
    const int off = cl * NP + q * V;
    for (int base = 0; base < E; base += R::CH) {
        const int e = base + off;
        const bool ok = act && e < E;
        const int xi = e / NP;             // block column within the row
        const int bb = xi / NP;            // block within the row
        int col = __shfl(colreg, bb & 63, 64);
        if (ok) {
            if (bb >= 64) col = ci[b0 + bb];
            const T xv = x[(int64_t)col * NP + (xi - bb * NP)];
            T a[V];
            load_vec<T, V>(Ar + e, a);
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] += a[v] * xv;
        }
    }
}

// Sum the C column groups (lanes q, q+L, q+2L, ...) into lanes 0..L-1 with a
// fixed-shape binary tree over the group index (log2 C shuffle rounds).
template <typename T, int V>
__device__ __forceinline__ void reduce_groups(T (&acc)[V], int L, int C) {
    const int lane = threadIdx.x & 63;
    const int cl = lane / L;
    for (int s = 1; s < C; s <<= 1) {
        const int src = min(lane + s * L, 63);
        const bool take = (cl % (2 * s) == 0) && (cl + s < C);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const T o = __shfl(acc[v], src, 64);
            if (take) acc[v] += o;
        }
    }
}

// Generic block size (runtime np): one column per lane group, 8-byte loads.
template <typename T>
__device__ __forceinline__ T row_times_x_rt(int beg, int end, const int* __restrict__ ci,
                                            const T* __restrict__ A, const T* __restrict__ x,
                                            int lane, int np) {
    const int G = 64 / np;
    const int r = lane % np;
    const int g = lane / np;
    T acc = 0;
    if (g < G) {
        for (int blk = beg; blk < end; ++blk) {
            const int col = uniform(ci[blk]);
            const T* Ab = A + (int64_t)blk * (np * np) + r;
            const T* xb = x + (int64_t)col * np;
            for (int c = g; c < np; c += G) acc += Ab[c * np] * xb[c];
        }
    }
    return acc;
}

// One block row per wave; for Np >= 16 two waves per block row instead (the
// first half of the row's blocks and the rest), their sums combined through
// LDS in a fixed order -- twice the waves, which shortens the tail of the
// grid (measured 131.4 -> 127.9 us at 32^3 p=3).
// MODE SPMV_AX_DOT (Np >= 16): y = A x and, per workgroup, the partial inner
// product x . y of its two rows (fixed order: lanes, then row 0 + row 1) in
// dpart[blockIdx.x].  MODE SPMV_RESID_TRUNC with yfull != nullptr (Np >= 16)
// also keeps the whole residual b - A x in yfull.
template <typename T, int NP, int MODE>
__global__ __launch_bounds__(256) void k_bsr_spmv(int n_rows, int np_rt, const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const T* __restrict__ A,
                                                  const T* __restrict__ x,
                                                  const T* __restrict__ b, T* __restrict__ y,
                                                  int npc, double* __restrict__ dpart, int rev,
                                                  T* __restrict__ yfull) {
    const int lane = threadIdx.x & 63;
    if constexpr (NP >= 16) {
        using R = RowCfg<T, NP, true>;
        __shared__ T part[2][NP];
        __shared__ double rowdot[2];
        const int w = threadIdx.x >> 6;
        const int row0 = uniform(blockIdx.x * 2 + (w >> 1));
        const int half = w & 1;
        const bool valid = row0 < n_rows;
        const int row = rev ? n_rows - 1 - row0 : row0;
        int beg = 0, nb = 0;
        if (valid) {
            const int b0 = uniform(rp[row]), n = uniform(rp[row + 1]) - b0;
            const int h0 = n / 2;
            beg = half ? b0 + h0 : b0;
            nb = half ? n - h0 : h0;
        }
        T acc[R::VEC];
#pragma unroll
        for (int v = 0; v < R::VEC; ++v) acc[v] = 0;
        row_stream<T, NP, true>(beg, nb, ci, A, x, lane, acc);
        reduce_groups<T, R::VEC>(acc, R::L, R::C);
        if (half && lane < R::L) {
#pragma unroll
            for (int v = 0; v < R::VEC; ++v) part[w >> 1][lane * R::VEC + v] = acc[v];
        }
        __syncthreads();
        double dot = 0.0;
        if (!half && valid && lane < R::L) {
#pragma unroll
            for (int v = 0; v < R::VEC; ++v) {
                const int r = lane * R::VEC + v;
                const T sum = acc[v] + part[w >> 1][r];
                const int64_t o = (int64_t)row * NP + r;
                if (MODE == SPMV_AX || MODE == SPMV_AX_DOT) y[o] = sum;
                else if (MODE == SPMV_RESID) y[o] = b[o] - sum;
                else {
                    const T res = b[o] - sum;
                    if (r < npc) y[(int64_t)row * npc + r] = res;
                    if (yfull) yfull[o] = res;
                }
                if (MODE == SPMV_AX_DOT) dot += (double)x[o] * (double)sum;
            }
        }
        if constexpr (MODE == SPMV_AX_DOT) {
            for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 64);
            if (!half && lane == 0) rowdot[w >> 1] = dot;
            __syncthreads();
            if (threadIdx.x == 0) dpart[blockIdx.x] = rowdot[0] + rowdot[1];
        }
    } else {
        const int row0 = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
        if (row0 >= n_rows) return;
        const int row = rev ? n_rows - 1 - row0 : row0;
        const int beg = uniform(rp[row]), end = uniform(rp[row + 1]);
        if constexpr (NP > 0) {
            using R = RowCfg<T, NP>;
            T acc[R::VEC];
#pragma unroll
            for (int v = 0; v < R::VEC; ++v) acc[v] = 0;
            row_stream<T, NP>(beg, end - beg, ci, A, x, lane, acc);
            reduce_groups<T, R::VEC>(acc, R::L, R::C);
            if (lane < R::L) {
#pragma unroll
                for (int v = 0; v < R::VEC; ++v) {
                    const int r = lane * R::VEC + v;
                    const int64_t o = (int64_t)row * NP + r;
                    if (MODE == SPMV_AX) y[o] = acc[v];
                    else if (MODE == SPMV_RESID) y[o] = b[o] - acc[v];
                    else if (r < npc) y[(int64_t)row * npc + r] = b[o] - acc[v];
                }
            }
        } else {
            const int np = np_rt;
            T acc = row_times_x_rt<T>(beg, end, ci, A, x, lane, np);
            acc = group_sum(acc, np, 64 / np);
            if (lane < np) {
                const int64_t o = (int64_t)row * np + lane;
                if (MODE == SPMV_AX) y[o] = acc;
                else if (MODE == SPMV_RESID) y[o] = b[o] - acc;
                else if (lane < npc) y[(int64_t)row * npc + lane] = b[o] - acc;
            }
        }
    }
}

// out = D r for the dense column-major n x n block D (n a multiple of V),
// r in LDS; same column-chunk streaming as row_stream.  Lanes 0..n/V-1 end up
// holding rows lane*V .. lane*V+V-1.
template <typename T, int V>
__device__ __forceinline__ void dense_apply(const T* __restrict__ D, int n, const T* r, int lane,
                                            T (&acc)[V]) {
    const int L = n / V;
    const int C = 64 / L;
    const int q = lane % L, cl = lane / L;
    const int E = n * n, CH = C * n;
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = 0;
    if (cl < C) {
        for (int base = 0; base < E; base += CH) {
            const int e = base + cl * n + q * V;
            if (e < E) {
                const T rv = r[e / n];
                T a[V];
                load_vec<T, V>(D + e, a);
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] += a[v] * rv;
            }
        }
    }
    reduce_groups<T, V>(acc, L, C);
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
                                                T* __restrict__ xout, T omega, int rev) {
    __shared__ T res[4][kMaxCell];
    const int np = NP ? NP : np_rt;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int cell0 = uniform(blockIdx.x * 4 + w);
    if (cell0 >= n_cells) return;
    const int cell = rev ? n_cells - 1 - cell0 : cell0;
    const int r0 = uniform(cell_ptr[cell]), r1 = uniform(cell_ptr[cell + 1]);
    const int nc = (r1 - r0) * np;
    for (int row = r0; row < r1; ++row) {
        const int64_t ob = (int64_t)row * np;
        T* rs = &res[w][(row - r0) * np];
        if constexpr (NP > 0) {
            using R = RowCfg<T, NP, (NP >= 16)>;
            T acc[R::VEC];
#pragma unroll
            for (int v = 0; v < R::VEC; ++v) acc[v] = 0;
            if (!FIRST) {
                const int beg = uniform(rp[row]), end = uniform(rp[row + 1]);
                row_stream<T, NP, (NP >= 16)>(beg, end - beg, ci, A, xin, lane, acc);
                reduce_groups<T, R::VEC>(acc, R::L, R::C);
            }
            if (lane < R::L) {
#pragma unroll
                for (int v = 0; v < R::VEC; ++v)
                    rs[lane * R::VEC + v] = b[ob + lane * R::VEC + v] - acc[v];
            }
        } else {
            T acc = 0;
            if (!FIRST) {
                acc = row_times_x_rt<T>(uniform(rp[row]), uniform(rp[row + 1]), ci, A, xin, lane, np);
                acc = group_sum(acc, np, 64 / np);
            }
            if (lane < np) rs[lane] = b[ob + lane] - acc;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const T* Dc = D + doff[cell];
    const int64_t base = (int64_t)r0 * np;
    constexpr int V = NP > 0 ? RowCfg<T, (NP > 0 ? NP : 1), (NP >= 16)>::VEC : 1;
    if (nc <= 64 * V) {
        T acc[V];
        dense_apply<T, V>(Dc, nc, res[w], lane, acc);
        if (lane < nc / V) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int64_t o = base + lane * V + v;
                xout[o] = (FIRST ? T(0) : xin[o]) + omega * acc[v];
            }
        }
    } else {
        for (int o = lane; o < nc; o += 64) {
            T acc = 0;
            for (int c = 0; c < nc; ++c) acc += Dc[(int64_t)c * nc + o] * res[w][c];
            xout[base + o] = (FIRST ? T(0) : xin[base + o]) + omega * acc;
        }
    }
}

// CG update of x and r (alpha = scal[i_rz] / scal[i_pq]) fused with the first
// sweep from zero of the next V-cycle on the new residual: per cell, x += alpha
// p, r -= alpha q, x1 = omega D^-1 r (the same product as k_jacobi<FIRST>), and
// the workgroup's partial of r . r (lanes, then the four cells in order) in
// dpart[blockIdx.x].
template <int NP>
__global__ __launch_bounds__(256) void k_cg_update_first(int n_cells,
                                                         const int* __restrict__ cell_ptr,
                                                         const int64_t* __restrict__ doff,
                                                         const double* __restrict__ D,
                                                         const double* __restrict__ scal,
                                                         int i_rz, int i_pq,
                                                         const double* __restrict__ p,
                                                         const double* __restrict__ q,
                                                         double* __restrict__ x,
                                                         double* __restrict__ r,
                                                         double* __restrict__ x1, double omega,
                                                         double* __restrict__ dpart) {
    using R = RowCfg<double, NP, (NP >= 16)>;
    constexpr int V = R::VEC;
    __shared__ double res[4][kMaxCell];
    __shared__ double wsum[4];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int cell = uniform(blockIdx.x * 4 + w);
    const double alpha = scal[i_rz] / scal[i_pq];
    double dsum = 0.0;
    if (cell < n_cells) {
        const int r0 = uniform(cell_ptr[cell]), r1 = uniform(cell_ptr[cell + 1]);
        const int nc = (r1 - r0) * NP;
        const int64_t base = (int64_t)r0 * NP;
        for (int o = lane; o < nc; o += 64) {
            x[base + o] += alpha * p[base + o];
            const double ro = r[base + o] - alpha * q[base + o];
            r[base + o] = ro;
            res[w][o] = ro;
            dsum += ro * ro;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const double* Dc = D + doff[cell];
        if (nc <= 64 * V) {
            double acc[V];
            dense_apply<double, V>(Dc, nc, res[w], lane, acc);
            if (lane < nc / V) {
#pragma unroll
                for (int v = 0; v < V; ++v) x1[base + lane * V + v] = omega * acc[v];
            }
        } else {
            for (int o = lane; o < nc; o += 64) {
                double acc = 0;
                for (int c = 0; c < nc; ++c) acc += Dc[(int64_t)c * nc + o] * res[w][c];
                x1[base + o] = omega * acc;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) dsum += __shfl_xor(dsum, off, 64);
    if (lane == 0) wsum[w] = dsum;
    __syncthreads();
    if (threadIdx.x == 0) dpart[blockIdx.x] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
}

// ---------------------------------------------------------------------------
// Symmetric level matrix kept as its diagonal and upper blocks (column >= row,
// the SIP matrix being symmetric).  Row i's product is its upper stream
// (contiguous, as above) plus, for every lower block (i, j), the transpose of
// the stored block (j, i):  (M_ji^T x_j)_r = sum_c M_ji(c, r) x_j(c),  i.e. the
// stored column r dotted with x_j.  The stored block was streamed when row j
// was, a few thousand rows earlier, so the second read mostly hits the
// memory-side cache; HBM sees each off-diagonal block once.
//
// Lower-block lane map: lane = cl * L + q holds rows q*V .. q*V+V-1 of stored
// columns cl, cl + CT, ... (CT columns per load step, KT = Np / CT steps per
// block), i.e. one partial sum per output mode r = m*CT + cl; the L lanes of a
// column are then added in lane order.
template <typename T, int NP>
struct SymCfg {
    using R = RowCfg<T, NP, true>;
    static constexpr int L = R::L;
    static constexpr int ct_of(int c) { return (NP % c == 0 && c * L <= 64) ? c : ct_of(c - 1); }
    static constexpr int CT = ct_of(NP);
    static constexpr int KT = NP / CT;
};

template <typename T, int NP>
__device__ __forceinline__ void lower_stream(int l0, int nl, const int* __restrict__ lci,
                                             const int* __restrict__ lidx,
                                             const T* __restrict__ As, const T* __restrict__ x,
                                             int lane, T (&acc)[SymCfg<T, NP>::KT]) {
    using S = SymCfg<T, NP>;
    constexpr int V = S::R::VEC;
    const int q = lane % S::L;
    const int cl = lane / S::L;
    const bool act = cl < S::CT;
    const int creg = lane < nl ? lci[l0 + lane] : 0;
    const int treg = lane < nl ? lidx[l0 + lane] : 0;
    for (int k = 0; k < nl; ++k) {
        int j = __shfl(creg, k & 63, 64);
        int t = __shfl(treg, k & 63, 64);
        if (k >= 64) {
            j = lci[l0 + k];
            t = lidx[l0 + k];
        }
        if (act) {
            T xv[V];
            load_vec<T, V>(x + (int64_t)j * NP + q * V, xv);
            const T* Sb = As + (int64_t)t * (NP * NP) + q * V;
#pragma unroll
            for (int m = 0; m < S::KT; ++m) {
                T a[V];
                load_vec<T, V>(Sb + (m * S::CT + cl) * NP, a);
#pragma unroll
                for (int v = 0; v < V; ++v) acc[m] += a[v] * xv[v];
            }
        }
    }
    // lanes with q == 0 receive the sum over the column's L lanes (lane order)
#pragma unroll
    for (int m = 0; m < S::KT; ++m) {
        T tot = acc[m];
        for (int d = 1; d < S::L; ++d) tot += __shfl(acc[m], min(lane + d, 63), 64);
        acc[m] = tot;
    }
}

// SpMV modes of k_bsr_spmv on the symmetric storage: two waves per block row,
// the first streams the upper blocks, the second the lower (transposed) ones;
// the sums meet in LDS (upper + lower, fixed order).
template <typename T, int NP, int MODE>
__global__ __launch_bounds__(256) void k_bsr_spmv_sym(int n_rows, const int* __restrict__ urp,
                                                      const int* __restrict__ uci,
                                                      const T* __restrict__ As,
                                                      const int* __restrict__ lrp,
                                                      const int* __restrict__ lci,
                                                      const int* __restrict__ lidx,
                                                      const T* __restrict__ x,
                                                      const T* __restrict__ b, T* __restrict__ y,
                                                      int npc, double* __restrict__ dpart,
                                                      int rev, T* __restrict__ yfull) {
    using R = RowCfg<T, NP, true>;
    using S = SymCfg<T, NP>;
    __shared__ T part[2][NP];
    __shared__ double rowdot[2];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int row0 = uniform(blockIdx.x * 2 + (w >> 1));
    const int half = w & 1;
    const bool valid = row0 < n_rows;
    const int row = rev ? n_rows - 1 - row0 : row0;
    T acc[R::VEC];
#pragma unroll
    for (int v = 0; v < R::VEC; ++v) acc[v] = 0;
    if (!half) {
        if (valid) {
            const int b0 = uniform(urp[row]);
            row_stream<T, NP, true>(b0, uniform(urp[row + 1]) - b0, uci, As, x, lane, acc);
        }
        reduce_groups<T, R::VEC>(acc, R::L, R::C);
    } else {
        T lacc[S::KT];
#pragma unroll
        for (int m = 0; m < S::KT; ++m) lacc[m] = 0;
        int l0 = 0, nl = 0;
        if (valid) {
            l0 = uniform(lrp[row]);
            nl = uniform(lrp[row + 1]) - l0;
        }
        lower_stream<T, NP>(l0, nl, lci, lidx, As, x, lane, lacc);
        const int q = lane % S::L, cl = lane / S::L;
        if (q == 0 && cl < S::CT) {
#pragma unroll
            for (int m = 0; m < S::KT; ++m) part[w >> 1][m * S::CT + cl] = lacc[m];
        }
    }
    __syncthreads();
    double dot = 0.0;
    if (!half && valid && lane < R::L) {
#pragma unroll
        for (int v = 0; v < R::VEC; ++v) {
            const int r = lane * R::VEC + v;
            const T sum = acc[v] + part[w >> 1][r];
            const int64_t o = (int64_t)row * NP + r;
            if (MODE == SPMV_AX || MODE == SPMV_AX_DOT) y[o] = sum;
            else if (MODE == SPMV_RESID) y[o] = b[o] - sum;
            else {
                const T res = b[o] - sum;
                if (r < npc) y[(int64_t)row * npc + r] = res;
                if (yfull) yfull[o] = res;
            }
            if (MODE == SPMV_AX_DOT) dot += (double)x[o] * (double)sum;
        }
    }
    if constexpr (MODE == SPMV_AX_DOT) {
        for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 64);
        if (!half && lane == 0) rowdot[w >> 1] = dot;
        __syncthreads();
        if (threadIdx.x == 0) dpart[blockIdx.x] = rowdot[0] + rowdot[1];
    }
}

// Damped block-Jacobi sweep (x_in given) on the symmetric storage: two waves
// per cell, the first streams the upper blocks of the cell's rows, the second
// the lower (transposed) ones; the row sums meet in LDS, the residual
// b - (upper + lower) is formed in a fixed order, and the first wave applies
// the cell-block inverse.
template <typename T, int NP>
__global__ __launch_bounds__(256) void k_jacobi_sym(int n_cells, const int* __restrict__ cell_ptr,
                                                    const int* __restrict__ urp,
                                                    const int* __restrict__ uci,
                                                    const T* __restrict__ As,
                                                    const int* __restrict__ lrp,
                                                    const int* __restrict__ lci,
                                                    const int* __restrict__ lidx,
                                                    const int64_t* __restrict__ doff,
                                                    const T* __restrict__ D,
                                                    const T* __restrict__ b,
                                                    const T* __restrict__ xin,
                                                    T* __restrict__ xout, T omega, int rev) {
    using R = RowCfg<T, NP, true>;
    using S = SymCfg<T, NP>;
    constexpr int V = R::VEC;
    __shared__ T up[2][kMaxCell];
    __shared__ T lo[2][kMaxCell];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int c2 = w >> 1;
    const int half = w & 1;
    const int cell0 = uniform(blockIdx.x * 2 + c2);
    const bool valid = cell0 < n_cells;
    const int cell = rev ? n_cells - 1 - cell0 : cell0;
    int r0 = 0, r1 = 0;
    if (valid) {
        r0 = uniform(cell_ptr[cell]);
        r1 = uniform(cell_ptr[cell + 1]);
    }
    const int nc = (r1 - r0) * NP;
    if (!half) {
        for (int row = r0; row < r1; ++row) {
            T acc[V];
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] = 0;
            const int b0 = uniform(urp[row]);
            row_stream<T, NP, true>(b0, uniform(urp[row + 1]) - b0, uci, As, xin, lane, acc);
            reduce_groups<T, V>(acc, R::L, R::C);
            if (lane < R::L) {
#pragma unroll
                for (int v = 0; v < V; ++v) up[c2][(row - r0) * NP + lane * V + v] = acc[v];
            }
        }
    } else {
        const int q = lane % S::L, cl = lane / S::L;
        for (int row = r0; row < r1; ++row) {
            T lacc[S::KT];
#pragma unroll
            for (int m = 0; m < S::KT; ++m) lacc[m] = 0;
            const int l0 = uniform(lrp[row]);
            lower_stream<T, NP>(l0, uniform(lrp[row + 1]) - l0, lci, lidx, As, xin, lane, lacc);
            if (q == 0 && cl < S::CT) {
#pragma unroll
                for (int m = 0; m < S::KT; ++m) lo[c2][(row - r0) * NP + m * S::CT + cl] = lacc[m];
            }
        }
    }
    __syncthreads();
    if (half || !valid) return;
    const int64_t base = (int64_t)r0 * NP;
    for (int e = lane; e < nc; e += 64) up[c2][e] = b[base + e] - (up[c2][e] + lo[c2][e]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const T* Dc = D + doff[cell];
    if (nc <= 64 * V) {
        T acc[V];
        dense_apply<T, V>(Dc, nc, up[c2], lane, acc);
        if (lane < nc / V) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int64_t o = base + lane * V + v;
                xout[o] = xin[o] + omega * acc[v];
            }
        }
    } else {
        for (int o = lane; o < nc; o += 64) {
            T acc = 0;
            for (int c = 0; c < nc; ++c) acc += Dc[(int64_t)c * nc + o] * up[c2][c];
            xout[base + o] = xin[base + o] + omega * acc;
        }
    }
}

// ---------------------------------------------------------------------------
// First post-smoothing sweep after a p-coarse correction, from the residual
// the pre-smoothing pass kept.  With x2 = x1 + P e (P the p-prolongation:
// e fills the leading NC modes of every block row) and r1 = b - M x1,
//   b - M x2 = r1 - (M P) e,
// and M P consists of the leading NC columns of every block -- with blocks
// column-major, the first NP*NC entries of each, stored contiguously as AP.
// So the sweep
//   x_out = x2 + omega D^-1 (r1 - (M P) e)
// streams NP*NC instead of NP*NP entries per block and needs no separate
// prolongation.  One wave per cell as k_jacobi; the AP blocks of a row are
// one contiguous stream of NP x NC column-major blocks.
template <typename T, int NP, int NC>
__device__ __forceinline__ void row_stream_nc(int b0, int nb, const int* __restrict__ ci,
                                              const T* __restrict__ AP, const T* __restrict__ e,
                                              int lane, T (&acc)[RowCfg<T, NP, true>::VEC]) {
    using R = RowCfg<T, NP, true>;
    constexpr int V = R::VEC;
    const int q = lane % R::L;
    const int cl = lane / R::L;
    const bool act = cl < R::C;
    const int colreg = lane < nb ? ci[b0 + lane] : 0;
    const T* Ar = AP + (int64_t)b0 * (NP * NC);
    const int E = nb * (NP * NC);
    const int off = cl * NP + q * V;
    for (int base = 0; base < E; base += R::CH) {
        const int ee = base + off;
        const bool ok = act && ee < E;
        const int xi = ee / NP;            // column within the row's stream
        const int bb = xi / NC;            // block within the row
        int col = __shfl(colreg, bb & 63, 64);
        if (ok) {
            if (bb >= 64) col = ci[b0 + bb];
            const T ev = e[(int64_t)col * NC + (xi - bb * NC)];
            T a[V];
            load_vec<T, V>(Ar + ee, a);
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] += a[v] * ev;
        }
    }
}

template <typename T, int NP, int NC>
__global__ __launch_bounds__(256) void k_jacobi_cc(int n_cells, const int* __restrict__ cell_ptr,
                                                   const int* __restrict__ rp,
                                                   const int* __restrict__ ci,
                                                   const T* __restrict__ AP,
                                                   const int64_t* __restrict__ doff,
                                                   const T* __restrict__ D,
                                                   const T* __restrict__ r1,
                                                   const T* __restrict__ x1,
                                                   const T* __restrict__ e,
                                                   T* __restrict__ xout, T omega, int rev) {
    using R = RowCfg<T, NP, true>;
    constexpr int V = R::VEC;
    __shared__ T res[4][kMaxCell];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int cell0 = uniform(blockIdx.x * 4 + w);
    if (cell0 >= n_cells) return;
    const int cell = rev ? n_cells - 1 - cell0 : cell0;
    const int r0 = uniform(cell_ptr[cell]), r1_ = uniform(cell_ptr[cell + 1]);
    const int nc = (r1_ - r0) * NP;
    for (int row = r0; row < r1_; ++row) {
        const int64_t ob = (int64_t)row * NP;
        T acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = 0;
        const int b0 = uniform(rp[row]);
        row_stream_nc<T, NP, NC>(b0, uniform(rp[row + 1]) - b0, ci, AP, e, lane, acc);
        reduce_groups<T, V>(acc, R::L, R::C);
        if (lane < R::L) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int r = lane * V + v;
                res[w][(row - r0) * NP + r] = r1[ob + r] - acc[v];
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const T* Dc = D + doff[cell];
    const int64_t base = (int64_t)r0 * NP;
    // x2 = x1 + P e at entry o of the cell (block row o / NP, mode o % NP)
    auto x2 = [&](int o) -> T {
        const int rr = o / NP, m = o - rr * NP;
        return x1[base + o] + (m < NC ? e[(int64_t)(r0 + rr) * NC + m] : T(0));
    };
    if (nc <= 64 * V) {
        T acc[V];
        dense_apply<T, V>(Dc, nc, res[w], lane, acc);
        if (lane < nc / V) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int o = lane * V + v;
                xout[base + o] = x2(o) + omega * acc[v];
            }
        }
    } else {
        for (int o = lane; o < nc; o += 64) {
            T acc = 0;
            for (int c = 0; c < nc; ++c) acc += Dc[(int64_t)c * nc + o] * res[w][c];
            xout[base + o] = x2(o) + omega * acc;
        }
    }
}

// ---------------------------------------------------------------------------
// Small blocks (Np <= 8, the p1 and aggregation levels): a block row holds
// only ~7 Np^2 entries, so with one wave per row the kernels are bound by
// per-wave overhead.  Here a group of kGS = 16 lanes takes one block row
// (SpMV) or one smoother cell (Jacobi), four groups per wave, with the same
// column-chunk streaming and fixed reduction tree inside the group.  Row and
// cell indices differ between the groups of a wave; every cross-lane read
// stays inside the reading lane's own group.
constexpr int kGS = 16;

template <typename T, int NP>
struct GrpCfg {
    static constexpr int VEC = RowCfg<T, NP>::VEC;
    static constexpr int L = NP / VEC;     // lanes per column
    static constexpr int C = kGS / L;      // columns per load step of a group
    static constexpr int CH = C * NP;
};

// Load steps per pass of grp_stream: two (fewer than 16 blocks' worth).  The
// level-1 grid of the 32^3 workload (~2,000 workgroups) is resident at once
// only at 8 waves per SIMD, i.e. at most 64 VGPRs; four or eight steps per
// pass cost that occupancy and were slower.
template <typename T, int NP, int NCOL>
struct GrpPass {
    static constexpr int CH = GrpCfg<T, NP>::CH;
    static constexpr int U0 = (16 * NP * NCOL + CH - 1) / CH;
    static constexpr int U = U0 < 1 ? 1 : (U0 > 2 ? 2 : U0);
};

// acc += (sum over the nb blocks at b0 of A_b x_col(b)) for one lane group;
// blocks are NP x NCOL, column-major.  The blocks are streamed U load steps
// at a time and every load of a pass is issued before its products, so a
// group waits for one memory round trip per pass, not one per load step (the
// small levels are latency-bound).
// With TWO the list holds the blocks of two consecutive block rows (the two
// species of a cell, adjacent in the row storage); blocks at positions >= nb0
// belong to the second row and go to acc1.  Lanes past the end of the list
// load entry 0 and add nothing.  Each lane adds its entries in list order, so
// a one-row list sums exactly as one row at a time.
template <typename T, int NP, int NCOL, bool TWO>
__device__ __forceinline__ void grp_stream(int b0, int nb, int nb0, const int* __restrict__ ci,
                                           const T* __restrict__ A, const T* __restrict__ x,
                                           int lane, T (&acc0)[GrpCfg<T, NP>::VEC],
                                           T (&acc1)[GrpCfg<T, NP>::VEC]) {
    using R = GrpCfg<T, NP>;
    constexpr int V = R::VEC, U = GrpPass<T, NP, NCOL>::U;
    const int gl = lane & (kGS - 1), gb = lane - gl;
    const int q = gl % R::L, cl = gl / R::L;
    const bool act = cl < R::C;
    const int cr0 = gl < nb ? ci[b0 + gl] : 0;
    const int cr1 = gl + kGS < nb ? ci[b0 + kGS + gl] : 0;
    const T* Ar = A + (int64_t)b0 * (NP * NCOL);
    const int E = nb * (NP * NCOL);
    const int off = cl * NP + q * V;
    for (int base = 0; base < E; base += U * R::CH) {
        T a[U][V], xv[U];
        int bu[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * R::CH + off;
            const bool ok = act && e < E;
            const int ec = ok ? e : 0;
            const int xi = ec / NP;                // (block, column) index
            const int bb = xi / NCOL;
            const int s0 = __shfl(cr0, gb + (bb & (kGS - 1)), 64);
            const int s1 = __shfl(cr1, gb + (bb & (kGS - 1)), 64);
            int col = bb < kGS ? s0 : s1;
            if (bb >= 2 * kGS) col = ci[b0 + bb];
            xv[u] = x[(int64_t)col * NCOL + (xi - bb * NCOL)];
            load_vec<T, V>(Ar + ec, a[u]);
            bu[u] = ok ? bb : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = bu[u] >= 0;
            const bool second = TWO && bu[u] >= nb0;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const T p = a[u][v] * xv[u];
                if (ok && !second) acc0[v] += p;
                if (TWO && ok && second) acc1[v] += p;
            }
        }
    }
}

// sum of the C column groups of a lane group into its lanes 0..L-1
template <typename T, int V>
__device__ __forceinline__ void reduce_groups_g(T (&acc)[V], int L, int C, int lane) {
    const int gl = lane & (kGS - 1), gb = lane - gl;
    const int cl = gl / L;
    for (int s = 1; s < C; s <<= 1) {
        const int src = min(lane + s * L, gb + kGS - 1);
        const bool take = (cl % (2 * s) == 0) && (cl + s < C);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const T o = __shfl(acc[v], src, 64);
            if (take) acc[v] += o;
        }
    }
}

template <typename T, int NP, int MODE>
__global__ __launch_bounds__(256) void k_bsr_spmv_g(int n_rows, const int* __restrict__ rp,
                                                    const int* __restrict__ ci,
                                                    const T* __restrict__ A,
                                                    const T* __restrict__ x,
                                                    const T* __restrict__ b, T* __restrict__ y,
                                                    int npc) {
    using R = GrpCfg<T, NP>;
    const int lane = threadIdx.x & 63;
    const int row = (int)blockIdx.x * (256 / kGS) + (int)(threadIdx.x / kGS);
    const bool valid = row < n_rows;
    int beg = 0, nb = 0;
    if (valid) {
        beg = rp[row];
        nb = rp[row + 1] - beg;
    }
    T acc[R::VEC];
#pragma unroll
    for (int v = 0; v < R::VEC; ++v) acc[v] = 0;
    grp_stream<T, NP, NP, false>(beg, nb, nb, ci, A, x, lane, acc, acc);
    reduce_groups_g<T, R::VEC>(acc, R::L, R::C, lane);
    const int gl = lane & (kGS - 1);
    if (valid && gl < R::L) {
#pragma unroll
        for (int v = 0; v < R::VEC; ++v) {
            const int r = gl * R::VEC + v;
            const int64_t o = (int64_t)row * NP + r;
            if (MODE == SPMV_AX) y[o] = acc[v];
            else if (MODE == SPMV_RESID) y[o] = b[o] - acc[v];
            else if (r < npc) y[(int64_t)row * npc + r] = b[o] - acc[v];
        }
    }
}

// Right-hand side of a cell of at most two block rows in the reduction's
// layout (lanes 0..L-1), loaded before the streams (it needs only the cell's
// first row); the cell's inverse is applied after the residual is in LDS,
// every column's load issued at once (lane o < nc owns unknown o).
template <typename T, int NP>
struct CellPre {
    static constexpr int CM = 2 * NP;
    T b0[GrpCfg<T, NP>::VEC], b1[GrpCfg<T, NP>::VEC];
    __device__ __forceinline__ void load(const T* __restrict__ b, int64_t base, int nr, int gl) {
        constexpr int V = GrpCfg<T, NP>::VEC;
        const int r = min(gl, GrpCfg<T, NP>::L - 1) * V;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            b0[v] = nr > 0 ? b[base + r + v] : T(0);
            b1[v] = nr > 1 ? b[base + NP + r + v] : T(0);
        }
    }
    // (D_c res)_o for lane o = gl < nc of the column-major nc x nc inverse Dc
    __device__ __forceinline__ static T apply(const T* __restrict__ Dc, const T* res, int nc,
                                              int gl) {
        const int o = min(gl, max(nc - 1, 0));
        T d[CM];
#pragma unroll
        for (int c = 0; c < CM; ++c) d[c] = Dc[(int64_t)min(c, max(nc - 1, 0)) * nc + o];
        T a = 0;
#pragma unroll
        for (int c = 0; c < CM; ++c)
            if (c < nc) a += d[c] * res[c];
        return a;
    }
};

template <typename T, int NP, bool FIRST>
__global__ __launch_bounds__(256) void k_jacobi_g(int n_cells, const int* __restrict__ cell_ptr,
                                                  const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const T* __restrict__ A,
                                                  const int64_t* __restrict__ doff,
                                                  const T* __restrict__ D,
                                                  const T* __restrict__ b,
                                                  const T* __restrict__ xin,
                                                  T* __restrict__ xout, T omega) {
    using R = GrpCfg<T, NP>;
    constexpr int V = R::VEC;
    constexpr int G = 256 / kGS;
    static_assert(2 * NP <= kGS, "a two-row cell must fit one lane group");
    __shared__ T res[G][kMaxCell];
    const int lane = threadIdx.x & 63;
    const int grp = threadIdx.x / kGS, gl = lane & (kGS - 1);
    const int cell = (int)blockIdx.x * G + grp;
    const bool valid = cell < n_cells;
    int r0 = 0, r1 = 0;
    if (valid) {
        r0 = cell_ptr[cell];
        r1 = cell_ptr[cell + 1];
    }
    const int nr = r1 - r0;
    const int nc = nr * NP;                        // <= kMaxCell (checked on the host)
    const int64_t base = (int64_t)r0 * NP;
    if (nr <= 2) {
        CellPre<T, NP> pre;
        pre.load(b, base, nr, gl);
        const T* Dc = D + (valid ? doff[cell] : 0);
        const T xo = !FIRST && gl < nc ? xin[base + gl] : T(0);
        T acc0[V], acc1[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc0[v] = acc1[v] = 0;
        if (!FIRST && nr > 0) {
            const int beg = rp[r0], mid = rp[r0 + 1], end = rp[r1];
            grp_stream<T, NP, NP, true>(beg, end - beg, mid - beg, ci, A, xin, lane, acc0, acc1);
            reduce_groups_g<T, V>(acc0, R::L, R::C, lane);
            reduce_groups_g<T, V>(acc1, R::L, R::C, lane);
        }
        if (gl < R::L) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                res[grp][gl * V + v] = pre.b0[v] - acc0[v];
                res[grp][NP + gl * V + v] = pre.b1[v] - acc1[v];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (gl < nc) xout[base + gl] = xo + omega * CellPre<T, NP>::apply(Dc, res[grp], nc, gl);
        return;
    }
    for (int row = r0; row < r1; ++row) {
        T acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = 0;
        if (!FIRST) {
            const int beg = rp[row], nb = rp[row + 1] - beg;
            grp_stream<T, NP, NP, false>(beg, nb, nb, ci, A, xin, lane, acc, acc);
            reduce_groups_g<T, V>(acc, R::L, R::C, lane);
        }
        if (gl < R::L) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int r = gl * V + v;
                res[grp][(row - r0) * NP + r] = b[(int64_t)row * NP + r] - acc[v];
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const T* Dc = D + doff[cell];
    for (int o = gl; o < nc; o += kGS) {
        T a = 0;
        for (int c = 0; c < nc; ++c) a += Dc[(int64_t)c * nc + o] * res[grp][c];
        xout[base + o] = (FIRST ? T(0) : xin[base + o]) + omega * a;
    }
}

// First post sweep after an aggregation coarse correction, the small-block
// form of k_jacobi_cc: with x2 = x1 + R e (fine row i takes R_i e_parent(i))
// and r1 = b - M x1 kept by the residual pass,
//   b - M x2 = r1 - (M R) e,
// where (M R)_iJ = sum over the row's blocks (i, j) with parent(j) = J of
// M_ij R_j (np x npc, column-major, formed at set-up; the distinct coarse
// neighbours of a row are fewer than its fine ones).  One 16-lane group per
// cell, as k_jacobi_g; the prolongation is fused.
template <typename T, int NP, int NC>
__global__ __launch_bounds__(256) void k_jacobi_cc_g(int n_cells, const int* __restrict__ cell_ptr,
                                                     const int* __restrict__ arp,
                                                     const int* __restrict__ arc,
                                                     const T* __restrict__ AR,
                                                     const int64_t* __restrict__ doff,
                                                     const T* __restrict__ D,
                                                     const T* __restrict__ r1,
                                                     const T* __restrict__ x1,
                                                     const T* __restrict__ e,
                                                     const int* __restrict__ parent,
                                                     const int* __restrict__ ridx,
                                                     const T* __restrict__ Rt,
                                                     T* __restrict__ xout, T omega) {
    using R = GrpCfg<T, NP>;
    constexpr int V = R::VEC;
    constexpr int G = 256 / kGS;
    static_assert(2 * NP <= kGS, "a two-row cell must fit one lane group");
    __shared__ T res[G][kMaxCell];
    const int lane = threadIdx.x & 63;
    const int grp = threadIdx.x / kGS, gl = lane & (kGS - 1);
    const int cell = (int)blockIdx.x * G + grp;
    const bool valid = cell < n_cells;
    int r0 = 0, r1c = 0;
    if (valid) {
        r0 = cell_ptr[cell];
        r1c = cell_ptr[cell + 1];
    }
    const int nr = r1c - r0;
    const int nc = nr * NP;                        // <= kMaxCell (checked on the host)
    const int64_t base = (int64_t)r0 * NP;
    if (nr <= 2) {
        CellPre<T, NP> pre;
        pre.load(r1, base, nr, gl);
        const T* Dc = D + (valid ? doff[cell] : 0);
        // x1 and the prolongation R_i e_parent(i) of unknown gl
        const int og = min(gl, max(nc - 1, 0));
        const int row = r0 + og / NP, a = og % NP;
        T xo = 0;
        if (gl < nc) {
            const T* Ri = Rt + (int64_t)ridx[row] * NP * NC + a * NC;
            const T* ep = e + (int64_t)parent[row] * NC;
            T pe = 0;
#pragma unroll
            for (int m = 0; m < NC; ++m) pe += Ri[m] * ep[m];
            xo = x1[base + gl] + pe;
        }
        T acc0[V], acc1[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc0[v] = acc1[v] = 0;
        if (nr > 0) {
            const int beg = arp[r0], mid = arp[r0 + 1], end = arp[r1c];
            grp_stream<T, NP, NC, true>(beg, end - beg, mid - beg, arc, AR, e, lane, acc0, acc1);
            reduce_groups_g<T, V>(acc0, R::L, R::C, lane);
            reduce_groups_g<T, V>(acc1, R::L, R::C, lane);
        }
        if (gl < R::L) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                res[grp][gl * V + v] = pre.b0[v] - acc0[v];
                res[grp][NP + gl * V + v] = pre.b1[v] - acc1[v];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (gl < nc) xout[base + gl] = xo + omega * CellPre<T, NP>::apply(Dc, res[grp], nc, gl);
        return;
    }
    for (int row = r0; row < r1c; ++row) {
        T acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = 0;
        const int beg = arp[row], nb = arp[row + 1] - beg;
        grp_stream<T, NP, NC, false>(beg, nb, nb, arc, AR, e, lane, acc, acc);
        reduce_groups_g<T, V>(acc, R::L, R::C, lane);
        if (gl < R::L) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int r = gl * V + v;
                res[grp][(row - r0) * NP + r] = r1[(int64_t)row * NP + r] - acc[v];
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const T* Dc = D + doff[cell];
    for (int o = gl; o < nc; o += kGS) {
        const int row = r0 + o / NP, a = o % NP;
        const T* Ri = Rt + (int64_t)ridx[row] * NP * NC + a * NC;
        const T* ep = e + (int64_t)parent[row] * NC;
        T pe = 0;
        for (int m = 0; m < NC; ++m) pe += Ri[m] * ep[m];
        T acc = 0;
        for (int c = 0; c < nc; ++c) acc += Dc[(int64_t)c * nc + o] * res[grp][c];
        xout[base + o] = (x1[base + o] + pe) + omega * acc;
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

// rc[c][m] = sum_{i in children(c)} sum_a R_i[a][m] rf[i][a]: one wave per
// coarse row; lane t takes the (child, fine mode) pairs t, t+64, ... in
// ascending order, then a fixed butterfly sums the lanes (no atomics).
template <typename T>
__global__ __launch_bounds__(256) void k_restrict_dense(int n_c, int npf, int npc,
                                                        const int* __restrict__ child_ptr,
                                                        const int* __restrict__ child_idx,
                                                        const int* __restrict__ ridx,
                                                        const T* __restrict__ R,
                                                        const T* __restrict__ rf,
                                                        T* __restrict__ rc) {
    const int lane = threadIdx.x & 63;
    const int c = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (c >= n_c) return;
    const int k0 = uniform(child_ptr[c]), nk = uniform(child_ptr[c + 1]) - k0;
    T acc[kMaxTransferModes];
#pragma unroll
    for (int m = 0; m < kMaxTransferModes; ++m) acc[m] = 0;
    for (int t = lane; t < nk * npf; t += 64) {
        const int k = t / npf, a = t - k * npf;
        const int i = child_idx[k0 + k];
        const T rv = rf[(int64_t)i * npf + a];
        const T* Ri = R + ((int64_t)ridx[i] * npf + a) * npc;
#pragma unroll
        for (int m = 0; m < kMaxTransferModes; ++m)
            if (m < npc) acc[m] += Ri[m] * rv;
    }
#pragma unroll
    for (int m = 0; m < kMaxTransferModes; ++m) {
        if (m < npc) {
            T v = acc[m];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == m) rc[(int64_t)c * npc + m] = v;
        }
    }
}

// Coarse blocks of more than kMaxTransferModes modes (aggregation levels that
// keep the fine degree, R_i up to 35 x 35): the restriction runs in two
// kernels so that no wave walks all children of a coarse row in sequence.
// (1) one wave per fine row i: t_i = R_i^T rf_i; lane = (coarse mode m,
//     group g), the G = 64 / npc groups take the fine modes a = g, g + G, ...
//     (npc consecutive lanes read one contiguous row of R_i), then a fixed
//     tree over the groups;
template <typename T>
__global__ __launch_bounds__(256) void k_restrict_rows_wide(int n_f, int npf, int npc,
                                                            const int* __restrict__ ridx,
                                                            const T* __restrict__ R,
                                                            const T* __restrict__ rf,
                                                            T* __restrict__ t) {
    const int lane = threadIdx.x & 63;
    const int i = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (i >= n_f) return;
    const int G = 64 / npc;
    const int m = lane % npc, g = lane / npc;
    const T* Ri = R + (int64_t)ridx[i] * npf * npc;
    const T* ri = rf + (int64_t)i * npf;
    T acc = 0;
    if (g < G)
        for (int a = g; a < npf; a += G) acc += Ri[a * npc + m] * ri[a];
    for (int st = 1; st < G; st <<= 1) {
        const T o = __shfl(acc, min(lane + st * npc, 63), 64);
        if (g % (2 * st) == 0 && g + st < G) acc += o;
    }
    if (lane < npc) t[(int64_t)i * npc + lane] = acc;
}

// (2) rc[c][m] = sum over the children of c, in ascending order, of t_i[m].
template <typename T>
__global__ void k_restrict_children(int n_c, int npc, const int* __restrict__ child_ptr,
                                    const int* __restrict__ child_idx, const T* __restrict__ t,
                                    T* __restrict__ rc) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n_c * npc) return;
    const int c = (int)(e / npc), m = (int)(e - (int64_t)c * npc);
    T acc = 0;
    for (int q = child_ptr[c]; q < child_ptr[c + 1]; ++q)
        acc += t[(int64_t)child_idx[q] * npc + m];
    rc[e] = acc;
}

// Prolongation for the same wide transfers, one wave per fine row i:
// xf_i += R_i xc_{parent(i)}; lane = (coarse mode m, group g) reads one
// contiguous row segment of R_i per fine mode a = g, g + G, ...; the products
// of a row are summed over the npc lanes of the group by a fixed tree.
template <typename T>
__global__ __launch_bounds__(256) void k_prolong_rows_wide(int n_f, int npf, int npc,
                                                           const int* __restrict__ parent,
                                                           const int* __restrict__ ridx,
                                                           const T* __restrict__ R,
                                                           const T* __restrict__ xc,
                                                           T* __restrict__ xf) {
    const int lane = threadIdx.x & 63;
    const int i = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (i >= n_f) return;
    const int G = 64 / npc;
    const int m = lane % npc, g = lane / npc;
    const T* Ri = R + (int64_t)ridx[i] * npf * npc;
    const T xm = g < G ? xc[(int64_t)parent[i] * npc + m] : T(0);
    const int steps = (npf + G - 1) / G;
    for (int k = 0; k < steps; ++k) {
        const int a = g + k * G;
        T v = (g < G && a < npf) ? Ri[a * npc + m] * xm : T(0);
        for (int st = 1; st < npc; st <<= 1) {
            const T o = __shfl(v, min(lane + st, 63), 64);
            if (m % (2 * st) == 0 && m + st < npc) v += o;
        }
        if (g < G && a < npf && m == 0) xf[(int64_t)i * npf + a] += v;
    }
}

// xf[i][a] += sum_m R_i[a][m] xc[parent(i)][m]
template <typename T>
__global__ void k_prolong_dense(int n_f, int npf, int npc, const int* __restrict__ parent,
                                const int* __restrict__ ridx,
                                const T* __restrict__ R, const T* __restrict__ xc,
                                T* __restrict__ xf) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_f * npf) return;
    const int i = (int)(t / npf);
    const int a = (int)(t - (int64_t)i * npf);
    const T* Ri = R + (int64_t)ridx[i] * npf * npc + a * npc;
    const T* xp = xc + (int64_t)parent[i] * npc;
    T acc = 0;
    for (int m = 0; m < npc; ++m) acc += Ri[m] * xp[m];
    xf[t] += acc;
}

// z = Ainv r, Ainv dense row-major (leading dimension ld, even); one wave per
// row, 16-byte loads, fixed-order lane partials then a butterfly.
__global__ __launch_bounds__(256) void k_coarse_gemv(int n, int ld, const double* __restrict__ Ainv,
                                                     const double* __restrict__ r,
                                                     double* __restrict__ z) {
    const int lane = threadIdx.x & 63;
    const int row = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (row >= n) return;
    const double* a = Ainv + (int64_t)row * ld;
    double acc = 0.0;
    const int n2 = n >> 1;
#pragma unroll 4
    for (int j = lane; j < n2; j += 64) {
        const double2 av = *reinterpret_cast<const double2*>(a + 2 * j);
        const double2 rv = *reinterpret_cast<const double2*>(r + 2 * j);
        acc += av.x * rv.x + av.y * rv.y;
    }
    if ((n & 1) && lane == 0) acc += a[n - 1] * r[n - 1];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) z[row] = acc;
}

// ---------------------------------------------------------------------------
// launchers

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T, int MODE>
static void spmv_np(hipStream_t s, int n_rows, int np, const int* rp, const int* ci, const T* A,
                    const T* x, const T* b, T* y, int npc, int rev, T* yfull) {
    dim3 g(nblk(n_rows, 4)), blk(256);
    dim3 gg(nblk(n_rows, 256 / kGS));
    switch (np) {
#define XDG_NPG(N) \
    case N: k_bsr_spmv_g<T, N, MODE><<<gg, blk, 0, s>>>(n_rows, rp, ci, A, x, b, y, npc); break;
        XDG_NPG(1) XDG_NPG(3) XDG_NPG(4) XDG_NPG(6)
#undef XDG_NPG
#define XDG_NP(N) \
    case N: k_bsr_spmv<T, N, MODE><<<g, blk, 0, s>>>(n_rows, np, rp, ci, A, x, b, y, npc, nullptr, rev, nullptr); break;
        XDG_NP(10)
#undef XDG_NP
#define XDG_NP2(N)                                                                          \
    case N:                                                                                 \
        k_bsr_spmv<T, N, MODE><<<nblk(n_rows, 2), blk, 0, s>>>(n_rows, np, rp, ci, A, x, b, y, \
                                                                npc, nullptr, rev, yfull);  \
        break;
        XDG_NP2(20) XDG_NP2(35)
#undef XDG_NP2
        default: k_bsr_spmv<T, 0, MODE><<<g, blk, 0, s>>>(n_rows, np, rp, ci, A, x, b, y, npc, nullptr, rev, nullptr);
    }
}

template <typename T>
void launch_spmv(hipStream_t s, int mode, int n_rows, int np, const int* rp, const int* ci,
                 const T* A, const T* x, const T* b, T* y, int npc, bool rev, T* yfull) {
    const int r = rev ? 1 : 0;
    if (mode == SPMV_AX) spmv_np<T, SPMV_AX>(s, n_rows, np, rp, ci, A, x, b, y, npc, r, nullptr);
    else if (mode == SPMV_RESID)
        spmv_np<T, SPMV_RESID>(s, n_rows, np, rp, ci, A, x, b, y, npc, r, nullptr);
    else spmv_np<T, SPMV_RESID_TRUNC>(s, n_rows, np, rp, ci, A, x, b, y, npc, r, yfull);
}

// y = A x and *out = x . y (FP64, Np = 20 or 35: the product's epilogue forms
// per-workgroup partials, a second kernel adds them in order); false when the
// block size has no fused form (the caller then runs the two steps apart)
bool launch_spmv_dot(hipStream_t s, int n_rows, int np, const int* rp, const int* ci,
                     const double* A, const double* x, double* y, double* partial,
                     double* out, bool rev) {
    const unsigned nb = nblk(n_rows, 2);
    const int r = rev ? 1 : 0;
    if (np == 20)
        k_bsr_spmv<double, 20, SPMV_AX_DOT><<<nb, 256, 0, s>>>(n_rows, np, rp, ci, A, x, nullptr,
                                                               y, 0, partial, r, nullptr);
    else if (np == 35)
        k_bsr_spmv<double, 35, SPMV_AX_DOT><<<nb, 256, 0, s>>>(n_rows, np, rp, ci, A, x, nullptr,
                                                               y, 0, partial, r, nullptr);
    else
        return false;
    launch_dot_final(s, partial, (int)nb, out);
    return true;
}

template <typename T, bool FIRST>
static void jacobi_np(hipStream_t s, int n_cells, int np, const int* cp, const int* rp,
                      const int* ci, const T* A, const int64_t* doff, const T* D, const T* b,
                      const T* xin, T* xout, T omega, int rev) {
    dim3 g(nblk(n_cells, 4)), blk(256);
    dim3 gg(nblk(n_cells, 256 / kGS));
    switch (np) {
#define XDG_NPG(N)                                                                          \
    case N:                                                                                 \
        k_jacobi_g<T, N, FIRST><<<gg, blk, 0, s>>>(n_cells, cp, rp, ci, A, doff, D, b, xin, \
                                                    xout, omega);                           \
        break;
        XDG_NPG(1) XDG_NPG(3) XDG_NPG(4) XDG_NPG(6)
#undef XDG_NPG
#define XDG_NP(N)                                                                       \
    case N:                                                                             \
        k_jacobi<T, N, FIRST><<<g, blk, 0, s>>>(n_cells, np, cp, rp, ci, A, doff, D, b, \
                                                 xin, xout, omega, rev);                \
        break;
        XDG_NP(10) XDG_NP(20) XDG_NP(35)
#undef XDG_NP
        default:
            k_jacobi<T, 0, FIRST><<<g, blk, 0, s>>>(n_cells, np, cp, rp, ci, A, doff, D, b, xin,
                                                     xout, omega, rev);
    }
}

template <typename T>
void launch_jacobi(hipStream_t s, bool first, int n_cells, int np, const int* cp, const int* rp,
                   const int* ci, const T* A, const int64_t* doff, const T* D, const T* b,
                   const T* xin, T* xout, T omega, bool rev) {
    const int r = rev ? 1 : 0;
    if (first) jacobi_np<T, true>(s, n_cells, np, cp, rp, ci, A, doff, D, b, xin, xout, omega, r);
    else jacobi_np<T, false>(s, n_cells, np, cp, rp, ci, A, doff, D, b, xin, xout, omega, r);
}

template <typename T, int MODE>
static void spmv_sym_mode(hipStream_t s, int n_rows, const SymRows<T>& m, const T* x,
                          const T* b, T* y, int npc, double* dpart, int rev, T* yfull) {
    k_bsr_spmv_sym<T, kSymNp, MODE><<<nblk(n_rows, 2), 256, 0, s>>>(
        n_rows, m.urp, m.uci, m.A, m.lrp, m.lci, m.lidx, x, b, y, npc, dpart, rev, yfull);
}

template <typename T>
void launch_spmv_sym(hipStream_t s, int mode, int n_rows, const SymRows<T>& m, const T* x,
                     const T* b, T* y, int npc, bool rev, T* yfull) {
    const int r = rev ? 1 : 0;
    if (mode == SPMV_AX)
        spmv_sym_mode<T, SPMV_AX>(s, n_rows, m, x, b, y, npc, nullptr, r, nullptr);
    else if (mode == SPMV_RESID)
        spmv_sym_mode<T, SPMV_RESID>(s, n_rows, m, x, b, y, npc, nullptr, r, nullptr);
    else spmv_sym_mode<T, SPMV_RESID_TRUNC>(s, n_rows, m, x, b, y, npc, nullptr, r, yfull);
}

void launch_spmv_dot_sym(hipStream_t s, int n_rows, const SymRows<double>& m, const double* x,
                         double* y, double* partial, double* out, bool rev) {
    const unsigned nb = nblk(n_rows, 2);
    spmv_sym_mode<double, SPMV_AX_DOT>(s, n_rows, m, x, nullptr, y, 0, partial, rev ? 1 : 0,
                                       nullptr);
    launch_dot_final(s, partial, (int)nb, out);
}

template <typename T>
void launch_jacobi_sym(hipStream_t s, int n_cells, const int* cp, const SymRows<T>& m,
                       const int64_t* doff, const T* D, const T* b, const T* xin, T* xout,
                       T omega, bool rev) {
    k_jacobi_sym<T, kSymNp><<<nblk(n_cells, 2), 256, 0, s>>>(n_cells, cp, m.urp, m.uci, m.A,
                                                             m.lrp, m.lci, m.lidx, doff, D, b,
                                                             xin, xout, omega, rev ? 1 : 0);
}

bool cc_supported(int np, int npc) { return (np == 20 || np == 35) && npc == 4; }
bool cc_dense_supported(int np, int npc) { return np == 4 && npc == 4; }

bool launch_cg_update_first(hipStream_t s, int n_cells, int np, const int* cp,
                            const int64_t* doff, const double* D, const double* scal, int i_rz,
                            int i_pq, int i_rr, const double* p, const double* q, double* x,
                            double* r, double* x1, double omega, double* partial) {
    const unsigned nb = nblk(n_cells, 4);
    if (np == 20)
        k_cg_update_first<20><<<nb, 256, 0, s>>>(n_cells, cp, doff, D, scal, i_rz, i_pq, p, q, x,
                                                 r, x1, omega, partial);
    else if (np == 35)
        k_cg_update_first<35><<<nb, 256, 0, s>>>(n_cells, cp, doff, D, scal, i_rz, i_pq, p, q, x,
                                                 r, x1, omega, partial);
    else
        return false;
    launch_dot_final(s, partial, (int)nb, const_cast<double*>(scal) + i_rr);
    return true;
}

template <typename T>
void launch_jacobi_cc_g(hipStream_t s, int n_cells, int np, int npc, const int* cp,
                        const int* arp, const int* arc, const T* AR, const int64_t* doff,
                        const T* D, const T* r1, const T* x1, const T* e, const int* parent,
                        const int* ridx, const T* R, T* xout, T omega) {
    if (np == 4 && npc == 4)
        k_jacobi_cc_g<T, 4, 4><<<nblk(n_cells, 256 / kGS), 256, 0, s>>>(
            n_cells, cp, arp, arc, AR, doff, D, r1, x1, e, parent, ridx, R, xout, omega);
}

template <typename T>
void launch_jacobi_cc(hipStream_t s, int n_cells, int np, int npc, const int* cp, const int* rp,
                      const int* ci, const T* AP, const int64_t* doff, const T* D, const T* r1,
                      const T* x1, const T* e, T* xout, T omega, bool rev) {
    const dim3 g(nblk(n_cells, 4)), blk(256);
    const int r = rev ? 1 : 0;
    if (np == 20 && npc == 4)
        k_jacobi_cc<T, 20, 4><<<g, blk, 0, s>>>(n_cells, cp, rp, ci, AP, doff, D, r1, x1, e, xout,
                                                omega, r);
    else if (np == 35 && npc == 4)
        k_jacobi_cc<T, 35, 4><<<g, blk, 0, s>>>(n_cells, cp, rp, ci, AP, doff, D, r1, x1, e, xout,
                                                omega, r);
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
void launch_restrict_dense(hipStream_t s, int n_c, int n_f, int npf, int npc, const int* cptr,
                           const int* cidx, const int* ridx, const T* R, const T* rf, T* rc,
                           T* tmp) {
    if (npc <= kMaxTransferModes) {
        k_restrict_dense<T><<<nblk(n_c, 4), 256, 0, s>>>(n_c, npf, npc, cptr, cidx, ridx, R, rf,
                                                          rc);
        return;
    }
    k_restrict_rows_wide<T><<<nblk(n_f, 4), 256, 0, s>>>(n_f, npf, npc, ridx, R, rf, tmp);
    k_restrict_children<T><<<nblk((int64_t)n_c * npc, 256), 256, 0, s>>>(n_c, npc, cptr, cidx,
                                                                          tmp, rc);
}
template <typename T>
void launch_prolong_dense(hipStream_t s, int n_f, int npf, int npc, const int* parent,
                          const int* ridx, const T* R, const T* xc, T* xf) {
    if (npc <= kMaxTransferModes)
        k_prolong_dense<T><<<nblk((int64_t)n_f * npf, 256), 256, 0, s>>>(n_f, npf, npc, parent,
                                                                         ridx, R, xc, xf);
    else
        k_prolong_rows_wide<T><<<nblk(n_f, 4), 256, 0, s>>>(n_f, npf, npc, parent, ridx, R, xc,
                                                            xf);
}
void launch_coarse_gemv(hipStream_t s, int n, int ld, const double* Ainv, const double* r,
                        double* z) {
    k_coarse_gemv<<<nblk(n, 4), 256, 0, s>>>(n, ld, Ainv, r, z);
}

#define XDG_INST(T)                                                                           \
    template void launch_spmv<T>(hipStream_t, int, int, int, const int*, const int*, const T*, \
                                 const T*, const T*, T*, int, bool, T*);                       \
    template void launch_jacobi<T>(hipStream_t, bool, int, int, const int*, const int*,        \
                                   const int*, const T*, const int64_t*, const T*, const T*,   \
                                   const T*, T*, T, bool);                                     \
    template void launch_restrict_trunc<T>(hipStream_t, int, int, int, const T*, T*);          \
    template void launch_prolong_trunc<T>(hipStream_t, int, int, int, const T*, T*);           \
    template void launch_restrict_dense<T>(hipStream_t, int, int, int, int, const int*,        \
                                           const int*, const int*, const T*, const T*, T*,     \
                                           T*);                                                \
    template void launch_prolong_dense<T>(hipStream_t, int, int, int, const int*, const int*,  \
                                          const T*, const T*, T*);                     \
    template void launch_spmv_sym<T>(hipStream_t, int, int, const SymRows<T>&, const T*,       \
                                     const T*, T*, int, bool, T*);                             \
    template void launch_jacobi_cc_g<T>(hipStream_t, int, int, int, const int*, const int*,    \
                                        const int*, const T*, const int64_t*, const T*,        \
                                        const T*, const T*, const T*, const int*, const int*,  \
                                        const T*, T*, T);                                      \
    template void launch_jacobi_cc<T>(hipStream_t, int, int, int, const int*, const int*,      \
                                      const int*, const T*, const int64_t*, const T*,          \
                                      const T*, const T*, const T*, T*, T, bool);              \
    template void launch_jacobi_sym<T>(hipStream_t, int, const int*, const SymRows<T>&,        \
                                       const int64_t*, const T*, const T*, const T*, T*, T,    \
                                       bool);
XDG_INST(double)
XDG_INST(float)
#undef XDG_INST

}  // namespace xdg
