// FP64 vector kernels of the Krylov solvers: deterministic inner products
// (fixed grid, fixed per-thread order, fixed tree) and fused CG updates whose
// scalars stay in device memory.
#include "xdg_internal.h"

namespace xdg {

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__device__ __forceinline__ double block_sum(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
    return t;   // valid in thread 0
}

__global__ __launch_bounds__(256) void k_dot_partial(int64_t n, const double* __restrict__ a,
                                                     const double* __restrict__ b,
                                                     double* __restrict__ partial) {
    __shared__ double sh[4];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        acc += a[i] * b[i];
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_dot_final(const double* __restrict__ partial, int np,
                                                   double* __restrict__ out) {
    __shared__ double sh[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partial[i];
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) *out = t;
}

// x += alpha p, r -= alpha q with alpha = scal[i_rz] / scal[i_pq]
__global__ void k_cg_update_xr(int64_t n, const double* __restrict__ scal, int i_rz, int i_pq,
                               const double* __restrict__ p, const double* __restrict__ q,
                               double* __restrict__ x, double* __restrict__ r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double alpha = scal[i_rz] / scal[i_pq];
    x[i] += alpha * p[i];
    r[i] -= alpha * q[i];
}

// the CG update and the partial sums of the new r . r over the grid of
// k_dot_partial (same threads, same order)
__global__ __launch_bounds__(256) void k_cg_update_xr_dot(int64_t n,
                                                          const double* __restrict__ scal,
                                                          int i_rz, int i_pq,
                                                          const double* __restrict__ p,
                                                          const double* __restrict__ q,
                                                          double* __restrict__ x,
                                                          double* __restrict__ r,
                                                          double* __restrict__ partial) {
    __shared__ double sh[4];
    const double alpha = scal[i_rz] / scal[i_pq];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += ri * ri;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// p = z + beta p with beta = scal[i_new] / scal[i_old]
__global__ void k_cg_update_p(int64_t n, const double* __restrict__ scal, int i_new, int i_old,
                              const double* __restrict__ z, double* __restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double beta = scal[i_new] / scal[i_old];
    p[i] = z[i] + beta * p[i];
}

// flexible CG direction: p = z - (scal[i_zq] / scal[i_pq]) p
__global__ void k_fcg_update_p(int64_t n, const double* __restrict__ scal, int i_zq, int i_pq,
                               const double* __restrict__ z, double* __restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double beta = scal[i_zq] / scal[i_pq];
    p[i] = z[i] - beta * p[i];
}

__global__ void k_axpy(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += a * x[i];
}

__global__ void k_scale_copy(int64_t n, double a, const double* __restrict__ x,
                             double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i];
}

void launch_dot(hipStream_t s, int64_t n, const double* a, const double* b, double* partial,
                double* out) {
    k_dot_partial<<<kDotBlocks, 256, 0, s>>>(n, a, b, partial);
    k_dot_final<<<1, 256, 0, s>>>(partial, kDotBlocks, out);
}
void launch_cg_update_xr(hipStream_t s, int64_t n, const double* scal, int i_rz, int i_pq,
                         const double* p, const double* q, double* x, double* r) {
    k_cg_update_xr<<<nblk(n, 256), 256, 0, s>>>(n, scal, i_rz, i_pq, p, q, x, r);
}
void launch_cg_update_xr_dot(hipStream_t s, int64_t n, double* scal, int i_rz, int i_pq,
                             int i_rr, const double* p, const double* q, double* x, double* r,
                             double* partial) {
    k_cg_update_xr_dot<<<kDotBlocks, 256, 0, s>>>(n, scal, i_rz, i_pq, p, q, x, r, partial);
    k_dot_final<<<1, 256, 0, s>>>(partial, kDotBlocks, scal + i_rr);
}
// fixed-order sum of many partials (one per workgroup of a fused product):
// 1024 threads, coalesced strided reads, then the wave and workgroup trees
__global__ __launch_bounds__(1024) void k_dot_final_wide(const double* __restrict__ partial,
                                                         int np, double* __restrict__ out) {
    __shared__ double sh[16];
    double acc = 0.0;
    // the thread's strided partials in order; eight loads in flight at a time
    constexpr int U = 8;
    const int stride = (int)blockDim.x;
    int i = threadIdx.x;
    for (; i + (U - 1) * stride < np; i += U * stride) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = partial[i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) acc += v[u];
    }
    for (; i < np; i += stride) acc += partial[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
        *out = t;
    }
}
void launch_dot_final(hipStream_t s, const double* partial, int np, double* out) {
    k_dot_final_wide<<<1, 1024, 0, s>>>(partial, np, out);
}
void launch_cg_update_p(hipStream_t s, int64_t n, const double* scal, int i_new, int i_old,
                        const double* z, double* p) {
    k_cg_update_p<<<nblk(n, 256), 256, 0, s>>>(n, scal, i_new, i_old, z, p);
}
void launch_fcg_update_p(hipStream_t s, int64_t n, const double* scal, int i_zq, int i_pq,
                         const double* z, double* p) {
    k_fcg_update_p<<<nblk(n, 256), 256, 0, s>>>(n, scal, i_zq, i_pq, z, p);
}
// scal[i] = sqrt(scal[i]); a zero (or negative) value becomes +inf so that a
// division by it yields zero
__global__ void k_sqrt_scalar(double* scal, int i) {
    const double v = scal[i];
    scal[i] = v > 0.0 ? sqrt(v) : __builtin_inf();
}
void launch_sqrt_scalar(hipStream_t s, double* scal, int i) {
    k_sqrt_scalar<<<1, 1, 0, s>>>(scal, i);
}
template <typename T>
__global__ void k_fill_zero(int64_t n, T* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = T(0);
}
// x = 0 by a kernel (no memset node when the caller captures the stream)
template <typename T>
void launch_fill_zero(hipStream_t s, int64_t n, T* x) {
    if (n > 0) k_fill_zero<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, x);
}
template void launch_fill_zero<double>(hipStream_t, int64_t, double*);
template void launch_fill_zero<float>(hipStream_t, int64_t, float*);

void launch_axpy(hipStream_t s, int64_t n, double a, const double* x, double* y) {
    k_axpy<<<nblk(n, 256), 256, 0, s>>>(n, a, x, y);
}
void launch_scale_copy(hipStream_t s, int64_t n, double a, const double* x, double* y) {
    k_scale_copy<<<nblk(n, 256), 256, 0, s>>>(n, a, x, y);
}

}  // namespace xdg

namespace xdg {

// partial[k][blk] = sum over this block's slice of V[k] . w
__global__ __launch_bounds__(256) void k_multidot_partial(int64_t n, int nv,
                                                          const double* __restrict__ V,
                                                          const double* __restrict__ w,
                                                          double* __restrict__ partial) {
    // groups of kG basis vectors share one pass over w; per-thread sums in
    // ascending index order, then the fixed block reduction per vector
    constexpr int kG = 8;
    __shared__ double sh[4];
    for (int k0 = 0; k0 < nv; k0 += kG) {
        const int g = min(kG, nv - k0);
        double acc[kG];
#pragma unroll
        for (int q = 0; q < kG; ++q) acc[q] = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * blockDim.x) {
            const double wv = w[i];
#pragma unroll
            for (int q = 0; q < kG; ++q)
                if (q < g) acc[q] += V[(int64_t)(k0 + q) * n + i] * wv;
        }
#pragma unroll
        for (int q = 0; q < kG; ++q) {
            if (q < g) {                      // g is uniform: every thread takes the same path
                const double t = block_sum(acc[q], sh);
                if (threadIdx.x == 0) partial[(int64_t)(k0 + q) * gridDim.x + blockIdx.x] = t;
                __syncthreads();
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_multidot_final(int nv, int nb,
                                                        const double* __restrict__ partial,
                                                        double* __restrict__ out) {
    __shared__ double sh[4];
    const int k = blockIdx.x;
    if (k >= nv) return;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += partial[(int64_t)k * nb + i];
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) out[k] = t;
}

template <bool NEG>
__global__ void k_multi_axpy(int64_t n, int nv, const double* __restrict__ V,
                             const double* __restrict__ coef, double* __restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int k = 0; k < nv; ++k) acc += coef[k] * V[(int64_t)k * n + i];
    w[i] = NEG ? w[i] - acc : w[i] + acc;
}

__global__ void k_div_scalar(int64_t n, const double* __restrict__ scal, int idx,
                             const double* __restrict__ x, double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i] / scal[idx];
}

void launch_multidot(hipStream_t s, int64_t n, int nv, const double* V, const double* w,
                     double* partial, double* out) {
    k_multidot_partial<<<kDotBlocks, 256, 0, s>>>(n, nv, V, w, partial);
    k_multidot_final<<<nv, 256, 0, s>>>(nv, kDotBlocks, partial, out);
}
void launch_multi_axpy_neg(hipStream_t s, int64_t n, int nv, const double* V, const double* coef,
                           double* w) {
    k_multi_axpy<true><<<nblk(n, 256), 256, 0, s>>>(n, nv, V, coef, w);
}
void launch_multi_axpy(hipStream_t s, int64_t n, int nv, const double* V, const double* coef,
                       double* x) {
    k_multi_axpy<false><<<nblk(n, 256), 256, 0, s>>>(n, nv, V, coef, x);
}
void launch_div_scalar(hipStream_t s, int64_t n, const double* scal, int i, const double* x,
                       double* y) {
    k_div_scalar<<<nblk(n, 256), 256, 0, s>>>(n, scal, i, x, y);
}

}  // namespace xdg
