// Learned per-cell smoother: a 45 -> 64 -> 64 -> 40 MLP with GELU, FP32.
//
// Parameter vector (floats, row-major [out][in]):
//   W1[64][45] b1[64] W2[64][64] b2[64] W3[40][64] b3[40]
// One wavefront evaluates the network for one sample: lane j owns hidden unit
// j (and output j < 40); activations pass between lanes through LDS.
// Training: every wave accumulates the gradient of its samples in registers
// (lane j holds row j of each weight matrix), writes one partial gradient per
// wave, and a second kernel sums the partials in wave order (deterministic).
#include "xdg_internal.h"

namespace xdg {

constexpr int kIn = 45, kHid = 64, kOut = 40;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid,
              oW3 = oB2 + kHid, oB3 = oW3 + kOut * kHid, kParams = oB3 + kOut;
static_assert(kParams == 9704, "parameter count");

__device__ __forceinline__ float gelu_f(float x) {
    return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_df(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
           x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int uniform_l(int v) { return __builtin_amdgcn_readfirstlane(v); }

// y (lanes < 40) = MLP(f); f, h1, h2 are per-wave LDS buffers, P the parameters.
__device__ __forceinline__ float mlp_wave(const float* P, const float* f, float* h1, float* h2,
                                          int lane, float* z1o = nullptr, float* z2o = nullptr) {
    float z = P[oB1 + lane];
    for (int i = 0; i < kIn; ++i) z += P[oW1 + lane * kIn + i] * f[i];
    if (z1o) *z1o = z;
    h1[lane] = gelu_f(z);
    wave_sync_lds();
    z = P[oB2 + lane];
    for (int i = 0; i < kHid; ++i) z += P[oW2 + lane * kHid + i] * h1[i];
    if (z2o) *z2o = z;
    h2[lane] = gelu_f(z);
    wave_sync_lds();
    float y = 0.f;
    if (lane < kOut) {
        y = P[oB3 + lane];
        for (int i = 0; i < kHid; ++i) y += P[oW3 + lane * kHid + i] * h2[i];
    }
    return y;
}

// Y[s] = MLP(X[s]) for n samples (persistent waves, parameters staged in LDS)
__global__ __launch_bounds__(256) void k_mlp_forward(int n, const float* __restrict__ params,
                                                     const float* __restrict__ X,
                                                     float* __restrict__ Y) {
    __shared__ float P[kParams];
    __shared__ float buf[4][kIn + 2 * kHid];
    for (int e = threadIdx.x; e < kParams; e += blockDim.x) P[e] = params[e];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float* f = buf[w];
    float* h1 = f + kIn;
    float* h2 = h1 + kHid;
    for (int s = uniform_l(blockIdx.x * 4 + w); s < n; s += gridDim.x * 4) {
        if (lane < kIn) f[lane] = X[(int64_t)s * kIn + lane];
        wave_sync_lds();
        const float y = mlp_wave(P, f, h1, h2, lane);
        if (lane < kOut) Y[(int64_t)s * kOut + lane] = y;
        wave_sync_lds();
    }
}

// Per-wave partial gradient of loss = sum_s |Y_s - T_s|^2 / n_total over the
// samples s in [s0, s0 + n) owned by this wave; also the partial loss.
__global__ __launch_bounds__(256) void k_mlp_grad(int n, int n_total,
                                                  const float* __restrict__ params,
                                                  const float* __restrict__ X,
                                                  const float* __restrict__ T,
                                                  float* __restrict__ partial,
                                                  float* __restrict__ partial_loss) {
    __shared__ float P[kParams];
    __shared__ float buf[4][kIn + 5 * kHid];
    for (int e = threadIdx.x; e < kParams; e += blockDim.x) P[e] = params[e];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wid = blockIdx.x * 4 + w, nw = gridDim.x * 4;
    float* f = buf[w];
    float* h1 = f + kIn;
    float* h2 = h1 + kHid;
    float* dy = h2 + kHid;
    float* dz2 = dy + kHid;
    float* dz1 = dz2 + kHid;
    float gW1[kIn], gW2[kHid], gW3[kHid];
    float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f, lsum = 0.f;
#pragma unroll
    for (int i = 0; i < kIn; ++i) gW1[i] = 0.f;
#pragma unroll
    for (int i = 0; i < kHid; ++i) gW2[i] = gW3[i] = 0.f;
    const float inv_n = 1.0f / (float)n_total;
    for (int s = uniform_l(wid); s < n; s += nw) {
        if (lane < kIn) f[lane] = X[(int64_t)s * kIn + lane];
        wave_sync_lds();
        float z1, z2;
        const float y = mlp_wave(P, f, h1, h2, lane, &z1, &z2);
        float d = 0.f;
        if (lane < kOut) {
            const float e = y - T[(int64_t)s * kOut + lane];
            lsum += e * e;
            d = 2.0f * e * inv_n;
        }
        dy[lane] = d;
        wave_sync_lds();
        if (lane < kOut) {
#pragma unroll
            for (int i = 0; i < kHid; ++i) gW3[i] += d * h2[i];
            gb3 += d;
        }
        float dh2 = 0.f;
        for (int k = 0; k < kOut; ++k) dh2 += P[oW3 + k * kHid + lane] * dy[k];
        const float d2 = dh2 * gelu_df(z2);
        dz2[lane] = d2;
        wave_sync_lds();
#pragma unroll
        for (int i = 0; i < kHid; ++i) gW2[i] += d2 * h1[i];
        gb2 += d2;
        float dh1 = 0.f;
        for (int k = 0; k < kHid; ++k) dh1 += P[oW2 + k * kHid + lane] * dz2[k];
        const float d1 = dh1 * gelu_df(z1);
#pragma unroll
        for (int i = 0; i < kIn; ++i) gW1[i] += d1 * f[i];
        gb1 += d1;
        wave_sync_lds();
    }
    float* out = partial + (int64_t)wid * kParams;
#pragma unroll
    for (int i = 0; i < kIn; ++i) out[oW1 + lane * kIn + i] = gW1[i];
    out[oB1 + lane] = gb1;
#pragma unroll
    for (int i = 0; i < kHid; ++i) out[oW2 + lane * kHid + i] = gW2[i];
    out[oB2 + lane] = gb2;
    if (lane < kOut) {
#pragma unroll
        for (int i = 0; i < kHid; ++i) out[oW3 + lane * kHid + i] = gW3[i];
        out[oB3 + lane] = gb3;
    }
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if (lane == 0) partial_loss[wid] = lsum * inv_n;
}

// grad[p] = sum over waves (ascending) of partial[w][p]; loss likewise
__global__ void k_mlp_reduce(int nw, const float* __restrict__ partial,
                             const float* __restrict__ partial_loss, float* __restrict__ grad,
                             float* __restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kParams) {
        float s = 0.f;
        for (int w = 0; w < nw; ++w) s += partial[(int64_t)w * kParams + p];
        grad[p] = s;
    }
    if (p == kParams) {
        float s = 0.f;
        for (int w = 0; w < nw; ++w) s += partial_loss[w];
        *loss = s;
    }
}

// Adam: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; w -= lr mhat / (sqrt(vhat) + eps)
__global__ void k_adam(int n, float* __restrict__ w, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.f - b1) * gp;
    const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    w[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// ---------------------------------------------------------------------------
// The learned first sweep of the level-0 smoother (x_in = 0, residual = b):
//   j_c = omega D_c^{-1} b_c,  s = |j_c|,  u = j_c / s placed in the species
//   slots (A: 0..19, B: 20..39), features u | geom_c (5 values);
//   x_c = j_c + s * MLP(features)[slots of the cell's rows]
// (the network proposes the part of the error the damped block-Jacobi step
// misses, in units of that step).
// A cell whose network output is non-finite or larger than `guard` (relative
// to s) keeps the plain Jacobi update (local fallback, counted in *nguard).
// FEAT: instead write, for the selected cells c = cell0 + i cell_step, the
//   features and the target (e_c - j_c) / s with the error e = x* - x_k
//   (b holds the residual of x_k) as sample i -- the training pairs.
// Inference runs over every cell (cell0 = 0, cell_step = 1).
template <bool FEAT>
__global__ __launch_bounds__(256) void k_learned_first(int n_sel, int cell0, int cell_step,
                                                       const int* __restrict__ cell_ptr,
                                                       const int* __restrict__ row_species,
                                                       const float* __restrict__ geom,
                                                       const int64_t* __restrict__ doff,
                                                       const double* __restrict__ D,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ xk,
                                                       const double* __restrict__ xs,
                                                       const float* __restrict__ params,
                                                       double omega, float guard,
                                                       double* __restrict__ x,
                                                       float* __restrict__ Xf,
                                                       float* __restrict__ Tf,
                                                       int* __restrict__ nguard) {
    constexpr int NP = 20;
    __shared__ float P[FEAT ? 1 : kParams];
    __shared__ float buf[4][kIn + 2 * kHid];
    __shared__ double rb[4][2 * NP];
    if (!FEAT) {
        for (int e = threadIdx.x; e < kParams; e += blockDim.x) P[e] = params[e];
        __syncthreads();
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float* f = buf[w];
    float* h1 = f + kIn;
    float* h2 = h1 + kHid;
    int guarded = 0;
    for (int i = uniform_l(blockIdx.x * 4 + w); i < n_sel; i += gridDim.x * 4) {
        const int c = cell0 + i * cell_step;
        const int r0 = uniform_l(cell_ptr[c]), r1 = uniform_l(cell_ptr[c + 1]);
        const int nc = (r1 - r0) * NP;            // 20 or 40 (checked on the host)
        if (lane < nc) rb[w][lane] = b[(int64_t)r0 * NP + lane];
        wave_sync_lds();
        // j = omega D^{-1} b on the cell block (column-major D)
        const double* Dc = D + doff[c];
        double j = 0.0;
        if (lane < nc)
            for (int k = 0; k < nc; ++k) j += Dc[(int64_t)k * nc + lane] * rb[w][k];
        j *= omega;
        double ss = lane < nc ? j * j : 0.0;
        for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
        const double sc = sqrt(ss);
        const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
        if (lane < kOut) f[lane] = 0.f;
        wave_sync_lds();
        if (lane < nc) {
            const int rr = lane / NP, k = lane - rr * NP;
            const int sp = row_species[r0 + rr];
            f[sp * NP + k] = (float)(j * inv);
        }
        if (lane < 5) f[kOut + lane] = geom[(int64_t)c * 5 + lane];
        wave_sync_lds();
        if constexpr (FEAT) {
            if (lane < kIn) Xf[(int64_t)i * kIn + lane] = f[lane];
            if (lane < kOut) h2[lane] = 0.f;
            wave_sync_lds();
            if (lane < nc) {
                const int rr = lane / NP, k = lane - rr * NP;
                const int sp = row_species[r0 + rr];
                const int64_t o = (int64_t)r0 * NP + lane;
                h2[sp * NP + k] = (float)(((xs[o] - xk[o]) - j) * inv);
            }
            wave_sync_lds();
            if (lane < kOut) Tf[(int64_t)i * kOut + lane] = h2[lane];
            wave_sync_lds();
            continue;
        } else {
        float y = mlp_wave(P, f, h1, h2, lane);
        // local fallback: non-finite or oversized proposals keep plain Jacobi
        float yy = lane < kOut ? y * y : 0.f;
        bool bad = !(y == y) || fabsf(y) > 3.0e38f;
        for (int off = 32; off > 0; off >>= 1) yy += __shfl_xor(yy, off, 64);
        bad = __any(bad) || !(sqrtf(yy) <= guard);
        if (bad) guarded += 1;
        wave_sync_lds();
        h1[lane] = bad ? 0.f : y;                 // reuse h1 as the output slot buffer
        wave_sync_lds();
        if (lane < nc) {
            const int rr = lane / NP, k = lane - rr * NP;
            const int sp = row_species[r0 + rr];
            x[(int64_t)r0 * NP + lane] = j + sc * (double)h1[sp * NP + k];
        }
        wave_sync_lds();
        }
    }
    if (!FEAT && lane == 0 && guarded) atomicAdd(nguard, guarded);
}

// ---------------------------------------------------------------------------
static inline unsigned nbk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

int mlp_param_count() { return kParams; }

void launch_mlp_forward(hipStream_t s, int n, const float* params, const float* X, float* Y) {
    const int g = (int)std::min<int64_t>(nbk(n, 4), 1024);
    k_mlp_forward<<<std::max(g, 1), 256, 0, s>>>(n, params, X, Y);
}

void launch_mlp_grad(hipStream_t s, int n, int n_total, int n_blocks, const float* params,
                     const float* X, const float* T, float* partial, float* partial_loss,
                     float* grad, float* loss) {
    k_mlp_grad<<<n_blocks, 256, 0, s>>>(n, n_total, params, X, T, partial, partial_loss);
    k_mlp_reduce<<<nbk(kParams + 1, 256), 256, 0, s>>>(n_blocks * 4, partial, partial_loss, grad,
                                                       loss);
}

void launch_adam(hipStream_t s, float* w, const float* g, float* m, float* v, float lr, float b1,
                 float b2, float c1, float c2, float eps) {
    k_adam<<<nbk(kParams, 256), 256, 0, s>>>(kParams, w, g, m, v, lr, b1, b2, c1, c2, eps);
}

void launch_learned_first(hipStream_t s, int n_cells, const int* cp, const int* row_species,
                          const float* geom, const int64_t* doff, const double* D,
                          const double* b, const float* params, double omega, float guard,
                          double* x, int* nguard) {
    const int g = (int)std::min<int64_t>(nbk(n_cells, 4), 2048);
    k_learned_first<false><<<std::max(g, 1), 256, 0, s>>>(n_cells, 0, 1, cp, row_species, geom, doff,
                                                           D, b, nullptr, nullptr, params, omega,
                                                           guard, x, nullptr, nullptr, nguard);
}

void launch_learned_features(hipStream_t s, int n_sel, int cell0, int cell_step, const int* cp,
                             const int* row_species, const float* geom, const int64_t* doff,
                             const double* D, const double* r, const double* xk,
                             const double* xs, double omega, float* Xf, float* Tf) {
    const int g = (int)std::min<int64_t>(nbk(n_sel, 4), 2048);
    k_learned_first<true><<<std::max(g, 1), 256, 0, s>>>(n_sel, cell0, cell_step, cp, row_species,
                                                          geom, doff, D,
                                                          r, xk, xs, nullptr, omega, 0.f, nullptr,
                                                          Xf, Tf, nullptr);
}

}  // namespace xdg
