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

// LDS copy of the parameters: rows of W2 and W3 padded to an odd stride so
// that both the forward products (lane = output row) and the backward
// products (lane = input column) read distinct banks; W1 rows (45) are odd.
constexpr int kS1 = kIn, kS2 = kHid + 1, kS3 = kHid + 1;
constexpr int lW1 = 0, lB1 = lW1 + kHid * kS1, lW2 = lB1 + kHid, lB2 = lW2 + kHid * kS2,
              lW3 = lB2 + kHid, lB3 = lW3 + kOut * kS3, kLds = lB3 + kOut;

__device__ __forceinline__ void stage_params(float* P, const float* __restrict__ g) {
    for (int e = threadIdx.x; e < kParams; e += blockDim.x) {
        int d;
        if (e < oB1) d = e;                                                   // W1, stride 45
        else if (e < oW2) d = lB1 + (e - oB1);
        else if (e < oB2) d = lW2 + ((e - oW2) / kHid) * kS2 + (e - oW2) % kHid;
        else if (e < oW3) d = lB2 + (e - oB2);
        else if (e < oB3) d = lW3 + ((e - oW3) / kHid) * kS3 + (e - oW3) % kHid;
        else d = lB3 + (e - oB3);
        P[d] = g[e];
    }
}

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

// y (lanes < 40) = MLP(f); f, h1, h2 are per-wave LDS buffers, P the
// parameters in the padded LDS layout.
__device__ __forceinline__ float mlp_wave(const float* P, const float* f, float* h1, float* h2,
                                          int lane, float* z1o = nullptr, float* z2o = nullptr) {
    float z = P[lB1 + lane];
#pragma unroll 9
    for (int i = 0; i < kIn; ++i) z += P[lW1 + lane * kS1 + i] * f[i];
    if (z1o) *z1o = z;
    h1[lane] = gelu_f(z);
    wave_sync_lds();
    z = P[lB2 + lane];
#pragma unroll 8
    for (int i = 0; i < kHid; ++i) z += P[lW2 + lane * kS2 + i] * h1[i];
    if (z2o) *z2o = z;
    h2[lane] = gelu_f(z);
    wave_sync_lds();
    float y = 0.f;
    if (lane < kOut) {
        y = P[lB3 + lane];
#pragma unroll 8
        for (int i = 0; i < kHid; ++i) y += P[lW3 + lane * kS3 + i] * h2[i];
    }
    return y;
}

// Inference with the weights in registers: lane j holds row j of W1 and W2
// and (j < 40) row j of W3; the activations of the previous layer are
// broadcast one at a time with readlane (no LDS traffic per weight).
struct MlpRegs {
    float w1[kIn], w2[kHid], w3[kHid];
    float b1, b2, b3;
};

__device__ __forceinline__ void load_regs(MlpRegs& R, const float* __restrict__ g, int lane) {
#pragma unroll
    for (int i = 0; i < kIn; ++i) R.w1[i] = g[oW1 + lane * kIn + i];
#pragma unroll
    for (int i = 0; i < kHid; ++i) R.w2[i] = g[oW2 + lane * kHid + i];
#pragma unroll
    for (int i = 0; i < kHid; ++i) R.w3[i] = lane < kOut ? g[oW3 + lane * kHid + i] : 0.f;
    R.b1 = g[oB1 + lane];
    R.b2 = g[oB2 + lane];
    R.b3 = lane < kOut ? g[oB3 + lane] : 0.f;
}

// f (inputs), h1, h2: per-wave LDS buffers; the weights come from registers
// and every activation is read by all lanes at once (an LDS broadcast).
// Returns output `lane` (valid for lane < 40).
__device__ __forceinline__ float mlp_regs(const MlpRegs& R, const float* f, float* h1, float* h2,
                                          int lane) {
    float z = R.b1;
#pragma unroll
    for (int i = 0; i < kIn; ++i) z += R.w1[i] * f[i];
    h1[lane] = gelu_f(z);
    wave_sync_lds();
    z = R.b2;
#pragma unroll
    for (int i = 0; i < kHid; ++i) z += R.w2[i] * h1[i];
    h2[lane] = gelu_f(z);
    wave_sync_lds();
    float y = R.b3;
#pragma unroll
    for (int i = 0; i < kHid; ++i) y += R.w3[i] * h2[i];
    return y;
}

// Y[s] = MLP(X[s]) for n samples (persistent waves, weights in registers)
__global__ __launch_bounds__(256) void k_mlp_forward(int n, const float* __restrict__ params,
                                                     const float* __restrict__ X,
                                                     float* __restrict__ Y) {
    __shared__ float act[4][48 + 2 * kHid];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    MlpRegs R;
    load_regs(R, params, lane);
    float* f = act[w];
    for (int s = uniform_l(blockIdx.x * 4 + w); s < n; s += gridDim.x * 4) {
        if (lane < kIn) f[lane] = X[(int64_t)s * kIn + lane];
        wave_sync_lds();
        const float y = mlp_regs(R, f, f + 48, f + 48 + kHid, lane);
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
    __shared__ float P[kLds];
    __shared__ float buf[4][kIn + 5 * kHid];
    stage_params(P, params);
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
#pragma unroll 8
        for (int k = 0; k < kOut; ++k) dh2 += P[lW3 + k * kS3 + lane] * dy[k];
        const float d2 = dh2 * gelu_df(z2);
        dz2[lane] = d2;
        wave_sync_lds();
#pragma unroll
        for (int i = 0; i < kHid; ++i) gW2[i] += d2 * h1[i];
        gb2 += d2;
        float dh1 = 0.f;
#pragma unroll 8
        for (int k = 0; k < kHid; ++k) dh1 += P[lW2 + k * kS2 + lane] * dz2[k];
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
// Training pairs of the learned first sweep.  For the selected cells
// c = cell0 + i cell_step and the residual b of an iterate x_k:
//   j_c = omega D_c^{-1} b_c,  s = |j_c|,  features u | geom_c with u = j_c / s
//   placed in the species slots (A: 0..19, B: 20..39), and the target
//   (e_c - j_c) / s with the error e = x* - x_k, in the same slots, scaled to
//   norm `clip` when longer (clip = 0: no scaling); written as sample i.
__global__ __launch_bounds__(256) void k_learned_pairs(int n_sel, int cell0, int cell_step,
                                                       const int* __restrict__ cell_ptr,
                                                       const int* __restrict__ row_species,
                                                       const float* __restrict__ geom,
                                                       const int64_t* __restrict__ doff,
                                                       const double* __restrict__ D,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ xk,
                                                       const double* __restrict__ xs,
                                                       double omega, float clip,
                                                       float* __restrict__ Xf,
                                                       float* __restrict__ Tf) {
    constexpr int NP = 20;
    __shared__ float buf[4][kIn + kOut];
    __shared__ double rb[4][2 * NP];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float* f = buf[w];
    float* t_s = f + kIn;
    for (int i = uniform_l(blockIdx.x * 4 + w); i < n_sel; i += gridDim.x * 4) {
        const int c = cell0 + i * cell_step;
        const int r0 = uniform_l(cell_ptr[c]), r1 = uniform_l(cell_ptr[c + 1]);
        const int nc = (r1 - r0) * NP;            // 20 or 40 (checked on the host)
        if (lane < nc) rb[w][lane] = b[(int64_t)r0 * NP + lane];
        wave_sync_lds();
        // j = omega D^{-1} b on the cell block (column-major D), unrolled for
        // the two cell sizes so that the column loads overlap
        const double* Dc = D + doff[c];
        double j = 0.0;
        if (lane < nc) {
            if (nc == NP) {
#pragma unroll
                for (int k = 0; k < NP; ++k) j += Dc[k * NP + lane] * rb[w][k];
            } else {
#pragma unroll
                for (int k = 0; k < 2 * NP; ++k) j += Dc[k * 2 * NP + lane] * rb[w][k];
            }
        }
        j *= omega;
        double ss = lane < nc ? j * j : 0.0;
        for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
        const double sc = sqrt(ss);
        const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
        int slot = 0;
        if (lane < nc) {
            const int rr = lane / NP;
            slot = row_species[r0 + rr] * NP + (lane - rr * NP);
        }
        double t = 0.0;
        if (lane < nc) t = ((xs[(int64_t)r0 * NP + lane] - xk[(int64_t)r0 * NP + lane]) - j) * inv;
        double tt = t * t;
        for (int off = 32; off > 0; off >>= 1) tt += __shfl_xor(tt, off, 64);
        const double tn = sqrt(tt);
        if (clip > 0.f && tn > (double)clip) t *= (double)clip / tn;
        if (lane < kOut) f[lane] = 0.f;
        if (lane < kOut) t_s[lane] = 0.f;
        wave_sync_lds();
        if (lane < nc) {
            f[slot] = (float)(j * inv);
            t_s[slot] = (float)t;
        }
        if (lane < 5) f[kOut + lane] = geom[(int64_t)c * 5 + lane];
        wave_sync_lds();
        if (lane < kIn) Xf[(int64_t)i * kIn + lane] = f[lane];
        if (lane < kOut) Tf[(int64_t)i * kOut + lane] = t_s[lane];
        wave_sync_lds();
    }
}

// ---------------------------------------------------------------------------
// The learned correction of the first sweep, applied after the plain first
// sweep has written j = omega D^{-1} b into x: per cell, s = |j_c|,
// features [j_c / s in species slots | geom_c], x_c = j_c + s * MLP(features).
// A wave takes chunks of kChunk consecutive cells: one round of loads brings
// the chunk's rows of x, row species, geometry and cell pointers into LDS,
// then the cells are evaluated one after another (weights in registers,
// activations read from LDS as broadcasts), and the chunk is written back.
constexpr int kChunk = 8;
constexpr int kChunkRows = 2 * kChunk;

__global__ __launch_bounds__(256) void k_learned_correct(int n_cells, const int* __restrict__ cell_ptr,
                                                         const int* __restrict__ row_species,
                                                         const float* __restrict__ geom,
                                                         const float* __restrict__ params,
                                                         float guard, double* __restrict__ x,
                                                         int* __restrict__ nguard) {
    constexpr int NP = 20;
    __shared__ double xs[4][kChunkRows * NP];
    __shared__ float act[4][48 + 2 * kHid];
    __shared__ float gs[4][kChunk * 5];
    __shared__ int spc[4][kChunkRows];
    __shared__ int cps[4][kChunk + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    MlpRegs R;
    load_regs(R, params, lane);
    float* f = act[w];
    float* h1 = f + 48;
    float* h2 = h1 + kHid;
    int guarded = 0;
    const int n_chunks = (n_cells + kChunk - 1) / kChunk;
    for (int ch = uniform_l(blockIdx.x * 4 + w); ch < n_chunks; ch += gridDim.x * 4) {
        const int c0 = ch * kChunk;
        const int nch = min(kChunk, n_cells - c0);
        if (lane <= nch) cps[w][lane] = cell_ptr[c0 + lane];
        if (lane < nch * 5) gs[w][lane] = geom[(int64_t)c0 * 5 + lane];
        wave_sync_lds();
        const int R0 = uniform_l(cps[w][0]), R1 = uniform_l(cps[w][nch]);
        const int nv = (R1 - R0) * NP;                 // <= kChunkRows * NP (host-checked cells)
        for (int k = lane; k < nv; k += 64) xs[w][k] = x[(int64_t)R0 * NP + k];
        if (lane < R1 - R0) spc[w][lane] = row_species[R0 + lane];
        wave_sync_lds();
        for (int cc = 0; cc < nch; ++cc) {
            const int r0 = uniform_l(cps[w][cc]) - R0, r1 = uniform_l(cps[w][cc + 1]) - R0;
            const int nc = (r1 - r0) * NP;
            const double j = lane < nc ? xs[w][r0 * NP + lane] : 0.0;
            double ss = j * j;
            for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
            const double sc = sqrt(ss);
            const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
            int slot = 0;
            if (lane < nc) {
                const int rr = lane / NP;
                slot = spc[w][r0 + rr] * NP + (lane - rr * NP);
            }
            if (lane < kOut) f[lane] = 0.f;
            wave_sync_lds();
            if (lane < nc) f[slot] = (float)(j * inv);
            if (lane < 5) f[kOut + lane] = gs[w][cc * 5 + lane];
            wave_sync_lds();
            const float y = mlp_regs(R, f, h1, h2, lane);
            // local fallback: non-finite or oversized proposals keep plain Jacobi
            float yy = lane < kOut ? y * y : 0.f;
            bool bad = lane < kOut && (!(y == y) || fabsf(y) > 3.0e38f);
            for (int off = 32; off > 0; off >>= 1) yy += __shfl_xor(yy, off, 64);
            bad = __any(bad) || !(sqrtf(yy) <= guard);
            if (bad) guarded += 1;
            const float ys = __shfl(y, slot, 64);
            if (lane < nc && !bad) xs[w][r0 * NP + lane] = j + sc * (double)ys;
            wave_sync_lds();
        }
        for (int k = lane; k < nv; k += 64) x[(int64_t)R0 * NP + k] = xs[w][k];
        wave_sync_lds();
    }
    if (lane == 0 && guarded) atomicAdd(nguard, guarded);
}

// ---------------------------------------------------------------------------
// BF16 inference: 16 cells per wave through the three layers as
// v_mfma_f32_16x16x16_bf16 products (bf16 operands, FP32 accumulation).
// Lane layouts (checked on gfx950): A lane l holds A[l % 16][4 (l / 16) + i],
// B lane l holds B[4 (l / 16) + i][l % 16], D lane l holds
// D[4 (l / 16) + r][l % 16], i, r < 4.  Rows are cells; the weights are the
// B operands, packed once per parameter change: tile (t, q) of layer L holds
// W_L[16 t + n][16 q + k] at B[k][n] (zero outside the matrix; the 45 inputs
// are padded to 48, the 40 outputs to 48).
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kT1 = 4, kQ1 = 3, kT2 = 4, kQ2 = 4, kT3 = 3, kQ3 = 4;
constexpr int kTiles = kT1 * kQ1 + kT2 * kQ2 + kT3 * kQ3;   // 40 operand tiles
constexpr int kPackedBf16 = kTiles * 64 * 4;

__device__ __forceinline__ unsigned short to_bf16(float f) {
    // round to nearest even (finite inputs; NaN stays NaN through the guard)
    const unsigned u = __float_as_uint(f);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__global__ void k_pack_bf16(const float* __restrict__ P, unsigned short* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kPackedBf16) return;
    const int i = e & 3, l = (e >> 2) & 63, tile = e >> 8;
    const int n = l & 15, k = 4 * (l >> 4) + i;
    float v = 0.f;
    if (tile < kT1 * kQ1) {
        const int t = tile / kQ1, q = tile % kQ1, row = 16 * t + n, col = 16 * q + k;
        if (col < kIn) v = P[oW1 + row * kIn + col];
    } else if (tile < kT1 * kQ1 + kT2 * kQ2) {
        const int tt = tile - kT1 * kQ1, t = tt / kQ2, q = tt % kQ2;
        v = P[oW2 + (16 * t + n) * kHid + 16 * q + k];
    } else {
        const int tt = tile - kT1 * kQ1 - kT2 * kQ2, t = tt / kQ3, q = tt % kQ3;
        const int row = 16 * t + n;
        if (row < kOut) v = P[oW3 + row * kHid + 16 * q + k];
    }
    out[e] = to_bf16(v);
}

constexpr int kBatch = 16;                 // cells per wave and batch (MFMA rows)
constexpr int kBatchRows = 2 * kBatch;

__global__ __launch_bounds__(256) void k_learned_correct_bf16(
    int n_cells, const int* __restrict__ cell_ptr, const int* __restrict__ row_species,
    const float* __restrict__ geom, const unsigned short* __restrict__ wpk,
    const float* __restrict__ params, float guard, double* __restrict__ x,
    int* __restrict__ nguard) {
    constexpr int NP = 20;
    __shared__ double xs[4][kBatchRows * NP];
    __shared__ double scs[4][kBatch];
    __shared__ __align__(16) unsigned short fa[4][kBatch][48];          // features (A operand of layer 1)
    __shared__ __align__(16) unsigned short ha[4][kBatch][kHid];        // hidden layer 1
    __shared__ __align__(16) unsigned short hb[4][kBatch][kHid];        // hidden layer 2
    __shared__ float ya[4][kBatch][48];                    // outputs
    __shared__ float gs[4][kBatch * 5];
    __shared__ int badc[4][kBatch];
    __shared__ int spc[4][kBatchRows];
    __shared__ int cps[4][kBatch + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    // weight operands and biases in registers
    bf16x4 B1[kT1 * kQ1], B2[kT2 * kQ2], B3[kT3 * kQ3];
    const bf16x4* W = reinterpret_cast<const bf16x4*>(wpk);
#pragma unroll
    for (int t = 0; t < kT1 * kQ1; ++t) B1[t] = W[t * 64 + lane];
#pragma unroll
    for (int t = 0; t < kT2 * kQ2; ++t) B2[t] = W[(kT1 * kQ1 + t) * 64 + lane];
#pragma unroll
    for (int t = 0; t < kT3 * kQ3; ++t) B3[t] = W[(kT1 * kQ1 + kT2 * kQ2 + t) * 64 + lane];
    float bb1[kT1], bb2[kT2], bb3[kT3];
#pragma unroll
    for (int t = 0; t < kT1; ++t) bb1[t] = params[oB1 + 16 * t + li];
#pragma unroll
    for (int t = 0; t < kT2; ++t) bb2[t] = params[oB2 + 16 * t + li];
#pragma unroll
    for (int t = 0; t < kT3; ++t) bb3[t] = 16 * t + li < kOut ? params[oB3 + 16 * t + li] : 0.f;
    int guarded = 0;
    const int n_batches = (n_cells + kBatch - 1) / kBatch;
    constexpr int kXv = kBatchRows * NP / 64;      // x values per lane and batch
    // next batch, loaded while the current one runs: cell pointers and
    // geometry first, then (once the pointers are in) x and the species
    int cp_n = 0;
    float g_n0 = 0.f, g_n1 = 0.f;
    double xv[kXv];
    int sp_n = 0;
    auto fetch_cells = [&](int b) {
        if (b >= n_batches) return;
        const int c0 = b * kBatch, nch = min(kBatch, n_cells - c0);
        cp_n = lane <= nch ? cell_ptr[c0 + lane] : 0;
        g_n0 = lane < nch * 5 ? geom[(int64_t)c0 * 5 + lane] : 0.f;
        g_n1 = lane + 64 < nch * 5 ? geom[(int64_t)c0 * 5 + lane + 64] : 0.f;
    };
    auto fetch_rows = [&](int b) {
        if (b >= n_batches) return;
        const int nch = min(kBatch, n_cells - b * kBatch);
        const int R0 = uniform_l(__shfl(cp_n, 0, 64)), R1 = uniform_l(__shfl(cp_n, nch, 64));
        const int nv = (R1 - R0) * NP;           // <= kBatchRows * NP (host-checked cells)
#pragma unroll
        for (int k = 0; k < kXv; ++k)
            xv[k] = lane + 64 * k < nv ? x[(int64_t)R0 * NP + lane + 64 * k] : 0.0;
        sp_n = lane < R1 - R0 ? row_species[R0 + lane] : 0;
    };
    const int stride = gridDim.x * 4;
    int bt = uniform_l(blockIdx.x * 4 + w);
    fetch_cells(bt);
    fetch_rows(bt);
    for (; bt < n_batches; bt += stride) {
        const int c0 = bt * kBatch;
        const int nch = min(kBatch, n_cells - c0);
        const int R0 = uniform_l(__shfl(cp_n, 0, 64)), R1 = uniform_l(__shfl(cp_n, nch, 64));
        const int nv = (R1 - R0) * NP;
        if (lane <= nch) cps[w][lane] = cp_n;
        if (lane < nch * 5) gs[w][lane] = g_n0;
        if (lane + 64 < nch * 5) gs[w][lane + 64] = g_n1;
#pragma unroll
        for (int k = 0; k < kXv; ++k)
            if (lane + 64 * k < nv) xs[w][lane + 64 * k] = xv[k];
        if (lane < R1 - R0) spc[w][lane] = sp_n;
        for (int e = lane; e < kBatch * 24; e += 64) reinterpret_cast<unsigned*>(&fa[w][0][0])[e] = 0u;
        fetch_cells(bt + stride);
        wave_sync_lds();
        // per cell (four lanes each): Jacobi-step norm and the normalised features
        const int gc = lane >> 2, sub = lane & 3;
        int r0 = 0, nc = 0;
        if (gc < nch) {
            r0 = cps[w][gc] - R0;
            nc = (cps[w][gc + 1] - R0 - r0) * NP;
        }
        double ss = 0.0;
        for (int v = sub; v < nc; v += 4) {
            const double j = xs[w][r0 * NP + v];
            ss += j * j;
        }
        ss += __shfl_xor(ss, 1, 64);
        ss += __shfl_xor(ss, 2, 64);
        const double sc = sqrt(ss);
        const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
        if (sub == 0 && gc < nch) scs[w][gc] = sc;
        for (int v = sub; v < nc; v += 4) {
            const int rr = v / NP;
            fa[w][gc][spc[w][r0 + rr] * NP + (v - rr * NP)] =
                to_bf16((float)(xs[w][r0 * NP + v] * inv));
        }
        if (gc < nch)
            for (int e = sub; e < 5; e += 4) fa[w][gc][kOut + e] = to_bf16(gs[w][gc * 5 + e]);
        fetch_rows(bt + stride);
        wave_sync_lds();
        // layer 1: [16 x 48] x [48 x 64]
        f32x4_t acc[4];
#pragma unroll
        for (int t = 0; t < kT1; ++t) acc[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < kQ1; ++q) {
            const bf16x4 a = *reinterpret_cast<const bf16x4*>(&fa[w][li][16 * q + 4 * lk]);
#pragma unroll
            for (int t = 0; t < kT1; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, B1[t * kQ1 + q], acc[t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < kT1; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                ha[w][4 * lk + r][16 * t + li] = to_bf16(gelu_f(acc[t][r] + bb1[t]));
        wave_sync_lds();
        // layer 2: [16 x 64] x [64 x 64]
#pragma unroll
        for (int t = 0; t < kT2; ++t) acc[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < kQ2; ++q) {
            const bf16x4 a = *reinterpret_cast<const bf16x4*>(&ha[w][li][16 * q + 4 * lk]);
#pragma unroll
            for (int t = 0; t < kT2; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, B2[t * kQ2 + q], acc[t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < kT2; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                hb[w][4 * lk + r][16 * t + li] = to_bf16(gelu_f(acc[t][r] + bb2[t]));
        wave_sync_lds();
        // layer 3: [16 x 64] x [64 x 48]
#pragma unroll
        for (int t = 0; t < kT3; ++t) acc[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < kQ3; ++q) {
            const bf16x4 a = *reinterpret_cast<const bf16x4*>(&hb[w][li][16 * q + 4 * lk]);
#pragma unroll
            for (int t = 0; t < kT3; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, B3[t * kQ3 + q], acc[t], 0, 0, 0);
        }
        // guard from the accumulators: lane (li, lk) holds outputs 16 t + li of
        // cells 4 lk + r; columns 40..47 are exactly zero (zero weights, bias)
        float yy[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            yy[r] = 0.f;
#pragma unroll
            for (int t = 0; t < kT3; ++t) {
                const float y = acc[t][r] + bb3[t];
                ya[w][4 * lk + r][16 * t + li] = y;
                yy[r] += y * y;
            }
        }
#pragma unroll
        for (int off = 1; off < 16; off <<= 1)
#pragma unroll
            for (int r = 0; r < 4; ++r) yy[r] += __shfl_xor(yy[r], off, 64);
        if (li == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // a non-finite proposal gives a non-finite sum: NaN <= guard is false
                const bool bad = !(sqrtf(yy[r]) <= guard);
                badc[w][4 * lk + r] = bad;
                if (bad && 4 * lk + r < nch) guarded += 1;
            }
        }
        wave_sync_lds();
        // per cell (four lanes each): x_c = j_c + s_c y_c unless guarded
        if (gc < nch && !badc[w][gc]) {
            const double scc = scs[w][gc];
            for (int v = sub; v < nc; v += 4) {
                const int rr = v / NP;
                xs[w][r0 * NP + v] += scc * (double)ya[w][gc][spc[w][r0 + rr] * NP + (v - rr * NP)];
            }
        }
        wave_sync_lds();
        for (int e = lane; e < nv; e += 64) x[(int64_t)R0 * NP + e] = xs[w][e];
        wave_sync_lds();
    }
    // lanes 0, 16, 32, 48 counted their cells
    guarded += __shfl_xor(guarded, 16, 64);
    guarded += __shfl_xor(guarded, 32, 64);
    if (lane == 0 && guarded) atomicAdd(nguard, guarded);
}

// ---------------------------------------------------------------------------
static inline unsigned nbk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

int mlp_param_count() { return kParams; }

// register-resident inference kernels (about 200 VGPRs, two waves per SIMD):
// one resident round of 4-wave blocks, each wave loops over samples/cells
constexpr int kInferBlocks = 512;

void launch_mlp_forward(hipStream_t s, int n, const float* params, const float* X, float* Y) {
    const int g = (int)std::min<int64_t>(nbk(n, 4), kInferBlocks);
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

void launch_learned_correct(hipStream_t s, int n_cells, const int* cp, const int* row_species,
                            const float* geom, const float* params, float guard, double* x,
                            int* nguard) {
    const int64_t chunks = (n_cells + kChunk - 1) / kChunk;
    const int g = (int)std::min<int64_t>(nbk(chunks, 4), kInferBlocks);
    k_learned_correct<<<std::max(g, 1), 256, 0, s>>>(n_cells, cp, row_species, geom, params, guard,
                                                     x, nguard);
}

int mlp_packed_bf16_count() { return kPackedBf16; }

void launch_pack_bf16(hipStream_t s, const float* params, unsigned short* out) {
    k_pack_bf16<<<nbk(kPackedBf16, 256), 256, 0, s>>>(params, out);
}

void launch_learned_correct_bf16(hipStream_t s, int n_cells, const int* cp, const int* row_species,
                                 const float* geom, const unsigned short* wpk,
                                 const float* params, float guard, double* x, int* nguard) {
    const int64_t batches = (n_cells + kBatch - 1) / kBatch;
    const int g = (int)std::min<int64_t>(nbk(batches, 4), kInferBlocks);
    k_learned_correct_bf16<<<std::max(g, 1), 256, 0, s>>>(n_cells, cp, row_species, geom, wpk,
                                                          params, guard, x, nguard);
}

void launch_learned_features(hipStream_t s, int n_sel, int cell0, int cell_step, const int* cp,
                             const int* row_species, const float* geom, const int64_t* doff,
                             const double* D, const double* r, const double* xk,
                             const double* xs, double omega, float clip, float* Xf, float* Tf) {
    const int g = (int)std::min<int64_t>(nbk(n_sel, 4), 2048);
    k_learned_pairs<<<std::max(g, 1), 256, 0, s>>>(n_sel, cell0, cell_step, cp, row_species, geom,
                                                   doff, D, r, xk, xs, omega, clip, Xf, Tf);
}

}  // namespace xdg
