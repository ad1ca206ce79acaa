// fca_mlp.hip -- learned initial powers for the EM: a per-bin MLP that
// predicts r = v1 / (v1 + v2) from features of y(n,f), trained and run by the
// kernels below (BF16 MFMA GEMMs with FP32 accumulation, FP32 master weights,
// AdamW). v_j^(0) = (r, 1 - r) * 2 ||y||^2 / M, so r = 1/2 is the plain start
// v_j = ||y||^2 / M. Not part of the paper; the EM entry points see it only
// through the v0 argument of fca_init.
//
// Network: x (IN = 3M - 1 features, zero-padded to KP = 32) -> 3 hidden
// layers of width H (32, 64, 128 or 256, chosen at creation) with GELU -> 1
// logit -> sigmoid.
// Features: log(|y_m|^2 + 1e-20) for each microphone, cos and sin of the
// phase of y_m relative to microphone 1 (m = 2..M), and f / (F - 1).
// Loss: mean binary cross-entropy with soft targets.
//
// Layouts: activations row-major [n][H] (bf16 copies also transposed
// [H][n] for the weight-gradient GEMMs); weights like a linear layer,
// W[out][in] (bf16 copies W and W^T). GEMM: C[m][c] = sum_k A[m][k] B[c][k]
// with both operands K-contiguous.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "fca.h"
#include "fca_internal.h"

namespace {

constexpr int kMaxHidden = 256;
constexpr int kKP = 32;        // padded input width
constexpr int kLayers = 3;     // hidden layers
constexpr int kGradSplits = 16;  // K splits of the weight-gradient GEMMs (K = batch)

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// erf by Abramowitz & Stegun 7.1.26 (|error| <= 1.5e-7, far below the BF16
// rounding the activations get; used by the GELU derivative): erf(a) = 1 - t (a1 + t (a2 + ... a5)) e^-a^2,
// t = 1 / (1 + p a), a = |x|, odd extension.
__device__ __forceinline__ float erf_as(float x) {
    const float a = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, a, 1.0f));
    float q = fmaf(t, 1.061405429f, -1.453152027f);
    q = fmaf(t, q, 1.421413741f);
    q = fmaf(t, q, -0.284496736f);
    q = fmaf(t, q, 0.254829592f);
    const float e = __builtin_amdgcn_exp2f(-a * a * 1.4426950408889634f);
    return copysignf(fmaf(-t * q, e, 1.0f), x);
}
// GELU(x) = x Phi(x) = max(x, 0) - t Phi(-t) with t = |x| (Phi: standard
// normal CDF). The even tail t Phi(-t) is replaced by t P(t), P of degree 6,
// fitted on [0, 4] by least squares with iteratively reweighted residuals,
// and t is clamped to 4 (where t Phi(-t) = 1.3e-4): |error| <= 2.1e-4 on the
// whole line in FP32, far below the BF16 rounding of the activations, and no
// transcendental instruction (under half the VALU work of the erf form).
// The backward uses the derivative of the exact GELU (erf_as).
__device__ __forceinline__ float gelu(float x) {
    const float t = fminf(fabsf(x), 4.0f);
    float p = -0.0006429001805372536f;
    p = fmaf(p, t, 0.009921977296471596f);
    p = fmaf(p, t, -0.057567618787288666f);
    p = fmaf(p, t, 0.13997237384319305f);
    p = fmaf(p, t, -0.042808666825294495f);
    p = fmaf(p, t, -0.3908194899559021f);
    p = fmaf(p, t, 0.5004920959472656f);
    return fmaf(-t, p, fmaxf(x, 0.0f));
}
__device__ __forceinline__ float gelu_grad(float x) {
    return 0.5f * (1.0f + erf_as(x * 0.70710678118654752f)) +
           x * 0.39894228040143268f * __builtin_amdgcn_exp2f(-0.5f * x * x * 1.4426950408889634f);
}

// ------------------------------------------------------------------ features
// Features of one bin (zero-padded to kKP), stored as T (a local FP32 array
// or a BF16 row in LDS); microphone m of the bin at yb[m * sm].
template <typename T>
__device__ __forceinline__ void bin_features(const float2* __restrict__ yb, int64_t sm, int M, float fpos, T* feat) {
    for (int j = 0; j < kKP; ++j) feat[j] = (T)0.0f;
    const float2 y0 = yb[0];
    const float p0 = y0.x * y0.x + y0.y * y0.y;
    for (int m = 0; m < M; ++m) {
        const float2 ym = yb[m * sm];
        const float pm = ym.x * ym.x + ym.y * ym.y;
        feat[m] = (T)logf(pm + 1e-20f);
        if (m > 0) {
            // y_m conj(y_0) / (|y_m| |y_0|), one reciprocal square root
            const float q = pm * p0;
            const float rden = q > 0.0f ? __builtin_amdgcn_rsqf(q) : 0.0f;
            const float cr = ym.x * y0.x + ym.y * y0.y, ci = ym.y * y0.x - ym.x * y0.y;
            feat[M + 2 * (m - 1)] = (T)(cr * rden);
            feat[M + 2 * (m - 1) + 1] = (T)(ci * rden);
        }
    }
    feat[3 * M - 2] = (T)fpos;
}

__global__ void mlp_features_kernel(const float2* __restrict__ y, const float* __restrict__ fpos, int n, int M,
                                    bf16* __restrict__ X, bf16* __restrict__ XT, int ldt) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    float feat[kKP];
    bin_features(y + (int64_t)b * M, 1, M, fpos[b], feat);
    for (int j = 0; j < kKP; ++j) {
        const bf16 h = (bf16)feat[j];
        X[(int64_t)b * kKP + j] = h;
        XT[(int64_t)j * ldt + b] = h;
    }
}

// ------------------------------------------------------------------ GEMM (BF16 MFMA, FP32 accumulate)
// C[m][c] = sum_k A[m][k] B[c][k]; A is rows x K (row pitch lda), B is
// cols x K (row pitch ldb).
// One workgroup = 4 waves = a 64 x 64 tile; each wave 32 x 32 = 2 x 2 MFMA
// 16x16x32 tiles. Operand lanes: lane l supplies row (l % 16) and the 8
// consecutive k starting at 8 (l / 16) of a 16 x 32 block, for A and B alike
// (the products pair the same k); the result tile gives lane l the rows
// 4 (l / 16) + r, r = 0..3, of column l % 16. K must be a multiple of 32.
enum Epi { kEpiFwd = 0, kEpiBwdGelu = 1, kEpiStore = 2 };

struct GemmArgs {
    const bf16* A;
    const bf16* B;
    int rows, cols, K;
    int lda, ldb;       // row pitches of A and B (elements, multiples of 8)
    const float* bias;  // kEpiFwd: [cols]
    const float* pre;   // kEpiBwdGelu: pre-activation [rows][cols] of the layer below
    float* out_f32;     // kEpiFwd: pre-activation; kEpiStore: result [rows][cols]
    bf16* out_bf;       // bf16 [rows][cols]: GELU(pre) (fwd) or dpre (bwd)
    bf16* out_bfT;      // bf16 [cols][ldt]: the same, transposed
    int ldt;
    int kchunk;         // K per split (blockIdx.z; 0 = all of K); kEpiStore writes split z at
                        // out_f32 + z rows cols
};

template <int EPI>
__global__ __launch_bounds__(256) void mlp_gemm_kernel(GemmArgs g) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = blockIdx.y * 64 + (w >> 1) * 32;
    const int c0 = blockIdx.x * 64 + (w & 1) * 32;
    const int li = lane & 15, lk = (lane >> 4) * 8;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero8 = (bf16x8){(bf16)0.f, (bf16)0.f, (bf16)0.f, (bf16)0.f, (bf16)0.f, (bf16)0.f, (bf16)0.f, (bf16)0.f};
    const int kb = g.kchunk > 0 ? blockIdx.z * g.kchunk : 0;
    const int ke = g.kchunk > 0 ? min(g.K, kb + g.kchunk) : g.K;
    if (EPI == kEpiStore && g.kchunk > 0) g.out_f32 += (int64_t)blockIdx.z * g.rows * g.cols;
    for (int k0 = kb; k0 < ke; k0 += 32) {
        bf16x8 av[2], bv[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int r = r0 + 16 * t + li;
            const int c = c0 + 16 * t + li;
            av[t] = (r < g.rows) ? *reinterpret_cast<const bf16x8*>(g.A + (int64_t)r * g.lda + k0 + lk) : zero8;
            bv[t] = (c < g.cols) ? *reinterpret_cast<const bf16x8*>(g.B + (int64_t)c * g.ldb + k0 + lk) : zero8;
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + 16 * a + (lane >> 4) * 4 + q;
                const int c = c0 + 16 * b + li;
                if (r >= g.rows || c >= g.cols) continue;
                const int64_t e = (int64_t)r * g.cols + c;
                float val = acc[a][b][q];
                if (EPI == kEpiFwd) {
                    val += g.bias[c];
                    g.out_f32[e] = val;
                    const bf16 h = (bf16)gelu(val);
                    g.out_bf[e] = h;
                    g.out_bfT[(int64_t)c * g.ldt + r] = h;
                } else if (EPI == kEpiBwdGelu) {
                    const bf16 d = (bf16)(val * gelu_grad(g.pre[e]));
                    g.out_bf[e] = d;
                    g.out_bfT[(int64_t)c * g.ldt + r] = d;
                } else {
                    g.out_f32[e] = val;
                }
            }
}

// ------------------------------------------------------------------ output layer, loss, its backward
// z = GELU(pre3) . w4 + b4, r = sigmoid(z); with targets: loss terms and
// dz = (r - t) / n. One wave per row.
__global__ void mlp_out_kernel(const float* __restrict__ pre3, const float* __restrict__ w4, const float* __restrict__ b4,
                               int n, int hidden, float* __restrict__ r_out, const float* __restrict__ target,
                               float* __restrict__ dz, double* __restrict__ loss_terms) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    float s = 0.0f;
    for (int o = lane; o < hidden; o += 64) s += gelu(pre3[(int64_t)row * hidden + o]) * w4[o];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        const float z = s + b4[0];
        const float r = 1.0f / (1.0f + expf(-z));
        if (r_out) r_out[row] = r;
        if (target) {
            const float t = target[row];
            // -[t log r + (1 - t) log(1 - r)] with log r = -softplus(-z)
            const double sp_neg = (z > 0) ? log1p(exp(-(double)z)) : -(double)z + log1p(exp((double)z));
            const double sp_pos = sp_neg + (double)z;
            loss_terms[row] = t * sp_neg + (1.0 - t) * sp_pos;
            dz[row] = (r - t) / (float)n;
        }
    }
}

// dpre3[b][o] = dz[b] w4[o] GELU'(pre3[b][o]) (bf16, both layouts)
__global__ void mlp_out_back_kernel(const float* __restrict__ pre3, const float* __restrict__ w4,
                                    const float* __restrict__ dz, int n, int hidden, bf16* __restrict__ d3,
                                    bf16* __restrict__ d3T, int ldt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * hidden) return;
    const int b = (int)(i / hidden), o = (int)(i % hidden);
    const bf16 d = (bf16)(dz[b] * w4[o] * gelu_grad(pre3[i]));
    d3[i] = d;
    d3T[(int64_t)o * ldt + b] = d;
}

// grad of w4 and b4: dw4[o] = sum_b dz[b] GELU(pre3[b][o]); db4 = sum_b dz[b].
// Two fixed-order stages: block c sums rows [kOgRows c, kOgRows (c + 1)) into
// part[c][0..H] (entry H: the dz sum), then one block sums the blocks. One
// thread per hidden unit (blockDim = H).
constexpr int kOgRows = 64;
__global__ void mlp_out_grad_part_kernel(const float* __restrict__ pre3, const float* __restrict__ dz, int n,
                                         float* __restrict__ part) {
    const int o = threadIdx.x, hidden = blockDim.x;
    const int b0 = blockIdx.x * kOgRows, b1 = min(n, b0 + kOgRows);
    float s = 0.0f, t = 0.0f;
    for (int b = b0; b < b1; ++b) {
        s += dz[b] * gelu(pre3[(int64_t)b * hidden + o]);
        t += dz[b];
    }
    part[(int64_t)blockIdx.x * (hidden + 1) + o] = s;
    if (o == 0) part[(int64_t)blockIdx.x * (hidden + 1) + hidden] = t;
}

__global__ void mlp_out_grad_sum_kernel(const float* __restrict__ part, int nblk, float* __restrict__ gw4,
                                        float* __restrict__ gb4) {
    const int o = threadIdx.x, hidden = blockDim.x;
    float s = 0.0f, t = 0.0f;
    for (int c = 0; c < nblk; ++c) {
        s += part[(int64_t)c * (hidden + 1) + o];
        if (o == 0) t += part[(int64_t)c * (hidden + 1) + hidden];
    }
    gw4[o] = s;
    if (o == 0) gb4[0] = t;
}

// bias gradients: gb[o] = sum_b d[o][b] from the transposed bf16 layout [H][ldt]; one block per o
__global__ void mlp_bias_grad_kernel(const bf16* __restrict__ dT, int n, int ldt, float* __restrict__ gb) {
    __shared__ float red[256];
    const int o = blockIdx.x;
    float s = 0.0f;
    for (int b = threadIdx.x; b < n; b += 256) s += (float)dT[(int64_t)o * ldt + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) gb[o] = red[0];
}

// ------------------------------------------------------------------ optimiser and weight copies
__global__ void mlp_adamw_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                                 float* __restrict__ m2, int64_t count, float lr, float b1, float b2, float eps,
                                 float wd, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    p[i] -= lr * ((a / c1) / (sqrtf(v / c2) + eps) + wd * p[i]);
}

// bf16 copies of a [rows][cols] fp32 weight: W and W^T
__global__ void mlp_weight_copy_kernel(const float* __restrict__ W, int rows, int cols, bf16* __restrict__ Wb,
                                       bf16* __restrict__ WTb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)rows * cols) return;
    const int r = (int)(i / cols), c = (int)(i % cols);
    const bf16 h = (bf16)W[i];
    Wb[i] = h;
    WTb[(int64_t)c * rows + r] = h;
}

// ------------------------------------------------------------------ fused inference (learned start)
// One workgroup (4 waves) per tile of kTile bins of y[F][N][M] in the order
// f N + n: features -> three hidden layers (BF16 MFMA 16x16x32, FP32
// accumulation) -> output layer -> sigmoid -> v0[j][f][n]. The activations of
// the tile stay in LDS; the weights are read from L2. The waves split the
// layer outputs into NCG column groups of 16 CT columns and 4 / NCG row
// groups of 16 RT rows (InferShape): for H >= 64 each wave owns 16 CT =
// H / 4 columns of all kTile rows, for H = 32 a pair of waves shares the 32
// columns and each owns half the rows. Same arithmetic as the training
// forward (features, bias, GELU, BF16 rounding of the hidden activations,
// FP32 output layer) up to the order of the output-layer sum.
constexpr int kRT = 8;            // row tiles of 16 per tile
constexpr int kTile = 16 * kRT;   // bins per workgroup
constexpr int kXP = kKP + 8;      // LDS row pitch of the features (bf16)

template <int H>
struct InferShape {
    static constexpr int NCG = H >= 64 ? 4 : H / 16;  // column groups (waves side by side)
    static constexpr int CT = H / (16 * NCG);         // column tiles of 16 per wave
    static constexpr int RT = kRT * NCG / 4;          // row tiles of 16 per wave
    static_assert((NCG == 2 || NCG == 4) && H % (16 * NCG) == 0 && NCG * (kRT / RT) == 4, "four waves per tile");
};

template <int H>
struct InferShared {
    static constexpr int kHP = H + 8;  // LDS row pitch of the hidden activations (bf16)
    bf16 X[kTile * kXP];
    bf16 Hs[kTile * kHP];
    float zp[InferShape<H>::NCG][kTile];
    float sv[kTile];
};

// out^T = W A^T for this wave's 16 CT output columns and RT x 16 rows (A
// points at the first of them): acc[ct][rt] is the 16 x 16 block (columns
// c0 + 16 ct.., rows 16 rt..), lane l holding columns c0 + 16 ct + 4 (l / 16)
// + q, q = 0..3, of row 16 rt + l % 16 (the MFMA A operand is W, the B
// operand the activations, both K-contiguous).
template <int K, int LDA, int CT, int RT>
__device__ __forceinline__ void infer_layer(const bf16* __restrict__ A, const bf16* __restrict__ W, int c0, int lane,
                                            f32x4 (&acc)[CT][RT]) {
    const int li = lane & 15, lk = (lane >> 4) * 8;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[ct][rt] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 wv[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
            wv[ct] = *reinterpret_cast<const bf16x8*>(W + (int64_t)(c0 + ct * 16 + li) * K + k0 + lk);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const bf16x8 hv = *reinterpret_cast<const bf16x8*>(A + (rt * 16 + li) * LDA + k0 + lk);
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                acc[ct][rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wv[ct], hv, acc[ct][rt], 0, 0, 0);
        }
    }
}

// H = bf16(GELU(acc + bias)) for this wave's columns and rows (Hs points at
// the first row): four consecutive columns of one row per lane and block
// (one 8-byte LDS write)
template <int CT, int RT, int LDH>
__device__ __forceinline__ void infer_store_hidden(const f32x4 (&acc)[CT][RT], const float* __restrict__ bias,
                                                   bf16* Hs, int c0, int lane) {
    const int li = lane & 15, cq = (lane >> 4) * 4;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const int col = c0 + ct * 16 + cq;
        const float4 b = *reinterpret_cast<const float4*>(bias + col);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
            const f32x4 v = acc[ct][rt];
            const bf16x4 h = (bf16x4){(bf16)gelu(v[0] + b.x), (bf16)gelu(v[1] + b.y), (bf16)gelu(v[2] + b.z),
                                      (bf16)gelu(v[3] + b.w)};
            *reinterpret_cast<bf16x4*>(Hs + (rt * 16 + li) * LDH + col) = h;
        }
    }
}

using InferJob = fca::MlpInferJob;

template <int H>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void mlp_infer_kernel(
    const InferJob* __restrict__ jobs, int njobs, int M, const bf16* __restrict__ W0, const bf16* __restrict__ W1,
    const bf16* __restrict__ W2, const float* __restrict__ bias0, const float* __restrict__ bias1,
    const float* __restrict__ bias2, const float* __restrict__ w4, const float* __restrict__ b4) {
    using Shape = InferShape<H>;
    constexpr int CT = Shape::CT, RT = Shape::RT, NCG = Shape::NCG;
    using Sh = InferShared<H>;
    extern __shared__ __align__(16) unsigned char smem[];
    Sh& sh = *reinterpret_cast<Sh*>(smem);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // the job owning this tile: the last one with tile0 <= blockIdx.x
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile0 <= (int64_t)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const InferJob job = jobs[lo];
    const int F = job.F, N = job.N;
    const int64_t FN = (int64_t)F * N;
    const int64_t r0 = ((int64_t)blockIdx.x - job.tile0) * kTile;
    if (tid < kTile) {
        const int64_t bin = r0 + tid;
        bf16* xr = sh.X + tid * kXP;
        float s = 0.0f;
        if (bin < FN) {
            const int f = (int)(bin / N), n = (int)(bin - (int64_t)f * N);
            const float2* yb = job.y + f * job.y_sf + n * job.y_sn;
            bin_features(yb, job.y_sm, M, F > 1 ? (float)f / (float)(F - 1) : 0.0f, xr);
            float p = 0.0f;
            for (int m = 0; m < M; ++m) {
                const float2 ym = yb[m * job.y_sm];
                p += ym.x * ym.x + ym.y * ym.y;
            }
            s = fmaxf(2.0f * p / (float)M, 1e-30f);
        } else {
            for (int j = 0; j < kKP; ++j) xr[j] = (bf16)0.0f;
        }
        sh.sv[tid] = s;
    }
    __syncthreads();
    const int cg = w % NCG, row0 = (w / NCG) * 16 * RT;  // this wave's column group and first row
    const int c0 = cg * 16 * CT;
    bf16* const hs = sh.Hs + row0 * Sh::kHP;
    f32x4 acc[CT][RT];
    infer_layer<kKP, kXP, CT, RT>(sh.X + row0 * kXP, W0, c0, lane, acc);
    infer_store_hidden<CT, RT, Sh::kHP>(acc, bias0, hs, c0, lane);
    __syncthreads();
    infer_layer<H, Sh::kHP, CT, RT>(hs, W1, c0, lane, acc);
    __syncthreads();  // every wave has read Hs before it is overwritten
    infer_store_hidden<CT, RT, Sh::kHP>(acc, bias1, hs, c0, lane);
    __syncthreads();
    infer_layer<H, Sh::kHP, CT, RT>(hs, W2, c0, lane, acc);
    // output layer: z = sum_c GELU(pre3_c) w4_c, this wave's columns per row
    const int li = lane & 15, cq = (lane >> 4) * 4;
    float part[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) part[rt] = 0.0f;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const int col = c0 + ct * 16 + cq;
        const float4 b = *reinterpret_cast<const float4*>(bias2 + col);
        const float4 wc = *reinterpret_cast<const float4*>(w4 + col);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const f32x4 v = acc[ct][rt];
            float x = part[rt];
            x = fmaf(gelu(v[0] + b.x), wc.x, x);
            x = fmaf(gelu(v[1] + b.y), wc.y, x);
            x = fmaf(gelu(v[2] + b.z), wc.z, x);
            x = fmaf(gelu(v[3] + b.w), wc.w, x);
            part[rt] = x;
        }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        float x = part[rt];
        x += __shfl_xor(x, 16, 64);
        x += __shfl_xor(x, 32, 64);
        if (lane < 16) sh.zp[cg][row0 + rt * 16 + li] = x;
    }
    __syncthreads();
    if (tid < kTile) {
        const int64_t bin = r0 + tid;
        if (bin < FN) {
            float zs;  // the column groups' partial sums, in a fixed order
            if constexpr (NCG == 4) zs = (sh.zp[0][tid] + sh.zp[1][tid]) + (sh.zp[2][tid] + sh.zp[3][tid]);
            else zs = sh.zp[0][tid] + sh.zp[1][tid];
            const float z = zs + b4[0];
            const float r = 1.0f / (1.0f + expf(-z));
            const float ri = fminf(fmaxf(r, 1e-6f), 1.0f - 1e-6f);
            const float s = sh.sv[tid];
            const int f = (int)(bin / N), n = (int)(bin - (int64_t)f * N);
            const int64_t o = f * job.o_sf + n;
            job.out[o] = ri * s;
            job.out[job.o_sj + o] = (1.0f - ri) * s;
            if (job.out2) {
                job.out2[o] = ri * s;
                job.out2[job.o_sj + o] = (1.0f - ri) * s;
            }
        }
    }
}

}  // namespace

// ------------------------------------------------------------------ host side
struct fca_mlp {
    int M = 0, in_dim = 0, hidden = 0, max_batch = 0, ldt = 0;
    hipStream_t stream = nullptr;
    int64_t nparam = 0;
    // fp32 master parameters, gradients, Adam moments (one allocation each, flat)
    float *p = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
    int64_t off_W[kLayers + 1] = {}, off_b[kLayers + 1] = {};
    bf16 *Wb[kLayers] = {}, *WTb[kLayers] = {};
    // activations
    bf16 *X = nullptr, *XT = nullptr;
    float* pre[kLayers] = {};
    bf16 *H[kLayers] = {}, *HT[kLayers] = {};
    bf16 *D = nullptr, *DT = nullptr, *D2 = nullptr, *D2T = nullptr;
    float *dz = nullptr, *r = nullptr;
    float* ogpart = nullptr;  // [max_batch / 64 + 1][H + 1] partial sums of the output-layer gradient
    float* gpart = nullptr;   // [kGradSplits][H][H] split-K partial weight gradients
    double* loss_terms = nullptr;
    // fused-inference job tables (grown on demand): pinned staging, device copy
    InferJob* jobs_host = nullptr;
    InferJob* jobs_dev = nullptr;
    int jobs_cap = 0;
    hipEvent_t jobs_ev = nullptr;       // the last upload from jobs_host
    hipEvent_t jobs_done_ev = nullptr;  // the last launch that reads jobs_dev
    int64_t step = 0;
    std::string err;
};

namespace {

thread_local std::string g_mlp_error;

template <typename P>
bool mlp_alloc(P** p, size_t bytes) {
    if (hipMalloc(reinterpret_cast<void**>(p), bytes ? bytes : 16) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return false;
    }
    return true;
}

void mlp_free(fca_mlp* m) {
    void* ptrs[] = {m->p, m->g, m->m1, m->m2, m->X, m->XT, m->D, m->DT, m->D2, m->D2T, m->dz, m->r, m->ogpart,
                    m->loss_terms, m->jobs_dev, m->gpart};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (m->jobs_host) (void)hipHostFree(m->jobs_host);
    if (m->jobs_ev) (void)hipEventDestroy(m->jobs_ev);
    if (m->jobs_done_ev) (void)hipEventDestroy(m->jobs_done_ev);
    for (int l = 0; l < kLayers; ++l) {
        if (m->Wb[l]) (void)hipFree(m->Wb[l]);
        if (m->WTb[l]) (void)hipFree(m->WTb[l]);
        if (m->pre[l]) (void)hipFree(m->pre[l]);
        if (m->H[l]) (void)hipFree(m->H[l]);
        if (m->HT[l]) (void)hipFree(m->HT[l]);
    }
}

int layer_in(const fca_mlp* m, int l) { return l == 0 ? kKP : m->hidden; }

hipError_t refresh_weights(fca_mlp* m) {
    // an inference on another stream may still read the BF16 weights
    if (m->jobs_done_ev) {
        hipError_t e = hipStreamWaitEvent(m->stream, m->jobs_done_ev, 0);
        if (e != hipSuccess) return e;
    }
    for (int l = 0; l < kLayers; ++l) {
        const int64_t cnt = (int64_t)m->hidden * layer_in(m, l);
        mlp_weight_copy_kernel<<<(unsigned)((cnt + 255) / 256), 256, 0, m->stream>>>(
            m->p + m->off_W[l], m->hidden, layer_in(m, l), m->Wb[l], m->WTb[l]);
    }
    return hipGetLastError();
}

template <int EPI>
hipError_t gemm(hipStream_t s, const GemmArgs& a) {
    const int splits = a.kchunk > 0 ? (a.K + a.kchunk - 1) / a.kchunk : 1;
    const dim3 grid((a.cols + 63) / 64, (a.rows + 63) / 64, splits);
    mlp_gemm_kernel<EPI><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

// out[i] = sum over the splits z of part[z][i], in split order
__global__ void mlp_split_sum_kernel(const float* __restrict__ part, int splits, int64_t count,
                                     float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.0f;
    for (int z = 0; z < splits; ++z) s += part[z * count + i];
    out[i] = s;
}

// forward of n <= max_batch bins (features, three hidden layers)
hipError_t forward(fca_mlp* m, const float2* y, const float* fpos, int n) {
    mlp_features_kernel<<<(n + 255) / 256, 256, 0, m->stream>>>(y, fpos, n, m->M, m->X, m->XT, m->ldt);
    const bf16* in = m->X;
    for (int l = 0; l < kLayers; ++l) {
        GemmArgs a{};
        a.A = in;
        a.B = m->Wb[l];
        a.rows = n;
        a.cols = m->hidden;
        a.K = layer_in(m, l);
        a.lda = layer_in(m, l);
        a.ldb = layer_in(m, l);
        a.bias = m->p + m->off_b[l];
        a.out_f32 = m->pre[l];
        a.out_bf = m->H[l];
        a.out_bfT = m->HT[l];
        a.ldt = m->ldt;
        hipError_t e = gemm<kEpiFwd>(m->stream, a);
        if (e != hipSuccess) return e;
        in = m->H[l];
    }
    return hipSuccess;
}

template <int H>
hipError_t launch_infer(const fca_mlp* m, const InferJob* jobs, int njobs, int64_t tiles, hipStream_t s) {
    static_assert(sizeof(InferShared<H>) <= 160 * 1024, "LDS of the fused inference kernel");
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(mlp_infer_kernel<H>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(InferShared<H>));
    if (e != hipSuccess) return e;
    mlp_infer_kernel<H><<<(unsigned)tiles, 256, sizeof(InferShared<H>), s>>>(
        jobs, njobs, m->M, m->Wb[0], m->Wb[1], m->Wb[2], m->p + m->off_b[0], m->p + m->off_b[1], m->p + m->off_b[2],
        m->p + m->off_W[kLayers], m->p + m->off_b[kLayers]);
    return hipGetLastError();
}

#define MLP_HIP(m, call)                                                            \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) {                                                     \
            (m)->err = std::string(#call) + ": " + hipGetErrorString(e_);           \
            return FCA_E_DEVICE;                                                    \
        }                                                                           \
    } while (0)

}  // namespace

extern "C" {

fca_status fca_mlp_create(int32_t M, int32_t hidden, uint64_t seed, int32_t max_batch, void* stream, fca_mlp** out) {
    if (!out) return FCA_E_ARG;
    *out = nullptr;
    if (M < 2 || M > fca::kMaxM || max_batch < 64 || max_batch % 64 != 0) {
        g_mlp_error = "fca_mlp_create: need 2 <= M <= 8 and max_batch a positive multiple of 64";
        return FCA_E_ARG;
    }
    if (hidden != 32 && hidden != 64 && hidden != 128 && hidden != kMaxHidden) {
        g_mlp_error = "fca_mlp_create: hidden width must be 32, 64, 128 or 256";
        return FCA_E_ARG;
    }
    fca_mlp* m = new (std::nothrow) fca_mlp();
    if (!m) return FCA_E_NOMEM;
    m->M = M;
    m->hidden = hidden;
    m->in_dim = 3 * M - 1;
    m->max_batch = max_batch;
    m->ldt = max_batch;
    m->stream = static_cast<hipStream_t>(stream);
    int64_t o = 0;
    for (int l = 0; l < kLayers; ++l) {
        m->off_W[l] = o;
        o += (int64_t)hidden * layer_in(m, l);
        m->off_b[l] = o;
        o += hidden;
    }
    m->off_W[kLayers] = o;
    o += hidden;
    m->off_b[kLayers] = o;
    o += 1;
    m->nparam = o;
    bool ok = mlp_alloc(&m->p, o * 4) && mlp_alloc(&m->g, o * 4) && mlp_alloc(&m->m1, o * 4) &&
              mlp_alloc(&m->m2, o * 4);
    for (int l = 0; l < kLayers && ok; ++l)
        ok = mlp_alloc(&m->Wb[l], (size_t)hidden * layer_in(m, l) * 2) &&
             mlp_alloc(&m->WTb[l], (size_t)hidden * layer_in(m, l) * 2) &&
             mlp_alloc(&m->pre[l], (size_t)max_batch * hidden * 4) &&
             mlp_alloc(&m->H[l], (size_t)max_batch * hidden * 2) && mlp_alloc(&m->HT[l], (size_t)max_batch * hidden * 2);
    ok = ok && mlp_alloc(&m->X, (size_t)max_batch * kKP * 2) && mlp_alloc(&m->XT, (size_t)max_batch * kKP * 2) &&
         mlp_alloc(&m->D, (size_t)max_batch * hidden * 2) && mlp_alloc(&m->DT, (size_t)max_batch * hidden * 2) &&
         mlp_alloc(&m->D2, (size_t)max_batch * hidden * 2) && mlp_alloc(&m->D2T, (size_t)max_batch * hidden * 2) &&
         mlp_alloc(&m->dz, (size_t)max_batch * 4) && mlp_alloc(&m->r, (size_t)max_batch * 4) &&
         mlp_alloc(&m->ogpart, (size_t)(max_batch / kOgRows + 1) * (hidden + 1) * 4) &&
         mlp_alloc(&m->gpart, (size_t)kGradSplits * hidden * std::max(hidden, kKP) * 4) &&
         mlp_alloc(&m->loss_terms, (size_t)max_batch * 8);
    if (!ok) {
        mlp_free(m);
        delete m;
        g_mlp_error = "fca_mlp_create: device allocation failed";
        return FCA_E_NOMEM;
    }
    // He-style initialisation (deterministic in the seed); padded inputs and
    // biases start at zero.
    std::vector<float> h(o, 0.0f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<float> nd(0.0f, 1.0f);
    for (int l = 0; l < kLayers; ++l) {
        const int fan_in = l == 0 ? m->in_dim : hidden;
        const float sd = std::sqrt(2.0f / fan_in);
        for (int r = 0; r < hidden; ++r)
            for (int c = 0; c < layer_in(m, l); ++c)
                h[m->off_W[l] + (int64_t)r * layer_in(m, l) + c] = (c < fan_in) ? sd * nd(rng) : 0.0f;
    }
    for (int c = 0; c < hidden; ++c) h[m->off_W[kLayers] + c] = std::sqrt(1.0f / hidden) * nd(rng);
    if (hipMemcpy(m->p, h.data(), o * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(m->m1, 0, o * 4) != hipSuccess || hipMemset(m->m2, 0, o * 4) != hipSuccess ||
        hipMemset(m->g, 0, o * 4) != hipSuccess || refresh_weights(m) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess) {
        (void)hipGetLastError();
        mlp_free(m);
        delete m;
        g_mlp_error = "fca_mlp_create: device initialisation failed";
        return FCA_E_DEVICE;
    }
    *out = m;
    return FCA_OK;
}

void fca_mlp_destroy(fca_mlp* m) {
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    // an inference enqueued on another stream (fca_set_learned_starts) may
    // still read the weights and the job table
    if (m->jobs_done_ev) (void)hipEventSynchronize(m->jobs_done_ev);
    mlp_free(m);
    delete m;
}

int64_t fca_mlp_num_params(const fca_mlp* m) { return m ? m->nparam : 0; }

const char* fca_mlp_last_error(const fca_mlp* m) { return m ? m->err.c_str() : g_mlp_error.c_str(); }

fca_status fca_mlp_get_params(fca_mlp* m, float* params) {
    if (!m || !params) return FCA_E_ARG;
    MLP_HIP(m, hipMemcpyAsync(params, m->p, m->nparam * 4, hipMemcpyDeviceToHost, m->stream));
    MLP_HIP(m, hipStreamSynchronize(m->stream));
    return FCA_OK;
}

fca_status fca_mlp_set_params(fca_mlp* m, const float* params) {
    if (!m || !params) return FCA_E_ARG;
    MLP_HIP(m, hipMemcpyAsync(m->p, params, m->nparam * 4, hipMemcpyHostToDevice, m->stream));
    MLP_HIP(m, refresh_weights(m));
    MLP_HIP(m, hipStreamSynchronize(m->stream));
    return FCA_OK;
}

fca_status fca_mlp_forward(fca_mlp* m, const float* y, const float* fpos, int32_t n, float* r_out) {
    if (!m || !y || !fpos || !r_out || n < 1 || n > m->max_batch) {
        if (m) m->err = "fca_mlp_forward: bad arguments";
        return FCA_E_ARG;
    }
    MLP_HIP(m, forward(m, reinterpret_cast<const float2*>(y), fpos, n));
    mlp_out_kernel<<<(n + 3) / 4, 256, 0, m->stream>>>(m->pre[kLayers - 1], m->p + m->off_W[kLayers],
                                                      m->p + m->off_b[kLayers], n, m->hidden, r_out, nullptr, nullptr,
                                                      nullptr);
    MLP_HIP(m, hipGetLastError());
    MLP_HIP(m, hipStreamSynchronize(m->stream));
    return FCA_OK;
}

fca_status fca_mlp_backward(fca_mlp* m, const float* y, const float* fpos, const float* target, int32_t n,
                            double* loss, float* grads_out) {
    if (!m || !y || !fpos || !target || n < 64 || n > m->max_batch || n % 64 != 0) {
        if (m) m->err = "fca_mlp_backward: need 64 <= n <= max_batch, n a multiple of 64";
        return FCA_E_ARG;
    }
    const hipStream_t s = m->stream;
    MLP_HIP(m, forward(m, reinterpret_cast<const float2*>(y), fpos, n));
    const float* w4 = m->p + m->off_W[kLayers];
    const int hid = m->hidden;
    mlp_out_kernel<<<(n + 3) / 4, 256, 0, s>>>(m->pre[kLayers - 1], w4, m->p + m->off_b[kLayers], n, hid, m->r, target,
                                               m->dz, m->loss_terms);
    const int ogb = (n + kOgRows - 1) / kOgRows;
    mlp_out_grad_part_kernel<<<ogb, hid, 0, s>>>(m->pre[kLayers - 1], m->dz, n, m->ogpart);
    mlp_out_grad_sum_kernel<<<1, hid, 0, s>>>(m->ogpart, ogb, m->g + m->off_W[kLayers], m->g + m->off_b[kLayers]);
    mlp_out_back_kernel<<<(unsigned)(((int64_t)n * hid + 255) / 256), 256, 0, s>>>(m->pre[kLayers - 1], w4, m->dz, n,
                                                                                  hid, m->D, m->DT, m->ldt);
    MLP_HIP(m, hipGetLastError());
    bf16 *dcur = m->D, *dcurT = m->DT, *dnext = m->D2, *dnextT = m->D2T;
    for (int l = kLayers - 1; l >= 0; --l) {
        // weight gradient: gW[o][k] = sum_b d[b][o] in[b][k]  (A = d^T, B = in^T, K = n)
        GemmArgs gw{};
        gw.A = dcurT;
        gw.B = l > 0 ? m->HT[l - 1] : m->XT;
        gw.rows = hid;
        gw.cols = layer_in(m, l);
        gw.K = n;
        gw.lda = m->ldt;
        gw.ldb = m->ldt;
        // K = n is long and the output small: the K range is split over
        // kGradSplits workgroup layers, summed afterwards in split order
        gw.kchunk = ((n / kGradSplits + 31) / 32) * 32;
        gw.out_f32 = m->gpart;
        MLP_HIP(m, gemm<kEpiStore>(s, gw));
        {
            const int splits = (n + gw.kchunk - 1) / gw.kchunk;
            const int64_t cnt = (int64_t)gw.rows * gw.cols;
            mlp_split_sum_kernel<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(m->gpart, splits, cnt,
                                                                               m->g + m->off_W[l]);
            MLP_HIP(m, hipGetLastError());
        }
        mlp_bias_grad_kernel<<<hid, 256, 0, s>>>(dcurT, n, m->ldt, m->g + m->off_b[l]);
        MLP_HIP(m, hipGetLastError());
        if (l > 0) {
            // d_prev[b][i] = (sum_o d[b][o] W[o][i]) GELU'(pre_prev[b][i])  (B = W^T)
            GemmArgs gd{};
            gd.A = dcur;
            gd.B = m->WTb[l];
            gd.rows = n;
            gd.cols = layer_in(m, l);
            gd.K = hid;
            gd.lda = hid;
            gd.ldb = hid;
            gd.pre = m->pre[l - 1];
            gd.out_bf = dnext;
            gd.out_bfT = dnextT;
            gd.ldt = m->ldt;
            MLP_HIP(m, gemm<kEpiBwdGelu>(s, gd));
            std::swap(dcur, dnext);
            std::swap(dcurT, dnextT);
        }
    }
    if (loss) {
        std::vector<double> lt(n);
        MLP_HIP(m, hipMemcpyAsync(lt.data(), m->loss_terms, (size_t)n * 8, hipMemcpyDeviceToHost, s));
        MLP_HIP(m, hipStreamSynchronize(s));
        double t = 0.0;
        for (int i = 0; i < n; ++i) t += lt[i];
        *loss = t / n;
    }
    if (grads_out) MLP_HIP(m, hipMemcpyAsync(grads_out, m->g, m->nparam * 4, hipMemcpyDeviceToHost, s));
    MLP_HIP(m, hipStreamSynchronize(s));
    return FCA_OK;
}

fca_status fca_mlp_adamw(fca_mlp* m, float lr, float beta1, float beta2, float eps, float weight_decay) {
    if (!m) return FCA_E_ARG;
    m->step += 1;
    const float c1 = 1.0f - std::pow(beta1, (float)m->step), c2 = 1.0f - std::pow(beta2, (float)m->step);
    mlp_adamw_kernel<<<(unsigned)((m->nparam + 255) / 256), 256, 0, m->stream>>>(m->p, m->g, m->m1, m->m2, m->nparam, lr,
                                                                                  beta1, beta2, eps, weight_decay, c1, c2);
    MLP_HIP(m, hipGetLastError());
    MLP_HIP(m, refresh_weights(m));
    MLP_HIP(m, hipStreamSynchronize(m->stream));
    return FCA_OK;
}

fca_status fca_mlp_init_powers_batch(fca_mlp* m, int32_t count, const float* const* ys, int32_t F,
                                     const int32_t* Ns, float* const* v0s) {
    if (!m) return FCA_E_ARG;
    if (count < 1 || !ys || !Ns || !v0s || F < 1) {
        m->err = "fca_mlp_init_powers_batch: need count >= 1, F >= 1 and the three arrays";
        return FCA_E_ARG;
    }
    std::vector<fca::MlpInferJob> jobs(count);
    for (int i = 0; i < count; ++i) {
        if (!ys[i] || !v0s[i] || Ns[i] < 1) {
            m->err = "fca_mlp_init_powers_batch: mixture " + std::to_string(i) + " has a null buffer or N < 1";
            return FCA_E_ARG;
        }
        const int64_t N = Ns[i];
        jobs[i] = fca::MlpInferJob{reinterpret_cast<const float2*>(ys[i]), v0s[i], nullptr, N * m->M, m->M, 1,
                                   (int64_t)F * N, N, 0, F, Ns[i]};
    }
    const char* err = nullptr;
    const hipError_t e = fca::mlp_infer_jobs(m, jobs.data(), count, m->stream, &err);
    if (err) {
        m->err = err;
        return e == hipErrorOutOfMemory ? FCA_E_NOMEM : FCA_E_ARG;
    }
    MLP_HIP(m, e);
    return FCA_OK;
}

fca_status fca_mlp_init_powers(fca_mlp* m, const float* y, int32_t F, int32_t N, float* v0_out) {
    if (!m || !y || !v0_out || F < 1 || N < 1) return FCA_E_ARG;
    return fca_mlp_init_powers_batch(m, 1, &y, F, &N, &v0_out);
}

}  // extern "C"

namespace fca {

int mlp_microphones(const fca_mlp* m) { return m ? m->M : 0; }

hipError_t mlp_infer_jobs(fca_mlp* m, MlpInferJob* jobs, int count, hipStream_t s, const char** err) {
    *err = nullptr;
    int64_t tiles = 0;
    for (int i = 0; i < count; ++i) {
        jobs[i].tile0 = tiles;
        tiles += ((int64_t)jobs[i].F * jobs[i].N + kTile - 1) / kTile;
    }
    if (tiles > INT32_MAX) {
        *err = "learned-start inference: too many bins in one call";
        return hipErrorInvalidValue;
    }
    hipError_t e;
    if (!m->jobs_ev && (e = hipEventCreateWithFlags(&m->jobs_ev, hipEventDisableTiming)) != hipSuccess) return e;
    if (!m->jobs_done_ev && (e = hipEventCreateWithFlags(&m->jobs_done_ev, hipEventDisableTiming)) != hipSuccess)
        return e;
    if (count > m->jobs_cap) {
        // nothing may still read the old tables
        if ((e = hipEventSynchronize(m->jobs_done_ev)) != hipSuccess) return e;
        if (m->jobs_host) (void)hipHostFree(m->jobs_host);
        if (m->jobs_dev) (void)hipFree(m->jobs_dev);
        m->jobs_host = nullptr;
        m->jobs_dev = nullptr;
        m->jobs_cap = 0;
        const int cap = std::max(count, 64);
        if (hipHostMalloc(reinterpret_cast<void**>(&m->jobs_host), (size_t)cap * sizeof(MlpInferJob),
                          hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            m->jobs_host = nullptr;
            *err = "learned-start inference: pinned allocation failed";
            return hipErrorOutOfMemory;
        }
        if (!mlp_alloc(&m->jobs_dev, (size_t)cap * sizeof(MlpInferJob))) {
            *err = "learned-start inference: device allocation failed";
            return hipErrorOutOfMemory;
        }
        m->jobs_cap = cap;
    }
    if ((e = hipEventSynchronize(m->jobs_ev)) != hipSuccess) return e;  // the staging buffer is free
    memcpy(m->jobs_host, jobs, (size_t)count * sizeof(MlpInferJob));
    // the weights come from the network's stream; the table from the last
    // launch that read it, possibly on another stream
    if (s != m->stream) {
        if ((e = hipStreamSynchronize(m->stream)) != hipSuccess) return e;
    }
    if ((e = hipStreamWaitEvent(s, m->jobs_done_ev, 0)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(m->jobs_dev, m->jobs_host, (size_t)count * sizeof(MlpInferJob), hipMemcpyHostToDevice,
                            s)) != hipSuccess)
        return e;
    if ((e = hipEventRecord(m->jobs_ev, s)) != hipSuccess) return e;
    switch (m->hidden) {
        case 32: e = launch_infer<32>(m, m->jobs_dev, count, tiles, s); break;
        case 64: e = launch_infer<64>(m, m->jobs_dev, count, tiles, s); break;
        case 128: e = launch_infer<128>(m, m->jobs_dev, count, tiles, s); break;
        default: e = launch_infer<kMaxHidden>(m, m->jobs_dev, count, tiles, s); break;
    }
    if (e != hipSuccess) return e;
    return hipEventRecord(m->jobs_done_ev, s);
}

}  // namespace fca
