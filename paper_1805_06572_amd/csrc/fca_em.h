// fca_em.h -- the FastFCA EM-iteration kernels of libfca, templated on the
// workgroup size NT; fca_em_nt256.hip and fca_em_nt128.hip instantiate them.
//
// em_kernel: one workgroup owns one (mixture, frequency) EM problem for all
// iterations of a call. Its frames stay in registers, so y(n,f) and v_j(n,f)
// cross HBM once per call, not once per iteration (em_stream_kernel re-reads
// them each pass when there are too many frames). Each iteration
// (Algorithm 1, steps 3-9):
//   per bin (one thread per frame, up to FPT frames per thread):
//     y~ = P^H y                                   eq. (tildey)
//     d_i = v1 lam_i + v2, mu~ and the posterior   eqs. (MMSEtilde), (updatePhitildeeff)
//     v_j' from the diagonal traces                eq. (updateveff)
//     log-likelihood term of theta^(l)             eq. (like) in the eigenbasis
//     running sums of Phi~_j / v_j'                eq. (updateStildeeff)
//   per frequency: FP64 reduction of the sums in a fixed order, then the
//   FP64 generalized eigendecomposition of (S~1, S~2) and P <- P Q,
//   Lambda <- Sigma (eqs. GEVDeff5, updatePeff, updateLambdaeff).
// The log-likelihood of a bin uses v1 R1 + v2 R2 = P^-H diag(d) P^-1 and
// |det P|^2 = 1 / det R2:
//   log p(y) = -M log(pi) + log|det P|^2 - sum_i log d_i - sum_i |y~_i|^2 / d_i.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fca_device.h"
#include "fca_internal.h"

namespace fca {

// ============================================================== EM iteration pieces
// LDS state of one (mixture, frequency) problem inside an EM workgroup.
template <int M, typename T, int NT_ = kEmThreads> struct EmShared {
    static constexpr int NTH = NT_;  // threads of the workgroup
    using Tb = T;
    using T2 = typename Vec2<T>::type;
    static constexpr int MM = M * M;
    static constexpr int NV = 2 * MM;             // reals accumulated per thread
    static constexpr int CH = NV < 32 ? NV : 32;  // values per reduction chunk
    static constexpr int NCH = (NV + CH - 1) / CH;
    static constexpr int G = NT_ / 32;            // row groups of the second reduction stage
    static constexpr int NW = NT_ / 64;
    double2 P[MM];      // basis P^(l) (FP64)
    double2 Pn[MM];     // basis after the update
    T2 Pt[MM];          // P^(l) in the bulk precision
    T lamT[M];
    double lam[M], lamN[M];
    double logdet;      // log |det P^(l)|^2
    int flag;           // FCA flag bits of the problem
    int bad;            // a non-finite or non-positive power appeared in this pass
    double2 S[2][MM];   // S~1, S~2 (full Hermitian, FP64)
    T red[NT_ * (CH + 1)];
    double wh[NW][64];  // per-wave partial column sums
    double wp[NW][NV];  // per-wave sums
    double llp[NT_];    // per-thread log-likelihood terms of the pass
    double piv[2][M];   // Cholesky pivots of the last two updates (by parity)
    int pend[2];        // that update succeeded; its log-determinant is pending
    GevdScratch ws;
};

template <int M, typename Sh>
__device__ __forceinline__ void em_load_state(Sh& sh, const double2* __restrict__ Pg,
                                              const double* __restrict__ lamg,
                                              const double* __restrict__ logdetg,
                                              const int* __restrict__ flagsg, int pid, int tid) {
    if (tid < M * M) sh.P[tid] = Pg[(int64_t)pid * kMaxM * kMaxM + tid];
    if (tid < M) sh.lam[tid] = lamg[(int64_t)pid * kMaxM + tid];
    if (tid == 0) {
        sh.logdet = logdetg[pid];
        sh.flag = flagsg[pid];
        sh.bad = 0;
    }
}

template <int M, typename Sh>
__device__ __forceinline__ void em_store_state(const Sh& sh, double2* __restrict__ Pg,
                                               double* __restrict__ lamg, double* __restrict__ logdetg,
                                               int* __restrict__ flagsg, int pid, int tid) {
    if (tid < M * M) Pg[(int64_t)pid * kMaxM * kMaxM + tid] = sh.P[tid];
    if (tid < M) lamg[(int64_t)pid * kMaxM + tid] = sh.lam[tid];
    if (tid == 0) {
        logdetg[pid] = sh.logdet;
        flagsg[pid] = sh.flag;
    }
}

// P^(l) and Lambda^(l) in the bulk precision; a __syncthreads must follow.
template <int M, typename Sh>
__device__ __forceinline__ void em_prepare(Sh& sh, int tid) {
    using T = typename Sh::Tb;
    if (tid < M * M) {
        const double2 p = sh.P[tid];
        sh.Pt[tid] = make_vec2<T>((T)p.x, (T)p.y);
    }
    if (tid < M) sh.lamT[tid] = (T)sh.lam[tid];
}

// One time-frequency bin of Algorithm 1, steps 3-7, in the eigenbasis:
//   y~ = P^H y                                      eq. (tildey)
//   d_i = v1 lam_i + v2                             (v1 Lambda + v2 I)
//   mu~1_i = v1 lam_i y~_i / d_i, mu~2_i = v2 y~_i / d_i          eq. (MMSEtilde)
//   c_i = v1 v2 lam_i / d_i  (diagonal of Phi~_j - mu~_j mu~_j^H)  eq. (updatePhitildeeff)
//   v1' = tr(Lambda^-1 Phi~1)/M, v2' = tr(Phi~2)/M                  eq. (updateveff)
//       = (v1/M) sum_i t1_i,  v2' = (v2/M) sum_i t2_i  with
//         t1_i = r_i (v1 lam_i e_i r_i + v2), t2_i = r_i (v2 e_i r_i + v1 lam_i),
//         e_i = |y~_i|^2, r_i = 1 / d_i
//   Phi~_j / v_j'  (eq. updateStildeeff), summed over the frames
//   llacc += -sum_i log d_i - sum_i |y~_i|^2 / d_i   (log-likelihood of theta^(l))
// `ok` masks padding frames (no contribution, powers unchanged).
// em_bin_front: everything up to the new powers; leaves y~ (ytr, yti), e_i,
// r_i, t1_i, t2_i (unless KeepT is false: then only their sums are formed,
// one fused multiply-add per term) and the new powers nv1, nv2 (also in
// nv1o, nv2o unless padding).
template <int M, typename T, bool KeepT = true>
__device__ __forceinline__ void em_bin_front(const T (&yr)[M], const T (&yi)[M], T a1, T a2, const T (&lm)[M],
                                             const typename Vec2<T>::type* Pt, bool ok, double& llacc, T& nv1o,
                                             T& nv2o, bool& bad, T (&ytr)[M], T (&yti)[M], T (&e)[M], T (&r)[M],
                                             T (&t1)[M], T (&t2)[M], T& nv1, T& nv2) {
    using T2 = typename Vec2<T>::type;
    using MT = Math<T>;
#pragma unroll
    for (int i = 0; i < M; ++i) {
        // from M = 5 on, P (2 M^2 values) is read column by column from LDS
        // rather than all hoisted into registers
        if constexpr (M > 4) __builtin_amdgcn_sched_barrier(0);
        T sr = T(0), si = T(0);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const T2 pmi = Pt[m * M + i];
            sr = fma(pmi.x, yr[m], fma(pmi.y, yi[m], sr));
            si = fma(pmi.x, yi[m], fma(-pmi.y, yr[m], si));
        }
        ytr[i] = sr;
        yti[i] = si;
        e[i] = fma(sr, sr, si * si);
    }
    T d[M];
    T quad = T(0);
#pragma unroll
    for (int i = 0; i < M; ++i) {
        d[i] = fma(a1, lm[i], a2);
        r[i] = MT::rcp(d[i]);
        quad = fma(e[i], r[i], quad);
    }
    T logd = T(0);
    if constexpr (sizeof(T) == 4) {
        // sum of the hardware log2 of each d_i (normal positive floats), one
        // scaling by ln 2
        float l2 = 0.0f;
#pragma unroll
        for (int i = 0; i < M; ++i) l2 += __builtin_amdgcn_logf(d[i]);
        logd = l2 * 0.69314718055994531f;
    } else {
#pragma unroll
        for (int i = 0; i < M; i += 2) {
            const T pd = (i + 1 < M) ? d[i] * d[i + 1] : d[i];
            logd += MT::log(pd);
        }
    }
    T s1 = T(0), s2 = T(0);
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const T er = e[i] * r[i];
        const T a1l = a1 * lm[i];
        if constexpr (KeepT) {
            t1[i] = r[i] * fma(a1l, er, a2);
            t2[i] = r[i] * fma(a2, er, a1l);
            s1 += t1[i];
            s2 += t2[i];
        } else {
            s1 = fma(r[i], fma(a1l, er, a2), s1);
            s2 = fma(r[i], fma(a2, er, a1l), s2);
        }
    }
    nv1 = a1 * s1 * (T(1) / T(M));
    nv2 = a2 * s2 * (T(1) / T(M));
    if (ok) {
        llacc += (double)(-logd - quad);
        bad = bad || !(nv1 > T(0)) || !(nv2 > T(0)) || !isfinite(nv1) || !isfinite(nv2);
    }
    if constexpr (sizeof(T) == 4) {
        // float bulk: keep the powers normal (tested for failure first, so a
        // NaN is still caught)
        nv1 = fmaxf(nv1, kPowerFloorF32);
        nv2 = fmaxf(nv2, kPowerFloorF32);
    }
    if (ok) {
        nv1o = nv1;
        nv2o = nv2;
    }
}

// The bin with the sums of Phi~_j / v_j' kept per thread. With
// z_i = r_i y~_i, k_j = v_j / v_j', alpha = v1 k_1, beta = v2 k_2:
//   (Phi~1 / v1')_ik = lam_i lam_k alpha z_i conj(z_k)    (i != k)
//   (Phi~1 / v1')_ii = lam_i k_1 t1_i
//   (Phi~2 / v2')_ik = beta z_i conj(z_k),   (Phi~2 / v2')_ii = k_2 t2_i
// so the per-thread sums leave out the lam factors of source 1 (constant
// per frequency; applied to the workgroup totals, wg_reduce_sums). Layout:
// the diagonal of source j at acc[j M^2 + i], the upper-triangle pair (i < k)
// at acc[j M^2 + M + 2 pair_index(M, i, k)] (+1 imaginary).
template <int M, typename T>
__device__ __forceinline__ void em_bin(const T (&yr)[M], const T (&yi)[M], T a1, T a2, const T (&lm)[M],
                                       const typename Vec2<T>::type* Pt, bool ok, T (&acc)[2 * M * M],
                                       double& llacc, T& nv1o, T& nv2o, bool& bad) {
    using MT = Math<T>;
    constexpr int MM = M * M;
    T ytr[M], yti[M], e[M], r[M], t1[M], t2[M], nv1, nv2;
    em_bin_front<M, T>(yr, yi, a1, a2, lm, Pt, ok, llacc, nv1o, nv2o, bad, ytr, yti, e, r, t1, t2, nv1, nv2);
    const T k1 = ok ? a1 * MT::rcp(nv1) : T(0);
    const T k2 = ok ? a2 * MT::rcp(nv2) : T(0);
    const T al = k1 * a1, be = k2 * a2;
    T zr[M], zi[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        zr[i] = r[i] * ytr[i];
        zi[i] = r[i] * yti[i];
        acc[i] = fma(k1, t1[i], acc[i]);
        acc[MM + i] = fma(k2, t2[i], acc[MM + i]);
    }
#pragma unroll
    for (int i = 0; i < M; ++i) {
#pragma unroll
        for (int q = i + 1; q < M; ++q) {
            const int o = M + 2 * pair_index(M, i, q);
            const T pr = fma(zr[i], zr[q], zi[i] * zi[q]);
            const T pi = fma(zi[i], zr[q], -zr[i] * zi[q]);
            acc[o] = fma(al, pr, acc[o]);
            acc[o + 1] = fma(al, pi, acc[o + 1]);
            acc[MM + o] = fma(be, pr, acc[MM + o]);
            acc[MM + o + 1] = fma(be, pi, acc[MM + o + 1]);
        }
    }
}

// ---------------------------------------------------------------- S~ accumulation on MFMA
// For M >= kMfmaMinM in the float bulk mode the sums of u_j u_j^H run on the
// matrix cores: per wave and 64 frames (one per lane) the real 2M x 64 matrix
// W_j = [Re u_j; Im u_j] (rows padded to 16 with zeros) is staged in LDS and
// G_j += W_j W_j^T is 16 MFMA 16x16x4 steps; then
//   Re (sum u u^H)_ik = G_ik + G_(M+i)(M+k),  Im (sum u u^H)_ik = G_(M+i)k - G_i(M+k).
// This removes the 2 M^2 per-thread accumulators (register spills at M = 8)
// and moves 16 M^2 of the 24 M^2 flops per bin off the vector ALUs.
constexpr int kMfmaMinM = 5;
// Staging layout of W_j for one wave: element (row r, frame f) at
// r * kStgRow + (f % 4) * 16 + f / 4, so that the 16 values a lane feeds to the
// 16 MFMA steps (row lane % 16, frames 4 kb + lane / 16, kb = 0..15) are
// contiguous (four 16-byte reads); the row pitch of 68 floats keeps those
// reads free of bank conflicts.
constexpr int kStgRow = 68;
constexpr int kStgSrc = 16 * kStgRow;  // floats per source block of a wave
using f32x4 = float __attribute__((ext_vector_type(4)));

template <int M, typename T>
constexpr bool use_mfma() { return M >= kMfmaMinM && sizeof(T) == 4; }

template <int M, int NT_> struct EmSharedMf {
    static constexpr int NTH = NT_;
    using Tb = float;
    using T2 = float2;
    static constexpr int MM = M * M;
    static constexpr int NV = 2 * M;  // per-thread diagonal terms
    static constexpr int CH = NV;
    static constexpr int G = NT_ / 32;
    static constexpr int NW = NT_ / 64;
    double2 P[MM];
    double2 Pn[MM];
    T2 Pt[MM];
    float lamT[M];
    double lam[M], lamN[M];
    double logdet;
    int flag;
    int bad;
    double2 S[2][MM];
    double fin[NV];
    double red2[G * CH];
    double llp[NT_];
    double piv[2][M];
    int pend[2];
    double Gm[2][256];  // W_j W_j^T summed over the waves (FP64)
    union alignas(16) {  // the staging rows are read back as float4
        float stg[NW][2 * kStgSrc];  // per wave: W_1 then W_2 (layout above)
        struct {
            float red[NT_ * (CH + 1)];
            float blk[NW][2][256];
        } r;
    } u;
    GevdScratch ws;
};

// Zero rows 2M..15 of this lane's staged frame (the padding of W_j to 16 rows);
// needed at every pass since the end-of-pass reduction reuses the area.
template <int M>
__device__ __forceinline__ void mf_zero_pad(float* __restrict__ stg, int lane) {
    const int col = (lane & 3) * 16 + (lane >> 2);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 2 * M; r < 16; ++r) stg[j * kStgSrc + r * kStgRow + col] = 0.0f;
}

// The bin with u_1, u_2 staged as this lane's column of W_1, W_2 and the
// diagonal terms c_i / v_j' summed per thread (cd); then G_j += W_j W_j^T over
// the wave's 64 frames. Must be called by all 64 lanes (wave-uniform control).
template <int M>
__device__ __forceinline__ void em_bin_mf(const float (&yr)[M], const float (&yi)[M], float a1, float a2,
                                          const float (&lm)[M], const float2* Pt, bool ok, double& llacc,
                                          float& nv1o, float& nv2o, bool& bad, float* __restrict__ stg,
                                          float (&cd)[2 * M], f32x4 (&am)[2], int lane) {
    float ytr[M], yti[M], e[M], r[M], t1[M], t2[M], nv1, nv2;
    em_bin_front<M, float, false>(yr, yi, a1, a2, lm, Pt, ok, llacc, nv1o, nv2o, bad, ytr, yti, e, r, t1, t2, nv1, nv2);
    const float w1 = ok ? __builtin_amdgcn_rsqf(nv1) : 0.0f;
    const float w2 = ok ? __builtin_amdgcn_rsqf(nv2) : 0.0f;
    const float iv1 = w1 * w1, iv2 = w2 * w2;
    float* __restrict__ c1 = stg + (lane & 3) * 16 + (lane >> 2);
    float* __restrict__ c2 = c1 + kStgSrc;
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const float g1 = a1 * lm[i] * r[i];
        const float g2 = a2 * r[i];
        const float c = g1 * a2;
        const float s1i = g1 * w1, s2i = g2 * w2;
        c1[i * kStgRow] = s1i * ytr[i];
        c1[(M + i) * kStgRow] = s1i * yti[i];
        c2[i * kStgRow] = s2i * ytr[i];
        c2[(M + i) * kStgRow] = s2i * yti[i];
        cd[i] = fma(c, iv1, cd[i]);
        cd[M + i] = fma(c, iv2, cd[M + i]);
    }
    wave_lds_sync();
    // this lane's operand for step kb is W_j(lane % 16, 4 kb + lane / 16)
    const float4* __restrict__ src = reinterpret_cast<const float4*>(stg + (lane & 15) * kStgRow + (lane >> 4) * 16);
    float4 a[2][4];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) a[j][q] = src[j * (kStgSrc / 4) + q];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            am[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j][q].x, a[j][q].x, am[j], 0, 0, 0);
            am[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j][q].y, a[j][q].y, am[j], 0, 0, 0);
            am[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j][q].z, a[j][q].z, am[j], 0, 0, 0);
            am[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j][q].w, a[j][q].w, am[j], 0, 0, 0);
        }
    }
    wave_lds_sync();
}

// End-of-pass reduction for the MFMA scheme: the per-thread log-likelihood
// terms stored for em_update, the per-thread diagonal terms (two fixed-order stages) and the per-wave Gram
// blocks (summed over the waves in FP64, fixed order) into S~_j = sums / N.
template <int M, int NT_>
__device__ __forceinline__ void wg_reduce_mf(EmSharedMf<M, NT_>& sh, const float (&cd)[2 * M], const f32x4 (&am)[2],
                                             double llacc, int nf, int tid) {
    constexpr int MM = M * M, CH = 2 * M, G = NT_ / 32, NW = NT_ / 64;
    const int lane = tid & 63, w = tid >> 6;
    sh.llp[tid] = llacc;
    __syncthreads();  // every wave is done with its staging rows (shared with red, blk)
#pragma unroll
    for (int c = 0; c < CH; ++c) sh.u.r.red[tid * (CH + 1) + c] = cd[c];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) sh.u.r.blk[w][j][(4 * (lane >> 4) + q) * 16 + (lane & 15)] = am[j][q];
    __syncthreads();
    for (int task = tid; task < CH * G; task += NT_) {
        const int c = task % CH, g = task / CH;
        double s = 0.0;
#pragma unroll 8
        for (int rr = 0; rr < 32; ++rr) s += (double)sh.u.r.red[(g * 32 + rr) * (CH + 1) + c];
        sh.red2[g * CH + c] = s;
    }
    for (int e = tid; e < 512; e += NT_) {
        const int j = e >> 8, ent = e & 255;
        double s = 0.0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) s += (double)sh.u.r.blk[ww][j][ent];
        sh.Gm[j][ent] = s;
    }
    __syncthreads();
    if (tid < CH) {
        double s = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) s += sh.red2[g * CH + tid];
        sh.fin[tid] = s;
    }
    __syncthreads();
    if (tid < 2 * MM) {
        const int j = tid / MM, ent = tid % MM, i = ent / M, q = ent % M;
        const int a = i < q ? i : q, b = i < q ? q : i;  // upper triangle, mirrored below it
        const double* Gj = sh.Gm[j];
        const double invn = 1.0 / (double)nf;
        double re = Gj[a * 16 + b] + Gj[(M + a) * 16 + (M + b)];
        double im = Gj[(M + a) * 16 + b] - Gj[a * 16 + (M + b)];
        if (a == b) {
            re += sh.fin[j * M + a];
            im = 0.0;
        }
        sh.S[j][ent] = make_double2(re * invn, (i <= q ? im : -im) * invn);
    }
    __syncthreads();
}

// After the reduction of a pass (S~_j in sh.S, per-thread log-likelihood
// terms in sh.llp): on wave 0 the FP64 GEVD of (S~1, S~2) and the basis
// update P <- P Q, Lambda <- Sigma (eqs. GEVDeff5, updatePeff,
// updateLambdaeff), which leaves its Cholesky pivots for log|det P|^2; beside
// it on wave 1, log|det P^(it)|^2 (the previous update's pivots) and
// LL(theta^(it)). Returns true when the caller must stop iterating: an
// evaluation-only pass, a problem frozen on entry, or a failure that froze it
// now (it then keeps theta^(it), whose log-likelihood stands for the later
// iterations). The last update's log-determinant stays pending
// (em_settle_logdet).
template <int M, typename Sh>
__device__ __forceinline__ bool em_update(Sh& sh, int it, int iters, int it_base, bool frozen_at_entry, int nf,
                                          double* __restrict__ ll, int64_t ll_stride, int pid, double eps2,
                                          int tid) {
    constexpr int NW = Sh::NW;
    const int ll_count = iters > 0 ? iters : 1;
    const bool last = (iters == 0) || frozen_at_entry;
    double tot = 0.0;
    if (tid < 64) {
        if (!last) {
            int flag = sh.bad ? kFlagNonFinite : 0;
            double dld = 0.0;
            // the eigendecomposition is this workgroup's critical path: give its
            // wave issue priority over co-resident waves streaming frames. It
            // writes the new basis and eigenvalues in place (FP64 and bulk
            // copies) unless it fails.
            using Tb = typename Sh::Tb;
            __builtin_amdgcn_s_setprio(3);
            if (!flag)
                flag = gevd_wave<M, sizeof(Tb) == 4, Tb>(sh.S[0], sh.S[1], sh.P, sh.ws, sh.P, sh.lam, &dld, eps2,
                                                        sh.Pt, sh.lamT, sh.piv[it & 1]);
            __builtin_amdgcn_s_setprio(0);
            if (flag & kFreezeMask) flag |= (it_base + it + 1) << kFlagIterShift;  // the failing iteration of the call
            if (tid == 0) {
                sh.pend[it & 1] = (flag & kFreezeMask) ? 0 : 1;
                sh.flag |= flag;
            }
        }
    } else if (tid < 128) {
        double logdet = sh.logdet;
        if (it > 0 && sh.pend[(it - 1) & 1]) logdet -= log_pivots<M>(sh.piv[(it - 1) & 1]);
        double part = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) part += sh.llp[w * 64 + (tid - 64)];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
        tot = part + (double)nf * (-(double)M * kLogPi + logdet);
        if (tid == 64) {
            sh.logdet = logdet;
            if (last)
                for (int l = it; l < ll_count; ++l) ll[(int64_t)l * ll_stride + pid] = tot;
            else
                ll[(int64_t)it * ll_stride + pid] = tot;
        }
    }
    __syncthreads();
    const bool frozen_now = !last && (sh.flag & kFreezeMask);
    if (frozen_now && tid == 64)
        for (int l = it + 1; l < ll_count; ++l) ll[(int64_t)l * ll_stride + pid] = tot;
    return last || frozen_now;
}

// log|det P|^2 of the last update of a call (pending after em_update), by
// thread 0 after the loop (whose last em_update ended with a barrier).
// last_it: the last iteration that ran an update, or -1.
template <int M, typename Sh>
__device__ __forceinline__ void em_settle_logdet(Sh& sh, int last_it, int tid) {
    if (tid == 0 && last_it >= 0 && sh.pend[last_it & 1]) sh.logdet -= log_pivots<M>(sh.piv[last_it & 1]);
}


// End of one pass over the frames (per-thread accumulators): FP64 reduction
// of the sums over the workgroup (fixed order), S~_j = sums / N, the
// log-likelihood terms stored per thread, then em_update.
template <int M, typename T, int NT_>
__device__ __forceinline__ bool em_finish(EmShared<M, T, NT_>& sh, const T (&acc)[2 * M * M], double llacc,
                                          bool bad, int it, int iters, int it_base, bool frozen_at_entry, int nf,
                                          double* __restrict__ ll, int64_t ll_stride, int pid, double eps2,
                                          int tid) {
    if (bad) sh.bad = 1;
    wg_reduce_sums<M, 2, true>(sh, acc, llacc, nf, tid, sh.lam);
    return em_update<M>(sh, it, iters, it_base, frozen_at_entry, nf, ll, ll_stride, pid, eps2, tid);
}

// Per-pass accumulation of one thread: per-thread sums (em_bin, em_finish)
// or the MFMA scheme (em_bin_mf, wg_reduce_mf), selected by
// use_mfma<M, T>(), with the matching LDS layout EmSh.
template <int M, typename T, int NT>
using EmSh = typename std::conditional<use_mfma<M, T>(), EmSharedMf<M, NT>, EmShared<M, T, NT>>::type;

template <int M, typename T, bool MF> struct PassAcc;

template <int M, typename T> struct PassAcc<M, T, false> {
    T acc[2 * M * M];
    template <typename Sh>
    __device__ __forceinline__ void init(Sh&, int) {
#pragma unroll
        for (int i = 0; i < 2 * M * M; ++i) acc[i] = T(0);
    }
    template <typename Sh>
    __device__ __forceinline__ void bin(Sh& sh, const T (&yr)[M], const T (&yi)[M], T a1, T a2, const T (&lm)[M],
                                        bool ok, double& llacc, T& n1, T& n2, bool& bad, int) {
        em_bin<M, T>(yr, yi, a1, a2, lm, sh.Pt, ok, acc, llacc, n1, n2, bad);
    }
    template <typename Sh>
    __device__ __forceinline__ bool finish(Sh& sh, double llacc, bool bad, int it, int iters, int it_base, bool frozen, int nf,
                                           double* __restrict__ ll, int64_t ll_stride, int pid, double eps2, int tid) {
        return em_finish<M, T>(sh, acc, llacc, bad, it, iters, it_base, frozen, nf, ll, ll_stride, pid, eps2, tid);
    }
};

template <int M> struct PassAcc<M, float, true> {
    float cd[2 * M];
    f32x4 am[2];
    template <typename Sh>
    __device__ __forceinline__ void init(Sh& sh, int tid) {
#pragma unroll
        for (int i = 0; i < 2 * M; ++i) cd[i] = 0.0f;
        am[0] = (f32x4){0.f, 0.f, 0.f, 0.f};
        am[1] = (f32x4){0.f, 0.f, 0.f, 0.f};
        mf_zero_pad<M>(sh.u.stg[tid >> 6], tid & 63);
    }
    template <typename Sh>
    __device__ __forceinline__ void bin(Sh& sh, const float (&yr)[M], const float (&yi)[M], float a1, float a2,
                                        const float (&lm)[M], bool ok, double& llacc, float& n1, float& n2, bool& bad,
                                        int tid) {
        em_bin_mf<M>(yr, yi, a1, a2, lm, sh.Pt, ok, llacc, n1, n2, bad, sh.u.stg[tid >> 6], cd, am, tid & 63);
    }
    template <typename Sh>
    __device__ __forceinline__ bool finish(Sh& sh, double llacc, bool bad, int it, int iters, int it_base, bool frozen, int nf,
                                           double* __restrict__ ll, int64_t ll_stride, int pid, double eps2, int tid) {
        if (bad) sh.bad = 1;
        wg_reduce_mf<M, Sh::NTH>(sh, cd, am, llacc, nf, tid);
        return em_update<M>(sh, it, iters, it_base, frozen, nf, ll, ll_stride, pid, eps2, tid);
    }
};

// ============================================================== EM kernel, frames resident
// One workgroup owns one (mixture, frequency) EM problem for all iterations of
// a call; each thread keeps FPT frames of y and v in registers, so y(n,f) and
// v_j(n,f) cross HBM once per call, not once per iteration.
// Waves per SIMD requested for em_kernel: three workgroups per CU where the
// per-thread frames fit in 168 registers (M <= 4, up to four frames per
// thread), two otherwise (eight frames per thread spill at three). FP64 at
// M = 4 with eight frames keeps the request of three, which the compiler
// cannot meet: it then takes accumulation registers at one workgroup per CU,
// where a request of two makes it spill to scratch instead. FP64 at M = 4 with four
// frames asks for two: 188 bytes of scratch per lane, but two workgroups per
// CU instead of one (513 frequencies in two waves of workgroups instead of
// three; 1.45 -> 1.19 ms per 50-iteration launch at M = 4, N = 1000).
template <int M, typename T, int FPT>
constexpr int em_waves_per_eu() {
    if (M == 4 && sizeof(T) == 8 && FPT == 8) return 3;
    if (M == 4 && sizeof(T) == 8 && FPT == 4) return 2;
    return (M <= 4 && FPT <= 4) ? 3 : 2;
}

template <int M, typename T, int FPT, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(em_waves_per_eu<M, T, FPT>()))) void em_kernel(
    const EmProblem* __restrict__ probs, const typename Vec2<T>::type* __restrict__ y,
    T* __restrict__ v, double2* __restrict__ Pg, double* __restrict__ lamg,
    double* __restrict__ logdetg, int* __restrict__ flagsg, double* __restrict__ ll,
    int64_t ll_stride, int iters, int it_base, double eps2) {
    using T2 = typename Vec2<T>::type;
    constexpr bool MF = use_mfma<M, T>();
    __shared__ EmSh<M, T, NT> sh;

    const EmProblem pr = probs[blockIdx.x];
    const int tid = threadIdx.x;
    const int nf = pr.n;
    const int npad = pr.npad;
    const int pid = pr.pid;
    em_load_state<M>(sh, Pg, lamg, logdetg, flagsg, pid, tid);

    T yr[FPT][M], yi[FPT][M], v1[FPT], v2[FPT];
    const T2* __restrict__ yb = y + pr.y_off;
#pragma unroll
    for (int k = 0; k < FPT; ++k) {
        const int n = k * NT + tid;
        const bool ok = n < nf;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            T2 val;
            if (ok) val = yb[(int64_t)m * npad + n];
            else { val.x = T(0); val.y = T(0); }
            yr[k][m] = val.x;
            yi[k][m] = val.y;
        }
        v1[k] = ok ? v[pr.v_off + n] : T(1);
        v2[k] = ok ? v[pr.v_off + pr.v2_off + n] : T(1);
    }
    em_prepare<M>(sh, tid);
    __syncthreads();
    const bool frozen_at_entry = (sh.flag & kFreezeMask) != 0;
    const int passes = (iters > 0 && !frozen_at_entry) ? iters : 1;

    // P and Lambda in the bulk precision: prepared here, then rewritten by
    // each basis update (published by its closing barrier)
    int last_it = -1;
    for (int it = 0; it < passes; ++it) {
        T lm[M];
#pragma unroll
        for (int a = 0; a < M; ++a) lm[a] = sh.lamT[a];
        PassAcc<M, T, MF> pa;
        pa.init(sh, tid);
        double llacc = 0.0;
        T v1n[FPT], v2n[FPT];
        bool bad = false;
#pragma unroll
        for (int k = 0; k < FPT; ++k) {
            v1n[k] = v1[k];
            v2n[k] = v2[k];
            if (k * NT >= nf) continue;  // uniform: the whole block of frames is padding
            // P is re-read from LDS for every frame (a broadcast read) rather than
            // held in registers across the frame loop, and frames are not
            // interleaved by the scheduler: both keep the register count low
            // enough for three workgroups per CU.
            __asm__ volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            pa.bin(sh, yr[k], yi[k], v1[k], v2[k], lm, (k * NT + tid) < nf, llacc, v1n[k], v2n[k], bad, tid);
        }
        last_it = (iters > 0 && !frozen_at_entry) ? it : -1;
        if (pa.finish(sh, llacc, bad, it, iters, it_base, frozen_at_entry, nf, ll, ll_stride, pid, eps2, tid)) break;
#pragma unroll
        for (int k = 0; k < FPT; ++k) {
            v1[k] = v1n[k];
            v2[k] = v2n[k];
        }
    }
    em_settle_logdet<M>(sh, last_it, tid);

    if (iters > 0 && !frozen_at_entry) {
#pragma unroll
        for (int k = 0; k < FPT; ++k) {
            const int n = k * NT + tid;
            if (n < nf) {
                v[pr.v_off + n] = v1[k];
                v[pr.v_off + pr.v2_off + n] = v2[k];
            }
        }
        em_store_state<M>(sh, Pg, lamg, logdetg, flagsg, pid, tid);
    }
}

// ============================================================== EM kernel, frames streamed
// Same iteration for problems with more frames than fit in registers: every
// pass re-reads y and v (L2 / MALL / HBM) in chunks of FPT frames per thread.
// v is double-buffered (second buffer at v + v_alt): pass l reads theta^(l)'s
// powers from one buffer and writes the new ones to the other, so a problem
// that freezes keeps its last complete iterate. On exit the committed powers
// are in the first buffer.
template <int M, typename T, int FPT, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 2 : 1))) void em_stream_kernel(
    const EmProblem* __restrict__ probs, const typename Vec2<T>::type* __restrict__ y,
    T* __restrict__ v, int64_t v_alt, double2* __restrict__ Pg, double* __restrict__ lamg,
    double* __restrict__ logdetg, int* __restrict__ flagsg, double* __restrict__ ll,
    int64_t ll_stride, int iters, int it_base, double eps2) {
    using T2 = typename Vec2<T>::type;
    constexpr bool MF = use_mfma<M, T>();
    __shared__ EmSh<M, T, NT> sh;

    const EmProblem pr = probs[blockIdx.x];
    const int tid = threadIdx.x;
    const int nf = pr.n;
    const int npad = pr.npad;
    const int pid = pr.pid;
    em_load_state<M>(sh, Pg, lamg, logdetg, flagsg, pid, tid);
    __syncthreads();
    em_prepare<M>(sh, tid);
    __syncthreads();
    const bool frozen_at_entry = (sh.flag & kFreezeMask) != 0;
    const int passes = (iters > 0 && !frozen_at_entry) ? iters : 1;
    const bool write_v = iters > 0 && !frozen_at_entry;
    const T2* __restrict__ yb = y + pr.y_off;
    int cur = 0;
    int last_it = -1;
    // the frames of one chunk: y and the powers of theta^(l). Lanes past the
    // last frame load the last frame (the bins mask them by `ok`), so every
    // load is unconditional: loads under a branch are waited for inside it,
    // one after the other, while these stay in flight until first used.
    auto load_chunk = [&](int base, const T* __restrict__ vsrc, T (&cyr)[FPT][M], T (&cyi)[FPT][M],
                          T (&ca1)[FPT], T (&ca2)[FPT]) {
#pragma unroll
        for (int k = 0; k < FPT; ++k) {
            const int n = min(base + k * NT + tid, nf - 1);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const T2 val = yb[(int64_t)m * npad + n];
                cyr[k][m] = val.x;
                cyi[k][m] = val.y;
            }
            ca1[k] = vsrc[n];
            ca2[k] = vsrc[pr.v2_off + n];
        }
    };
    for (int it = 0; it < passes; ++it) {
        T lm[M];
#pragma unroll
        for (int a = 0; a < M; ++a) lm[a] = sh.lamT[a];
        PassAcc<M, T, MF> pa;
        pa.init(sh, tid);
        double llacc = 0.0;
        bool bad = false;
        const T* __restrict__ vin = v + (cur ? v_alt : 0) + pr.v_off;
        T* __restrict__ vout = v + (cur ? 0 : v_alt) + pr.v_off;
        for (int base = 0; base < nf; base += NT * FPT) {
            T yr[FPT][M], yi[FPT][M], a1[FPT], a2[FPT];
            load_chunk(base, vin, yr, yi, a1, a2);
#pragma unroll
            for (int k = 0; k < FPT; ++k) {
                const int n = base + k * NT + tid;
                const bool ok = n < nf;
                T n1 = a1[k], n2 = a2[k];
                pa.bin(sh, yr[k], yi[k], a1[k], a2[k], lm, ok, llacc, n1, n2, bad, tid);
                if (ok && write_v) {
                    vout[n] = n1;
                    vout[pr.v2_off + n] = n2;
                }
            }
        }
        last_it = write_v ? it : -1;
        if (pa.finish(sh, llacc, bad, it, iters, it_base, frozen_at_entry, nf, ll, ll_stride, pid, eps2, tid)) break;
        cur ^= 1;
    }
    em_settle_logdet<M>(sh, last_it, tid);

    if (write_v) {
        if (cur) {
            for (int n = tid; n < nf; n += NT) {
                v[pr.v_off + n] = v[v_alt + pr.v_off + n];
                v[pr.v_off + pr.v2_off + n] = v[v_alt + pr.v_off + pr.v2_off + n];
            }
        }
        em_store_state<M>(sh, Pg, lamg, logdetg, flagsg, pid, tid);
    }
}

// Jacobi stopping threshold (squared, relative): full double precision in
// FP64 mode; 1e-8 in the float bulk mode, where the per-bin arithmetic is
// itself only float-accurate (the eigendecomposition still runs in double).
constexpr double kEps2Fp64 = 1e-30;
constexpr double kEps2Fp32Bulk = 1e-16;

template <int M, typename T, int NT>
hipError_t launch_em_fpt(int fpt, const EmProblem* probs, int count, const void* y, void* v, int64_t v_alt,
                         double2* P, double* lam, double* logdet, int* flags, double* ll, int64_t ll_stride,
                         int iters, int it_base, hipStream_t s) {
    using T2 = typename Vec2<T>::type;
    const double eps2 = sizeof(T) == 8 ? kEps2Fp64 : kEps2Fp32Bulk;
    const dim3 grid(count), block(NT);
    const T2* yy = static_cast<const T2*>(y);
    T* vv = static_cast<T*>(v);
    switch (fpt) {
        case 0:
            if constexpr (NT == kEmThreads) {
                em_stream_kernel<M, T, kStreamFramesPerThread, NT><<<grid, block, 0, s>>>(
                    probs, yy, vv, v_alt, P, lam, logdet, flags, ll, ll_stride, iters, it_base, eps2);
                break;
            } else {
                return hipErrorInvalidValue;  // streamed problems run with kEmThreads threads only
            }
        case 1: em_kernel<M, T, 1, NT><<<grid, block, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, ll_stride, iters, it_base, eps2); break;
        case 2: em_kernel<M, T, 2, NT><<<grid, block, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, ll_stride, iters, it_base, eps2); break;
        case 4: em_kernel<M, T, 4, NT><<<grid, block, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, ll_stride, iters, it_base, eps2); break;
        case 8: em_kernel<M, T, 8, NT><<<grid, block, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, ll_stride, iters, it_base, eps2); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NT>
hipError_t launch_em_nt(int M, bool fp64, int fpt, const EmProblem* probs, int count, const void* y, void* v,
                        int64_t v_alt, double2* P, double* lam, double* logdet, int* flags, double* ll,
                        int64_t ll_stride, int iters, int it_base, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    switch (M) {
#define FCA_EM_CASE(MM_)                                                                                      \
    case MM_:                                                                                                  \
        return fp64 ? launch_em_fpt<MM_, double, NT>(fpt, probs, count, y, v, v_alt, P, lam, logdet, flags, ll, \
                                                     ll_stride, iters, it_base, s)                                      \
                    : launch_em_fpt<MM_, float, NT>(fpt, probs, count, y, v, v_alt, P, lam, logdet, flags, ll,  \
                                                    ll_stride, iters, it_base, s);
        FCA_EM_CASE(1) FCA_EM_CASE(2) FCA_EM_CASE(3) FCA_EM_CASE(4)
        FCA_EM_CASE(5) FCA_EM_CASE(6) FCA_EM_CASE(7) FCA_EM_CASE(8)
#undef FCA_EM_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fca
