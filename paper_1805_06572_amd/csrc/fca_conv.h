// fca_conv.h -- the conventional FCA EM (Section 2) on gfx950, the
// frame-wise algorithm FastFCA replaces: per bin, the mixture covariance
// v1 R1 + v2 R2 is factorised (Cholesky) and the E-step needs its solves and
// matrix products (eqs. MMSE, postquadexp); the M-step is eqs. vupdate and
// Supdate. It runs on the same context and state as the FastFCA kernels: on
// entry R_j are recovered from the eigenbasis form (R2 = P^-H P^-1,
// R1 = P^-H Lambda P^-1), on exit the eigenbasis form is recomputed by the
// FP64 GEVD, so the two algorithms can be interleaved and compared.
//
// Organisation mirrors em_kernel: one workgroup owns one (mixture,
// frequency) problem for all iterations of a call, frames resident in
// registers (at most kMaxFrames), FP64 fixed-order workgroup sums, FP64
// per-frequency inverses R_j^-1 (eq. vupdate uses the old R_j).
// Instantiated by fca_conv_lo.hip (M <= 4) and fca_conv_m5.hip ..
// fca_conv_m8.hip, so the slow compilations run in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "fca_device.h"
#include "fca_internal.h"

namespace fca {

template <int M, typename T> struct ConvShared {
    using T2 = typename Vec2<T>::type;
    static constexpr int NTH = kEmThreads;
    static constexpr int MM = M * M;
    static constexpr int NV = 2 * MM;
    static constexpr int CH = NV < 32 ? NV : 32;
    static constexpr int NCH = (NV + CH - 1) / CH;
    static constexpr int G = kEmThreads / 32;
    static constexpr int NW = kEmThreads / 64;
    double2 S[2][MM];     // R_1, R_2 (FP64, full Hermitian); the sums land here
    double2 Sold[2][MM];  // R_j of theta^(l), kept for freezing
    T2 St[2][MM];         // R_j in the bulk precision
    T2 Si[2][MM];         // R_j^-1 in the bulk precision
    int flag, bad;
    T red[kEmThreads * (CH + 1)];
    double wh[NW][64];
    double wp[NW][NV];
    double LL[NW];
    double2 Id[MM], Pn[MM];
    double lamN[M];
    GevdScratch ws;
};

// One time-frequency bin of the conventional EM:
//   R = v1 R1 + v2 R2 = L L^H                         (covariance of y, eq. like)
//   log p(y) term: -log det R - ||L^-1 y||^2
//   w = R^-1 y, mu_j = v_j R_j w                      eq. (MMSE)
//   C = v1 R1 R^-1 (v2 R2)                            eq. (postquadexp), the same for j = 1, 2
//   Phi_j = mu_j mu_j^H + C
//   v_j' = Re tr(R_j^-1 Phi_j) / M                    eq. (vupdate), old R_j
//   sums_j += Phi_j / v_j'                             eq. (Supdate), upper triangle
template <int M, typename T>
__device__ __forceinline__ void conv_bin(const T (&yr)[M], const T (&yi)[M], T a1, T a2,
                                         const typename Vec2<T>::type* S1, const typename Vec2<T>::type* S2,
                                         const typename Vec2<T>::type* S1i, const typename Vec2<T>::type* S2i,
                                         bool ok, T (&acc)[2 * M * M], double& llacc, T& nv1o, T& nv2o,
                                         bool& bad) {
    using MT = Math<T>;
    constexpr int MM = M * M;
    // ---- Cholesky factor of R (lower triangle), reciprocal pivots
    T Lr[M][M], Li[M][M], invd[M];
    T logdet = T(0);
#pragma unroll
    for (int j = 0; j < M; ++j) {
        T d = a1 * S1[j * M + j].x + a2 * S2[j * M + j].x;
#pragma unroll
        for (int q = 0; q < j; ++q) d -= Lr[j][q] * Lr[j][q] + Li[j][q] * Li[j][q];
        invd[j] = MT::rsqrt(d);
        Lr[j][j] = d * invd[j];
        Li[j][j] = T(0);
        logdet += MT::log(d);
#pragma unroll
        for (int i = j + 1; i < M; ++i) {
            T sr = a1 * S1[i * M + j].x + a2 * S2[i * M + j].x;
            T si = a1 * S1[i * M + j].y + a2 * S2[i * M + j].y;
#pragma unroll
            for (int q = 0; q < j; ++q) {  // - L_iq conj(L_jq)
                sr -= Lr[i][q] * Lr[j][q] + Li[i][q] * Li[j][q];
                si -= Li[i][q] * Lr[j][q] - Lr[i][q] * Li[j][q];
            }
            Lr[i][j] = sr * invd[j];
            Li[i][j] = si * invd[j];
        }
    }
    // ---- z = L^-1 y, quad = ||z||^2, w = L^-H z
    T zr[M], zi[M], wr[M], wi[M];
    T quad = T(0);
#pragma unroll
    for (int i = 0; i < M; ++i) {
        T sr = yr[i], si = yi[i];
#pragma unroll
        for (int q = 0; q < i; ++q) {
            sr -= Lr[i][q] * zr[q] - Li[i][q] * zi[q];
            si -= Lr[i][q] * zi[q] + Li[i][q] * zr[q];
        }
        zr[i] = sr * invd[i];
        zi[i] = si * invd[i];
        quad += zr[i] * zr[i] + zi[i] * zi[i];
    }
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
        T sr = zr[i], si = zi[i];
#pragma unroll
        for (int q = i + 1; q < M; ++q) {  // - conj(L_qi) w_q
            sr -= Lr[q][i] * wr[q] + Li[q][i] * wi[q];
            si -= Lr[q][i] * wi[q] - Li[q][i] * wr[q];
        }
        wr[i] = sr * invd[i];
        wi[i] = si * invd[i];
    }
    // ---- mu_j = v_j R_j w
    T m1r[M], m1i[M], m2r[M], m2i[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        T s1r = T(0), s1i = T(0), s2r = T(0), s2i = T(0);
#pragma unroll
        for (int q = 0; q < M; ++q) {
            const auto p1 = S1[i * M + q], p2 = S2[i * M + q];
            s1r += p1.x * wr[q] - p1.y * wi[q];
            s1i += p1.x * wi[q] + p1.y * wr[q];
            s2r += p2.x * wr[q] - p2.y * wi[q];
            s2i += p2.x * wi[q] + p2.y * wr[q];
        }
        m1r[i] = a1 * s1r;
        m1i[i] = a1 * s1i;
        m2r[i] = a2 * s2r;
        m2i[i] = a2 * s2i;
    }
    // ---- C = v1 R1 X with X = R^-1 (v2 R2), column by column
    T Cr[M][M], Ci[M][M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        T tr_[M], ti_[M], xr[M], xi[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
            T sr = a2 * S2[i * M + c].x, si = a2 * S2[i * M + c].y;
#pragma unroll
            for (int q = 0; q < i; ++q) {
                sr -= Lr[i][q] * tr_[q] - Li[i][q] * ti_[q];
                si -= Lr[i][q] * ti_[q] + Li[i][q] * tr_[q];
            }
            tr_[i] = sr * invd[i];
            ti_[i] = si * invd[i];
        }
#pragma unroll
        for (int i = M - 1; i >= 0; --i) {
            T sr = tr_[i], si = ti_[i];
#pragma unroll
            for (int q = i + 1; q < M; ++q) {
                sr -= Lr[q][i] * xr[q] + Li[q][i] * xi[q];
                si -= Lr[q][i] * xi[q] - Li[q][i] * xr[q];
            }
            xr[i] = sr * invd[i];
            xi[i] = si * invd[i];
        }
#pragma unroll
        for (int i = 0; i < M; ++i) {
            T sr = T(0), si = T(0);
#pragma unroll
            for (int q = 0; q < M; ++q) {
                const auto p1 = S1[i * M + q];
                sr += p1.x * xr[q] - p1.y * xi[q];
                si += p1.x * xi[q] + p1.y * xr[q];
            }
            Cr[i][c] = a1 * sr;
            Ci[i][c] = a1 * si;
        }
    }
    // ---- v_j' = Re[mu_j^H R_j^-1 mu_j + tr(R_j^-1 C)] / M
    T q1 = T(0), q2 = T(0);
#pragma unroll
    for (int a = 0; a < M; ++a) {
#pragma unroll
        for (int b = 0; b < M; ++b) {
            const auto s1 = S1i[a * M + b], s2 = S2i[a * M + b];
            // Re(conj(mu_a) Si_ab mu_b) and Re(Si_ab C_ba)
            const T t1r = s1.x * m1r[b] - s1.y * m1i[b], t1i = s1.x * m1i[b] + s1.y * m1r[b];
            const T t2r = s2.x * m2r[b] - s2.y * m2i[b], t2i = s2.x * m2i[b] + s2.y * m2r[b];
            q1 += m1r[a] * t1r + m1i[a] * t1i + s1.x * Cr[b][a] - s1.y * Ci[b][a];
            q2 += m2r[a] * t2r + m2i[a] * t2i + s2.x * Cr[b][a] - s2.y * Ci[b][a];
        }
    }
    T nv1 = q1 * (T(1) / T(M));
    T nv2 = q2 * (T(1) / T(M));
    if (ok) {
        llacc += (double)(-logdet - quad);
        bad = bad || !(nv1 > T(0)) || !(nv2 > T(0)) || !isfinite(nv1) || !isfinite(nv2);
    }
    if constexpr (sizeof(T) == 4) {
        // the same power floor as the FastFCA float path
        nv1 = fmaxf(nv1, kPowerFloorF32);
        nv2 = fmaxf(nv2, kPowerFloorF32);
    }
    if (ok) {
        nv1o = nv1;
        nv2o = nv2;
    }
    const T iv1 = ok ? MT::rcp(nv1) : T(0);
    const T iv2 = ok ? MT::rcp(nv2) : T(0);
    // ---- sums of Phi_j / v_j' (Hermitian part of C), upper triangle
#pragma unroll
    for (int i = 0; i < M; ++i) {
        acc[i] += (m1r[i] * m1r[i] + m1i[i] * m1i[i] + Cr[i][i]) * iv1;
        acc[MM + i] += (m2r[i] * m2r[i] + m2i[i] * m2i[i] + Cr[i][i]) * iv2;
#pragma unroll
        for (int q = i + 1; q < M; ++q) {
            const int o = M + 2 * pair_index(M, i, q);
            const T hr = T(0.5) * (Cr[i][q] + Cr[q][i]);
            const T hi = T(0.5) * (Ci[i][q] - Ci[q][i]);
            // mu_i conj(mu_q)
            acc[o] += (m1r[i] * m1r[q] + m1i[i] * m1i[q] + hr) * iv1;
            acc[o + 1] += (m1i[i] * m1r[q] - m1r[i] * m1i[q] + hi) * iv1;
            acc[MM + o] += (m2r[i] * m2r[q] + m2i[i] * m2i[q] + hr) * iv2;
            acc[MM + o + 1] += (m2i[i] * m2r[q] - m2r[i] * m2i[q] + hi) * iv2;
        }
    }
}

template <int M, typename T, int FPT>
__global__ __launch_bounds__(kEmThreads) void conv_em_kernel(
    const EmProblem* __restrict__ probs, const typename Vec2<T>::type* __restrict__ y, T* __restrict__ v,
    double2* __restrict__ Pg, double* __restrict__ lamg, double* __restrict__ logdetg, int* __restrict__ flagsg,
    double* __restrict__ ll, int64_t ll_stride, int iters, int it_base) {
    using T2 = typename Vec2<T>::type;
    constexpr int NT = kEmThreads;
    constexpr int MM = M * M, NV = 2 * MM, NW = kEmThreads / 64;
    __shared__ ConvShared<M, T> sh;
    const EmProblem pr = probs[blockIdx.x];
    const int tid = threadIdx.x;
    const int nf = pr.n, npad = pr.npad, pid = pr.pid;
    const int ll_count = iters > 0 ? iters : 1;

    if (tid < MM) sh.Id[tid] = make_double2((tid % (M + 1)) == 0 ? 1.0 : 0.0, 0.0);
    if (tid == 0) {
        sh.flag = flagsg[pid];
        sh.bad = 0;
        // R_j of the current eigenbasis form: R2 = P^-H P^-1, R1 = P^-H Lambda P^-1
        double2 X[M][M];
        invert<M>(Pg + (int64_t)pid * kMaxM * kMaxM, X);
        const double* lm = lamg + (int64_t)pid * kMaxM;
        for (int a = 0; a < M; ++a)
            for (int b = 0; b < M; ++b) {
                double2 s1 = make_double2(0.0, 0.0), s2 = make_double2(0.0, 0.0);
                for (int k = 0; k < M; ++k) {
                    const double2 t = cmulc(X[k][b], X[k][a]);
                    s2 = cadd(s2, t);
                    s1 = cadd(s1, cscale(lm[k], t));
                }
                if (a == b) { s1.y = 0.0; s2.y = 0.0; }
                sh.S[0][a * M + b] = s1;
                sh.S[1][a * M + b] = s2;
            }
    }
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
    __syncthreads();
    const bool frozen_at_entry = (sh.flag & kFreezeMask) != 0;
    const int passes = (iters > 0 && !frozen_at_entry) ? iters : 1;

    for (int it = 0; it < passes; ++it) {
        if (tid == 0) {
            double2 X1[M][M], X2[M][M];
            const bool ok1 = invert<M>(sh.S[0], X1);
            const bool ok2 = invert<M>(sh.S[1], X2);
            if (!ok1 || !ok2) sh.bad = 1;
            for (int a = 0; a < M; ++a)
                for (int b = 0; b < M; ++b) {
                    const int e = a * M + b;
                    sh.Sold[0][e] = sh.S[0][e];
                    sh.Sold[1][e] = sh.S[1][e];
                    sh.St[0][e] = make_vec2<T>((T)sh.S[0][e].x, (T)sh.S[0][e].y);
                    sh.St[1][e] = make_vec2<T>((T)sh.S[1][e].x, (T)sh.S[1][e].y);
                    sh.Si[0][e] = make_vec2<T>((T)X1[a][b].x, (T)X1[a][b].y);
                    sh.Si[1][e] = make_vec2<T>((T)X2[a][b].x, (T)X2[a][b].y);
                }
        }
        __syncthreads();
        T acc[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] = T(0);
        double llacc = 0.0;
        T v1n[FPT], v2n[FPT];
        bool bad = false;
#pragma unroll
        for (int k = 0; k < FPT; ++k) {
            v1n[k] = v1[k];
            v2n[k] = v2[k];
            if (k * NT >= nf) continue;
            conv_bin<M, T>(yr[k], yi[k], v1[k], v2[k], sh.St[0], sh.St[1], sh.Si[0], sh.Si[1], (k * NT + tid) < nf,
                           acc, llacc, v1n[k], v2n[k], bad);
        }
        if (bad) sh.bad = 1;
        wg_reduce_sums<M>(sh, acc, llacc, nf, tid, nullptr);
        if (tid == 0) {
            double tot = 0.0;
            for (int w = 0; w < NW; ++w) tot += sh.LL[w];
            tot += -(double)nf * (double)M * kLogPi;
            const bool last = (iters == 0) || frozen_at_entry;
            if (last) {
                for (int l = it; l < ll_count; ++l) ll[(int64_t)l * ll_stride + pid] = tot;
            } else {
                ll[(int64_t)it * ll_stride + pid] = tot;
                bool finite = true;
                for (int e = 0; e < MM; ++e) finite = finite && cfinite(sh.S[0][e]) && cfinite(sh.S[1][e]);
                if (sh.bad || !finite) {
                    // frozen at theta^(it); the failing iteration of the call is recorded
                    sh.flag |= kFlagNonFinite | ((it_base + it + 1) << kFlagIterShift);
                    for (int e = 0; e < MM; ++e) {
                        sh.S[0][e] = sh.Sold[0][e];
                        sh.S[1][e] = sh.Sold[1][e];
                    }
                    for (int l = it + 1; l < ll_count; ++l) ll[(int64_t)l * ll_stride + pid] = tot;
                }
            }
        }
        __syncthreads();
        if (iters == 0 || frozen_at_entry || (sh.flag & kFreezeMask)) break;
#pragma unroll
        for (int k = 0; k < FPT; ++k) {
            v1[k] = v1n[k];
            v2[k] = v2n[k];
        }
    }

    if (iters > 0 && !frozen_at_entry) {
#pragma unroll
        for (int k = 0; k < FPT; ++k) {
            const int n = k * NT + tid;
            if (n < nf) {
                v[pr.v_off + n] = v1[k];
                v[pr.v_off + pr.v2_off + n] = v2[k];
            }
        }
        // back to the eigenbasis form (eq. GEVD): P^H R2 P = I, P^H R1 P = Lambda,
        // log|det P|^2 = -log det R2
        if (tid < 64) {
            double dld = 0.0;
            const int flag = gevd_wave<M>(sh.S[0], sh.S[1], sh.Id, sh.ws, sh.Pn, sh.lamN, &dld, 1e-30);
            wave_lds_sync();
            if (!(flag & kFreezeMask)) {
                if (tid < MM) Pg[(int64_t)pid * kMaxM * kMaxM + tid] = sh.Pn[tid];
                if (tid < M) lamg[(int64_t)pid * kMaxM + tid] = sh.lamN[tid];
                if (tid == 0) logdetg[pid] = dld;
            }
            if (tid == 0) flagsg[pid] = sh.flag | (flag & kFreezeMask);
        }
    }
}

// The same iteration for problems with more frames than fit in registers:
// every pass re-reads y and the powers in chunks of kEmThreads frames (one
// per thread). The powers are double-buffered (second buffer at v + v_alt)
// as in em_stream_kernel: pass l reads theta^(l)'s powers from one buffer and
// writes the new ones to the other, so a problem that freezes keeps its last
// complete iterate; on exit the committed powers are in the first buffer.
// A thread meets its frames in the order the resident kernel keeps them, so
// the sums, and the results, equal that kernel's bit for bit.
template <int M, typename T>
__global__ __launch_bounds__(kEmThreads) void conv_stream_kernel(
    const EmProblem* __restrict__ probs, const typename Vec2<T>::type* __restrict__ y, T* __restrict__ v,
    int64_t v_alt, double2* __restrict__ Pg, double* __restrict__ lamg, double* __restrict__ logdetg,
    int* __restrict__ flagsg, double* __restrict__ ll, int64_t ll_stride, int iters, int it_base) {
    using T2 = typename Vec2<T>::type;
    constexpr int NT = kEmThreads;
    constexpr int MM = M * M, NV = 2 * MM, NW = kEmThreads / 64;
    __shared__ ConvShared<M, T> sh;
    const EmProblem pr = probs[blockIdx.x];
    const int tid = threadIdx.x;
    const int nf = pr.n, npad = pr.npad, pid = pr.pid;
    const int ll_count = iters > 0 ? iters : 1;

    if (tid < MM) sh.Id[tid] = make_double2((tid % (M + 1)) == 0 ? 1.0 : 0.0, 0.0);
    if (tid == 0) {
        sh.flag = flagsg[pid];
        sh.bad = 0;
        double2 X[M][M];
        invert<M>(Pg + (int64_t)pid * kMaxM * kMaxM, X);
        const double* lm = lamg + (int64_t)pid * kMaxM;
        for (int a = 0; a < M; ++a)
            for (int b = 0; b < M; ++b) {
                double2 s1 = make_double2(0.0, 0.0), s2 = make_double2(0.0, 0.0);
                for (int k = 0; k < M; ++k) {
                    const double2 t = cmulc(X[k][b], X[k][a]);
                    s2 = cadd(s2, t);
                    s1 = cadd(s1, cscale(lm[k], t));
                }
                if (a == b) { s1.y = 0.0; s2.y = 0.0; }
                sh.S[0][a * M + b] = s1;
                sh.S[1][a * M + b] = s2;
            }
    }
    __syncthreads();
    const T2* __restrict__ yb = y + pr.y_off;
    const bool frozen_at_entry = (sh.flag & kFreezeMask) != 0;
    const int passes = (iters > 0 && !frozen_at_entry) ? iters : 1;
    const bool write_v = iters > 0 && !frozen_at_entry;
    int cur = 0;
    for (int it = 0; it < passes; ++it) {
        if (tid == 0) {
            double2 X1[M][M], X2[M][M];
            const bool ok1 = invert<M>(sh.S[0], X1);
            const bool ok2 = invert<M>(sh.S[1], X2);
            if (!ok1 || !ok2) sh.bad = 1;
            for (int a = 0; a < M; ++a)
                for (int b = 0; b < M; ++b) {
                    const int e = a * M + b;
                    sh.Sold[0][e] = sh.S[0][e];
                    sh.Sold[1][e] = sh.S[1][e];
                    sh.St[0][e] = make_vec2<T>((T)sh.S[0][e].x, (T)sh.S[0][e].y);
                    sh.St[1][e] = make_vec2<T>((T)sh.S[1][e].x, (T)sh.S[1][e].y);
                    sh.Si[0][e] = make_vec2<T>((T)X1[a][b].x, (T)X1[a][b].y);
                    sh.Si[1][e] = make_vec2<T>((T)X2[a][b].x, (T)X2[a][b].y);
                }
        }
        __syncthreads();
        T acc[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] = T(0);
        double llacc = 0.0;
        bool bad = false;
        const T* __restrict__ vin = v + (cur ? v_alt : 0) + pr.v_off;
        T* __restrict__ vout = v + (cur ? 0 : v_alt) + pr.v_off;
        for (int base = 0; base < nf; base += NT) {
            const int n = base + tid;
            const bool ok = n < nf;
            const int nc = ok ? n : nf - 1;   // lanes past the last frame load it and are masked
            T yr[M], yi[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const T2 val = yb[(int64_t)m * npad + nc];
                yr[m] = ok ? val.x : T(0);
                yi[m] = ok ? val.y : T(0);
            }
            const T a1 = ok ? vin[nc] : T(1), a2 = ok ? vin[pr.v2_off + nc] : T(1);
            T n1 = a1, n2 = a2;
            conv_bin<M, T>(yr, yi, a1, a2, sh.St[0], sh.St[1], sh.Si[0], sh.Si[1], ok, acc, llacc, n1, n2, bad);
            if (ok && write_v) {
                vout[n] = n1;
                vout[pr.v2_off + n] = n2;
            }
        }
        if (bad) sh.bad = 1;
        wg_reduce_sums<M>(sh, acc, llacc, nf, tid, nullptr);
        if (tid == 0) {
            double tot = 0.0;
            for (int w = 0; w < NW; ++w) tot += sh.LL[w];
            tot += -(double)nf * (double)M * kLogPi;
            const bool last = (iters == 0) || frozen_at_entry;
            if (last) {
                for (int l = it; l < ll_count; ++l) ll[(int64_t)l * ll_stride + pid] = tot;
            } else {
                ll[(int64_t)it * ll_stride + pid] = tot;
                bool finite = true;
                for (int e = 0; e < MM; ++e) finite = finite && cfinite(sh.S[0][e]) && cfinite(sh.S[1][e]);
                if (sh.bad || !finite) {
                    sh.flag |= kFlagNonFinite | ((it_base + it + 1) << kFlagIterShift);
                    for (int e = 0; e < MM; ++e) {
                        sh.S[0][e] = sh.Sold[0][e];
                        sh.S[1][e] = sh.Sold[1][e];
                    }
                    for (int l = it + 1; l < ll_count; ++l) ll[(int64_t)l * ll_stride + pid] = tot;
                }
            }
        }
        __syncthreads();
        if (iters == 0 || frozen_at_entry || (sh.flag & kFreezeMask)) break;
        cur ^= 1;
    }

    if (write_v) {
        if (cur) {
            for (int n = tid; n < nf; n += NT) {
                v[pr.v_off + n] = v[v_alt + pr.v_off + n];
                v[pr.v_off + pr.v2_off + n] = v[v_alt + pr.v_off + pr.v2_off + n];
            }
        }
        if (tid < 64) {
            double dld = 0.0;
            const int flag = gevd_wave<M>(sh.S[0], sh.S[1], sh.Id, sh.ws, sh.Pn, sh.lamN, &dld, 1e-30);
            wave_lds_sync();
            if (!(flag & kFreezeMask)) {
                if (tid < MM) Pg[(int64_t)pid * kMaxM * kMaxM + tid] = sh.Pn[tid];
                if (tid < M) lamg[(int64_t)pid * kMaxM + tid] = sh.lamN[tid];
                if (tid == 0) logdetg[pid] = dld;
            }
            if (tid == 0) flagsg[pid] = sh.flag | (flag & kFreezeMask);
        }
    }
}

// fpt 0: the streamed kernel (powers double-buffered at v + v_alt).
template <int M, typename T>
hipError_t launch_conv_fpt(int fpt, const EmProblem* probs, int count, const void* y, void* v, int64_t v_alt,
                           double2* P, double* lam, double* logdet, int* flags, double* ll, int64_t ll_stride,
                           int iters, int it_base, hipStream_t s) {
    using T2 = typename Vec2<T>::type;
    const T2* yy = static_cast<const T2*>(y);
    T* vv = static_cast<T*>(v);
    switch (fpt) {
        case 0: conv_stream_kernel<M, T><<<count, kEmThreads, 0, s>>>(probs, yy, vv, v_alt, P, lam, logdet, flags, ll, ll_stride, iters, it_base); break;
        case 1: conv_em_kernel<M, T, 1><<<count, kEmThreads, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, ll_stride, iters, it_base); break;
        case 2: conv_em_kernel<M, T, 2><<<count, kEmThreads, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, ll_stride, iters, it_base); break;
        case 4: conv_em_kernel<M, T, 4><<<count, kEmThreads, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, ll_stride, iters, it_base); break;
        case 8: conv_em_kernel<M, T, 8><<<count, kEmThreads, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, ll_stride, iters, it_base); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fca
