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

#include "fca_device.h"
#include "fca_internal.h"

namespace fca {

// ============================================================== EM iteration pieces
// LDS state of one (mixture, frequency) problem inside an EM workgroup.
template <int M, typename T, int NT_ = kEmThreads> struct EmShared {
    static constexpr int NTH = NT_;  // threads of the workgroup
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
    double fin[NV];
    T red[NT_ * (CH + 1)];
    double red2[G * CH];
    double LL[NW];
    GevdScratch ws;
};

template <int M, typename T, int NT_>
__device__ __forceinline__ void em_load_state(EmShared<M, T, NT_>& sh, const double2* __restrict__ Pg,
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

template <int M, typename T, int NT_>
__device__ __forceinline__ void em_store_state(const EmShared<M, T, NT_>& sh, double2* __restrict__ Pg,
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
template <int M, typename T, int NT_>
__device__ __forceinline__ void em_prepare(EmShared<M, T, NT_>& sh, int tid) {
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
//   acc += (mu~_j mu~_j^H + diag c) / v_j'  (upper triangle)       eq. (updateStildeeff)
//   llacc += -sum_i log d_i - sum_i |y~_i|^2 / d_i   (log-likelihood of theta^(l))
// `ok` masks padding frames (no contribution, powers unchanged).
template <int M, typename T>
__device__ __forceinline__ void em_bin(const T (&yr)[M], const T (&yi)[M], T a1, T a2, const T (&lm)[M],
                                       const typename Vec2<T>::type* Pt, bool ok, T (&acc)[2 * M * M],
                                       double& llacc, T& nv1o, T& nv2o, bool& bad) {
    using T2 = typename Vec2<T>::type;
    using MT = Math<T>;
    constexpr int MM = M * M;
    T ytr[M], yti[M], e[M], r[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
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
#pragma unroll
    for (int i = 0; i < M; i += 2) {
        const T pd = (i + 1 < M) ? d[i] * d[i + 1] : d[i];
        logd += MT::log(pd);
    }
    // v1' = (v1/M) sum r_i (v1 lam_i e_i r_i + v2), v2' = (v2/M) sum r_i (v2 e_i r_i + v1 lam_i)
    T s1 = T(0), s2 = T(0);
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const T er = e[i] * r[i];
        s1 = fma(r[i], fma(a1 * lm[i], er, a2), s1);
        s2 = fma(r[i], fma(a2, er, a1 * lm[i]), s2);
    }
    const T nv1 = a1 * s1 * (T(1) / T(M));
    const T nv2 = a2 * s2 * (T(1) / T(M));
    if (ok) {
        llacc += (double)(-logd - quad);
        bad = bad || !(nv1 > T(0)) || !(nv2 > T(0)) || !isfinite(nv1) || !isfinite(nv2);
        nv1o = nv1;
        nv2o = nv2;
    }
    // u_j = mu~_j / sqrt(v_j') makes the rank-one term u_j u_j^H
    const T w1 = ok ? MT::rsqrt(nv1) : T(0);
    const T w2 = ok ? MT::rsqrt(nv2) : T(0);
    const T iv1 = w1 * w1, iv2 = w2 * w2;
    T u1r[M], u1i[M], u2r[M], u2i[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const T g1 = a1 * lm[i] * r[i];
        const T g2 = a2 * r[i];
        const T c = g1 * a2;
        const T s1i = g1 * w1, s2i = g2 * w2;
        u1r[i] = s1i * ytr[i];
        u1i[i] = s1i * yti[i];
        u2r[i] = s2i * ytr[i];
        u2i[i] = s2i * yti[i];
        acc[i] = fma(s1i * s1i, e[i], fma(c, iv1, acc[i]));
        acc[MM + i] = fma(s2i * s2i, e[i], fma(c, iv2, acc[MM + i]));
    }
#pragma unroll
    for (int i = 0; i < M; ++i) {
#pragma unroll
        for (int q = i + 1; q < M; ++q) {
            const int o = M + 2 * pair_index(M, i, q);
            acc[o] = fma(u1r[i], u1r[q], fma(u1i[i], u1i[q], acc[o]));
            acc[o + 1] = fma(u1i[i], u1r[q], fma(-u1r[i], u1i[q], acc[o + 1]));
            acc[MM + o] = fma(u2r[i], u2r[q], fma(u2i[i], u2i[q], acc[MM + o]));
            acc[MM + o + 1] = fma(u2i[i], u2r[q], fma(-u2r[i], u2i[q], acc[MM + o + 1]));
        }
    }
}

// End of one pass over the frames: FP64 reduction of the accumulators and of
// the log-likelihood over the workgroup (fixed order), S~_j = sums / N, record
// LL(theta^(it)), then the FP64 GEVD of (S~1, S~2) and the basis update
// P <- P Q, Lambda <- Sigma (eqs. GEVDeff5, updatePeff, updateLambdaeff) on
// wave 0. Returns true when the caller must stop iterating: an evaluation-only
// pass, a problem frozen on entry, or a failure that froze it now (it then
// keeps theta^(it), whose log-likelihood stands for the later iterations).
template <int M, typename T, int NT_>
__device__ __forceinline__ bool em_finish(EmShared<M, T, NT_>& sh, const T (&acc)[2 * M * M], double llacc,
                                          bool bad, int it, int iters, bool frozen_at_entry, int nf,
                                          double* __restrict__ ll, int64_t ll_stride, int pid, double eps2,
                                          int tid) {
    constexpr int MM = M * M, NW = NT_ / 64;
    const int ll_count = iters > 0 ? iters : 1;
    if (bad) sh.bad = 1;
    wg_reduce_sums<M>(sh, acc, llacc, nf, tid);
    if (tid < 64) {
        const bool last = (iters == 0) || frozen_at_entry;
        double tot = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) tot += sh.LL[w];
        tot += (double)nf * (-(double)M * kLogPi + sh.logdet);
        if (last) {
            if (tid == 0)
                for (int l = it; l < ll_count; ++l) ll[(int64_t)l * ll_stride + pid] = tot;
        } else {
            if (tid == 0) ll[(int64_t)it * ll_stride + pid] = tot;
            int flag = sh.bad ? kFlagNonFinite : 0;
            double dld = 0.0;
            // the eigendecomposition is this workgroup's critical path: give its
            // wave issue priority over co-resident waves streaming frames
            __builtin_amdgcn_s_setprio(3);
            if (!flag) flag = gevd_wave<M>(sh.S[0], sh.S[1], sh.P, sh.ws, sh.Pn, sh.lamN, &dld, eps2);
            __builtin_amdgcn_s_setprio(0);
            wave_lds_sync();
            if (flag & kFreezeMask) {
                if (tid == 0)
                    for (int l = it + 1; l < ll_count; ++l) ll[(int64_t)l * ll_stride + pid] = tot;
            } else {
                if (tid < MM) sh.P[tid] = sh.Pn[tid];
                if (tid < M) sh.lam[tid] = sh.lamN[tid];
                if (tid == 0) sh.logdet += dld;
            }
            if (tid == 0) sh.flag |= flag;
        }
    }
    __syncthreads();
    return iters == 0 || frozen_at_entry || (sh.flag & kFreezeMask);
}

// ============================================================== EM kernel, frames resident
// One workgroup owns one (mixture, frequency) EM problem for all iterations of
// a call; each thread keeps FPT frames of y and v in registers, so y(n,f) and
// v_j(n,f) cross HBM once per call, not once per iteration.
template <int M, typename T, int FPT, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void em_kernel(
    const EmProblem* __restrict__ probs, const typename Vec2<T>::type* __restrict__ y,
    T* __restrict__ v, double2* __restrict__ Pg, double* __restrict__ lamg,
    double* __restrict__ logdetg, int* __restrict__ flagsg, double* __restrict__ ll,
    int64_t ll_stride, int iters, double eps2) {
    using T2 = typename Vec2<T>::type;
    constexpr int NV = 2 * M * M;
    __shared__ EmShared<M, T, NT> sh;

    const EmProblem pr = probs[blockIdx.x];
    const int tid = threadIdx.x;
    const int nf = pr.n;
    const int npad = pr.npad;
    const int pid = pr.pid;
    em_load_state(sh, Pg, lamg, logdetg, flagsg, pid, tid);

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
        em_prepare(sh, tid);
        __syncthreads();
        T lm[M];
#pragma unroll
        for (int a = 0; a < M; ++a) lm[a] = sh.lamT[a];
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
            if (k * NT >= nf) continue;  // uniform: the whole block of frames is padding
            // P is re-read from LDS for every frame (a broadcast read) rather than
            // held in registers across the frame loop, and frames are not
            // interleaved by the scheduler: both keep the register count low
            // enough for three workgroups per CU.
            __asm__ volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            em_bin<M, T>(yr[k], yi[k], v1[k], v2[k], lm, sh.Pt, (k * NT + tid) < nf, acc, llacc, v1n[k],
                         v2n[k], bad);
        }
        if (em_finish<M, T>(sh, acc, llacc, bad, it, iters, frozen_at_entry, nf, ll, ll_stride, pid, eps2, tid))
            break;
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
        em_store_state(sh, Pg, lamg, logdetg, flagsg, pid, tid);
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
__global__ __launch_bounds__(NT) void em_stream_kernel(
    const EmProblem* __restrict__ probs, const typename Vec2<T>::type* __restrict__ y,
    T* __restrict__ v, int64_t v_alt, double2* __restrict__ Pg, double* __restrict__ lamg,
    double* __restrict__ logdetg, int* __restrict__ flagsg, double* __restrict__ ll,
    int64_t ll_stride, int iters, double eps2) {
    using T2 = typename Vec2<T>::type;
    constexpr int NV = 2 * M * M;
    __shared__ EmShared<M, T, NT> sh;

    const EmProblem pr = probs[blockIdx.x];
    const int tid = threadIdx.x;
    const int nf = pr.n;
    const int npad = pr.npad;
    const int pid = pr.pid;
    em_load_state(sh, Pg, lamg, logdetg, flagsg, pid, tid);
    __syncthreads();
    const bool frozen_at_entry = (sh.flag & kFreezeMask) != 0;
    const int passes = (iters > 0 && !frozen_at_entry) ? iters : 1;
    const bool write_v = iters > 0 && !frozen_at_entry;
    const T2* __restrict__ yb = y + pr.y_off;
    int cur = 0;

    for (int it = 0; it < passes; ++it) {
        em_prepare(sh, tid);
        __syncthreads();
        T lm[M];
#pragma unroll
        for (int a = 0; a < M; ++a) lm[a] = sh.lamT[a];
        T acc[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] = T(0);
        double llacc = 0.0;
        bool bad = false;
        const T* __restrict__ vin = v + (cur ? v_alt : 0) + pr.v_off;
        T* __restrict__ vout = v + (cur ? 0 : v_alt) + pr.v_off;
        for (int base = 0; base < nf; base += NT * FPT) {
            T yr[FPT][M], yi[FPT][M], a1[FPT], a2[FPT];
#pragma unroll
            for (int k = 0; k < FPT; ++k) {
                const int n = base + k * NT + tid;
                const bool ok = n < nf;
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    T2 val;
                    if (ok) val = yb[(int64_t)m * npad + n];
                    else { val.x = T(0); val.y = T(0); }
                    yr[k][m] = val.x;
                    yi[k][m] = val.y;
                }
                a1[k] = ok ? vin[n] : T(1);
                a2[k] = ok ? vin[pr.v2_off + n] : T(1);
            }
#pragma unroll
            for (int k = 0; k < FPT; ++k) {
                const int n = base + k * NT + tid;
                const bool ok = n < nf;
                T n1 = a1[k], n2 = a2[k];
                em_bin<M, T>(yr[k], yi[k], a1[k], a2[k], lm, sh.Pt, ok, acc, llacc, n1, n2, bad);
                if (ok && write_v) {
                    vout[n] = n1;
                    vout[pr.v2_off + n] = n2;
                }
            }
        }
        if (em_finish<M, T>(sh, acc, llacc, bad, it, iters, frozen_at_entry, nf, ll, ll_stride, pid, eps2, tid))
            break;
        cur ^= 1;
    }

    if (write_v) {
        if (cur) {
            for (int n = tid; n < nf; n += NT) {
                v[pr.v_off + n] = v[v_alt + pr.v_off + n];
                v[pr.v_off + pr.v2_off + n] = v[v_alt + pr.v_off + pr.v2_off + n];
            }
        }
        em_store_state(sh, Pg, lamg, logdetg, flagsg, pid, tid);
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
                         int iters, hipStream_t s) {
    using T2 = typename Vec2<T>::type;
    const double eps2 = sizeof(T) == 8 ? kEps2Fp64 : kEps2Fp32Bulk;
    const dim3 grid(count), block(NT);
    const T2* yy = static_cast<const T2*>(y);
    T* vv = static_cast<T*>(v);
    switch (fpt) {
        case 0:
            if constexpr (NT == kEmThreads) {
                em_stream_kernel<M, T, kStreamFramesPerThread, NT><<<grid, block, 0, s>>>(
                    probs, yy, vv, v_alt, P, lam, logdet, flags, ll, ll_stride, iters, eps2);
                break;
            } else {
                return hipErrorInvalidValue;  // streamed problems run with kEmThreads threads only
            }
        case 1: em_kernel<M, T, 1, NT><<<grid, block, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, ll_stride, iters, eps2); break;
        case 2: em_kernel<M, T, 2, NT><<<grid, block, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, ll_stride, iters, eps2); break;
        case 4: em_kernel<M, T, 4, NT><<<grid, block, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, ll_stride, iters, eps2); break;
        case 8: em_kernel<M, T, 8, NT><<<grid, block, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, ll_stride, iters, eps2); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NT>
hipError_t launch_em_nt(int M, bool fp64, int fpt, const EmProblem* probs, int count, const void* y, void* v,
                        int64_t v_alt, double2* P, double* lam, double* logdet, int* flags, double* ll,
                        int64_t ll_stride, int iters, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    switch (M) {
#define FCA_EM_CASE(MM_)                                                                                      \
    case MM_:                                                                                                  \
        return fp64 ? launch_em_fpt<MM_, double, NT>(fpt, probs, count, y, v, v_alt, P, lam, logdet, flags, ll, \
                                                     ll_stride, iters, s)                                      \
                    : launch_em_fpt<MM_, float, NT>(fpt, probs, count, y, v, v_alt, P, lam, logdet, flags, ll,  \
                                                    ll_stride, iters, s);
        FCA_EM_CASE(1) FCA_EM_CASE(2) FCA_EM_CASE(3) FCA_EM_CASE(4)
        FCA_EM_CASE(5) FCA_EM_CASE(6) FCA_EM_CASE(7) FCA_EM_CASE(8)
#undef FCA_EM_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fca
