// fca_device.h -- device helpers of the FastFCA library (gfx950 only).
//
// Complex arithmetic on double2, per-precision fast math for the per-bin
// E/M-step, and the FP64 generalized eigendecomposition of a Hermitian-
// definite pencil used once per frequency and iteration (Section 3, eqs.
// GEVDeff5 / updatePeff / updateLambdaeff; existence by the Appendix
// theorem).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fca_internal.h"

namespace fca {

constexpr int kJacobiMaxSweeps = 16;

// ---------------------------------------------------------------- complex FP64
__host__ __device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__host__ __device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// a * b
__host__ __device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__host__ __device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y));
}
// acc + a * b
__host__ __device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc) {
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}
// acc + a * conj(b)
__host__ __device__ __forceinline__ double2 cfmac(double2 a, double2 b, double2 acc) {
    return make_double2(fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.y, b.x, fma(-a.x, b.y, acc.y)));
}
__host__ __device__ __forceinline__ double cabs2(double2 a) { return fma(a.x, a.x, a.y * a.y); }
__host__ __device__ __forceinline__ bool cfinite(double2 a) { return __builtin_isfinite(a.x) && __builtin_isfinite(a.y); }

// ---------------------------------------------------------------- per-precision math
// Reciprocal, reciprocal square root and natural log used by the per-bin
// arithmetic. float: the hardware approximations (about 1 ulp), adequate for
// the float bulk mode. double: Newton-refined hardware reciprocal (full
// precision for normal inputs), libm-accurate rsqrt and log.
template <typename T> struct Math;

template <> struct Math<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float log(float x) { return __logf(x); }
};

template <> struct Math<double> {
    static __device__ __forceinline__ double rcp(double x) {
        double r = __builtin_amdgcn_rcp(x);
        double e = fma(-x, r, 1.0);
        r = fma(r, e, r);
        e = fma(-x, r, 1.0);
        return fma(r, e, r);
    }
    static __device__ __forceinline__ double rsqrt(double x) { return 1.0 / sqrt(x); }
    static __device__ __forceinline__ double log(double x) { return ::log(x); }
};

// ---------------------------------------------------------------- GEVD (FP64)
// Generalized eigendecomposition of the pencil (A, B), A Hermitian, B
// Hermitian positive definite, folded into a basis update: on return
// Pnew = Pold * Q with Q^H B Q = I and Q^H A Q = diag(lam), and
// *dlogdet = -log det B (= log |det Q|^2). One thread; every array index is a
// compile-time constant after unrolling so the working matrices live in
// registers. A, B and Pold are full M x M row-major (Hermitian inputs: the
// upper triangle is used). Returns FCA flag bits (0 on success).
//
// Method: B = L L^H (Cholesky); C = L^-1 A L^-H; cyclic complex Jacobi
// rotations diagonalise C = W diag(lam) W^H and are applied to the columns
// of V = Pold L^-H, so V ends as Pold L^-H W = Pold Q. (The Appendix proof
// whitens with the eigendecomposition of B instead; any factor of B gives
// the same pencil eigenvalues and a valid Q.)
template <int M>
__host__ __device__ int gevd_update(const double2* __restrict__ A, const double2* __restrict__ B,
                           const double2* __restrict__ Pold, double2* __restrict__ Pnew,
                           double* __restrict__ lam, double* __restrict__ dlogdet, int* sweeps_used) {
    // ---- Cholesky B = L L^H; W = L^-1 (both lower triangular)
    double2 L[M][M];
    double pivprod = 1.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double d = B[j * M + j].x;
#pragma unroll
        for (int k = 0; k < j; ++k) d -= cabs2(L[j][k]);
        if (!(d > 0.0) || !__builtin_isfinite(d)) return kFlagNotPD;
        pivprod *= d;
        const double ljj = sqrt(d);
        const double inv = 1.0 / ljj;
        L[j][j] = make_double2(ljj, 0.0);
#pragma unroll
        for (int i = j + 1; i < M; ++i) {
            // B is Hermitian: B[i][j] = conj(B[j][i]) from the upper triangle
            double2 s = cconj(B[j * M + i]);
#pragma unroll
            for (int k = 0; k < j; ++k) s = csub(s, cmulc(L[i][k], L[j][k]));
            L[i][j] = cscale(inv, s);
        }
    }
    double2 W[M][M];
#pragma unroll
    for (int j = 0; j < M; ++j) W[j][j] = make_double2(1.0 / L[j][j].x, 0.0);
#pragma unroll
    for (int j = 0; j < M; ++j) {
#pragma unroll
        for (int i = j + 1; i < M; ++i) {
            double2 s = make_double2(0.0, 0.0);
#pragma unroll
            for (int k = j; k < i; ++k) s = cfma(L[i][k], W[k][j], s);
            W[i][j] = cscale(-W[i][i].x, s);
        }
    }
    // log det B = log prod_j L_jj^2; fall back to a sum of logs on range trouble
    double ld;
    if (pivprod > 1e-300 && pivprod < 1e300) {
        ld = ::log(pivprod);
    } else {
        ld = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) ld += 2.0 * ::log(L[j][j].x);
    }
    *dlogdet = -ld;

    // ---- C = W A W^H (Hermitian; upper triangle kept, diagonal real)
    double2 T[M][M];  // T = W A
#pragma unroll
    for (int i = 0; i < M; ++i) {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            double2 s = make_double2(0.0, 0.0);
#pragma unroll
            for (int a = 0; a <= i; ++a) {
                const double2 Aak = (a <= k) ? A[a * M + k] : cconj(A[k * M + a]);
                s = cfma(W[i][a], (a == k) ? make_double2(Aak.x, 0.0) : Aak, s);
            }
            T[i][k] = s;
        }
    }
    double2 C[M][M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
#pragma unroll
        for (int k = i; k < M; ++k) {
            double2 s = make_double2(0.0, 0.0);
#pragma unroll
            for (int b = 0; b <= k; ++b) s = cfmac(T[i][b], W[k][b], s);
            C[i][k] = s;
        }
        C[i][i].y = 0.0;
    }
    // ---- V = Pold W^H
    double2 V[M][M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            double2 s = make_double2(0.0, 0.0);
#pragma unroll
            for (int b = 0; b <= k; ++b) s = cfmac(Pold[i * M + b], W[k][b], s);
            V[i][k] = s;
        }
    }

    // ---- cyclic Jacobi on C (upper triangle), rotations applied to V.
    // Rotation of the (p,q) plane: G_pp = G_qq = c, G_pq = s e, G_qp = -s conj(e)
    // with e = C_pq / |C_pq|, t = s / c = sign(tau) / (|tau| + sqrt(1 + tau^2)),
    // tau = (C_qq - C_pp) / (2 |C_pq|). Then (G^H C G)_pq = 0,
    // C_pp -= t |C_pq|, C_qq += t |C_pq|. A rotation is skipped when
    // |C_pq|^2 <= eps^2 |C_pp C_qq| (relative threshold, eps = 1e-15).
    int flag = 0;
    int sweep = 0;
    for (; sweep < kJacobiMaxSweeps; ++sweep) {
        bool rotated = false;
#pragma unroll
        for (int p = 0; p < M - 1; ++p) {
#pragma unroll
            for (int q = p + 1; q < M; ++q) {
                const double2 h = C[p][q];
                const double hh = cabs2(h);
                const double a = C[p][p].x, b = C[q][q].x;
                if (hh > 1e-30 * fabs(a * b) && hh > 1e-300) {
                    rotated = true;
                    const double habs = sqrt(hh);
                    const double rh = 1.0 / habs;
                    const double tau = 0.5 * (b - a) * rh;
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(fma(tau, tau, 1.0)));
                    const double c = 1.0 / sqrt(fma(t, t, 1.0));
                    const double s = t * c;
                    const double2 e = cscale(rh, h);
                    const double2 se = cscale(s, e);           // s e
                    const double2 sec = cconj(se);             // s conj(e)
                    C[p][p].x = a - t * habs;
                    C[q][q].x = b + t * habs;
                    C[p][q] = make_double2(0.0, 0.0);
#pragma unroll
                    for (int k = 0; k < M; ++k) {
                        if (k == p || k == q) continue;
                        // column entries C_kp, C_kq from the stored upper triangle
                        const double2 ckp = (k < p) ? C[k][p] : cconj(C[p][k]);
                        const double2 ckq = (k < q) ? C[k][q] : cconj(C[q][k]);
                        const double2 nkp = csub(cscale(c, ckp), cmul(sec, ckq));
                        const double2 nkq = cadd(cmul(se, ckp), cscale(c, ckq));
                        if (k < p) C[k][p] = nkp; else C[p][k] = cconj(nkp);
                        if (k < q) C[k][q] = nkq; else C[q][k] = cconj(nkq);
                    }
#pragma unroll
                    for (int i = 0; i < M; ++i) {
                        const double2 vp = V[i][p], vq = V[i][q];
                        V[i][p] = csub(cscale(c, vp), cmul(sec, vq));
                        V[i][q] = cadd(cmul(se, vp), cscale(c, vq));
                    }
                }
            }
        }
        if (!rotated) break;
    }
    if (sweep == kJacobiMaxSweeps) flag |= kFlagSweeps;
    *sweeps_used = sweep;

    bool finite = true;
#pragma unroll
    for (int i = 0; i < M; ++i) {
        lam[i] = C[i][i].x;
        finite = finite && __builtin_isfinite(lam[i]);
#pragma unroll
        for (int k = 0; k < M; ++k) {
            Pnew[i * M + k] = V[i][k];
            finite = finite && cfinite(V[i][k]);
        }
    }
    if (!finite || !__builtin_isfinite(*dlogdet)) flag |= kFlagNonFinite;
    return flag;
}

}  // namespace fca
