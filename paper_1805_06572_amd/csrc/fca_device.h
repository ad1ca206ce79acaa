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

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

constexpr double kLogPi = 1.1447298858494002;

template <typename T> __device__ __forceinline__ typename Vec2<T>::type make_vec2(T x, T y) {
    typename Vec2<T>::type r;
    r.x = x;
    r.y = y;
    return r;
}

// Index of the off-diagonal pair (i < k) of an M x M matrix, row-major over
// the strict upper triangle.
__host__ __device__ constexpr int pair_index(int M, int i, int k) {
    return i * M - i * (i + 1) / 2 + (k - i - 1);
}

// ---------------------------------------------------------------- inverse of P
// Gauss-Jordan elimination with partial pivoting, FP64. Returns false if P is
// numerically singular.
template <int M>
__device__ bool invert(const double2* __restrict__ P, double2 (&X)[M][M]) {
    double2 A[M][M];
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
        for (int k = 0; k < M; ++k) {
            A[i][k] = P[i * M + k];
            X[i][k] = make_double2(i == k ? 1.0 : 0.0, 0.0);
        }
    bool ok = true;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        // pivot search among rows c..M-1 (swap by value, indices stay static)
        double best = cabs2(A[c][c]);
#pragma unroll
        for (int r = c + 1; r < M; ++r) {
            const double mag = cabs2(A[r][c]);
            if (mag > best) {
                best = mag;
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    const double2 ta = A[c][k]; A[c][k] = A[r][k]; A[r][k] = ta;
                    const double2 tx = X[c][k]; X[c][k] = X[r][k]; X[r][k] = tx;
                }
            }
        }
        if (!(best > 0.0)) ok = false;
        const double2 piv = A[c][c];
        const double inv_mag = 1.0 / cabs2(piv);
        const double2 pinv = make_double2(piv.x * inv_mag, -piv.y * inv_mag);
#pragma unroll
        for (int k = 0; k < M; ++k) {
            A[c][k] = cmul(A[c][k], pinv);
            X[c][k] = cmul(X[c][k], pinv);
        }
#pragma unroll
        for (int r = 0; r < M; ++r) {
            if (r == c) continue;
            const double2 fct = A[r][c];
#pragma unroll
            for (int k = 0; k < M; ++k) {
                A[r][k] = csub(A[r][k], cmul(fct, A[c][k]));
                X[r][k] = csub(X[r][k], cmul(fct, X[c][k]));
            }
        }
    }
    return ok;
}

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

// Orders the LDS accesses of one wavefront: a wave executes its LDS
// instructions in issue order, so after this point every lane sees what the
// other lanes of the same wave stored before it. Also a compiler barrier.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroup sums of the per-thread accumulators (FP64 across threads, fixed
// order) into S~_j = sums / N as full Hermitian matrices in sh.S, and of the
// per-thread log-likelihood terms: per wave into sh.LL, or (DeferLL) stored
// per thread in sh.llp for a later fixed-order sum off this path. The
// accumulator layout per source j (offset j M^2): diagonal i at i, the
// off-diagonal pair (i < k) at M + 2 pair_index(M, i, k) (+1 imaginary).
// NS sources (2 unless given); with lam != NULL the sums of every source
// j < NS - 1 are scaled to entry (i, k) times lam_j[i] lam_j[k] (off the
// diagonal) or lam_j[i] (on it), lam_j = lam + j lam_stride.
// Each wave first sums its own 64 rows (no workgroup barrier: a wave starts
// as soon as its own frames are done), in chunks of CH values: lane (h, c)
// adds rows h, h + H, ... of column c (H = 64 / CH lanes per column, four
// interleaved partial sums); unless there is one chunk with H <= 4, the H
// partials of a column are then added per wave. One workgroup barrier, then wave 0 adds the
// per-wave sums (in wave order) and writes S: on return sh.S (and sh.LL) are
// complete for wave 0 only (the caller's next workgroup barrier publishes
// them).
// Sh provides red, wh, wp, LL (or llp), S and the constants CH, NCH,
// NV, NW.
template <int M, int NS = 2, bool DeferLL = false, typename Sh, typename T>
__device__ __forceinline__ void wg_reduce_sums(Sh& sh, const T (&acc)[NS * M * M], double llacc, int nf, int tid,
                                               const double* lam, int lam_stride = 0) {
    constexpr int MM = M * M, NV = Sh::NV, CH = Sh::CH, NCH = Sh::NCH, NW = Sh::NW;
    constexpr int H = 64 / CH;
    // one chunk with few partials per column: wave 0 adds them directly
    constexpr bool kDirect = NCH == 1 && H <= 4;
    const int lane = tid & 63, w = tid >> 6;
    if constexpr (DeferLL) {
        sh.llp[tid] = llacc;
    } else {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) llacc += __shfl_xor(llacc, off, 64);
        if (lane == 0) sh.LL[w] = llacc;
    }
    T* __restrict__ red = sh.red + w * 64 * (CH + 1);
    const int c = lane % CH, h = lane / CH;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
#pragma unroll
        for (int q = 0; q < CH; ++q)
            if (ch * CH + q < NV) red[lane * (CH + 1) + q] = acc[ch * CH + q];
        wave_lds_sync();
        if (h < H) {
            double p[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k * H < 64; ++k) {
                const int r = h + k * H;
                if (r < 64) p[k & 3] += (double)red[r * (CH + 1) + c];
            }
            sh.wh[w][h * CH + c] = (p[0] + p[1]) + (p[2] + p[3]);
        }
        if constexpr (!kDirect) {
            wave_lds_sync();
            if (lane < CH && ch * CH + lane < NV) {
                double sum = 0.0;
#pragma unroll
                for (int hh = 0; hh < H; ++hh) sum += sh.wh[w][hh * CH + lane];
                sh.wp[w][ch * CH + lane] = sum;
            }
            wave_lds_sync();
        }
    }
    __syncthreads();
    if (w != 0) return;
    // the workgroup total of accumulator e: per wave the H partials (one
    // chunk) or the per-wave sum, added in wave order
    auto total = [&](int e) {
        double sum = 0.0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            if constexpr (kDirect) {
                double part = 0.0;
#pragma unroll
                for (int hh = 0; hh < H; ++hh) part += sh.wh[ww][hh * CH + e];
                sum += part;
            } else {
                sum += sh.wp[ww][e];
            }
        }
        return sum;
    };
    for (int t = lane; t < NV; t += 64) {
        const int j = t / MM, ent = t % MM, i = ent / M, q = ent % M;
        double sc = 1.0 / (double)nf;
        if (lam && j < NS - 1) {
            const double* lj = lam + j * lam_stride;
            sc *= (i == q) ? lj[i] : lj[i] * lj[q];
        }
        double2 val;
        if (i == q) {
            val = make_double2(total(j * MM + i) * sc, 0.0);
        } else {
            const int o = j * MM + M + 2 * pair_index(M, i < q ? i : q, i < q ? q : i);
            const double re = total(o) * sc, im = total(o + 1) * sc;
            val = make_double2(re, i < q ? im : -im);
        }
        sh.S[j][ent] = val;
    }
    wave_lds_sync();
}

// ---------------------------------------------------------------- FP64 helpers
// Hardware reciprocal / reciprocal square root refined by two Newton steps
// (full double precision for normal positive inputs).
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
    double r = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x;
    r = r * fma(-h * r, r, 1.5);
    return r * fma(-h * r, r, 1.5);
}
// One Newton step only: for quantities whose rounding does not matter beyond
// single precision (a Jacobi rotation angle may be slightly off; only its
// cosine/sine pair must be exactly consistent).
__device__ __forceinline__ double rcp_nr1(double x) {
    double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsqrt_nr1(double x) {
    double r = __builtin_amdgcn_rsq(x);
    return r * fma(-0.5 * x * r, r, 1.5);
}

// ---------------------------------------------------------------- GEVD (FP64)
// Working storage of one wave-parallel eigendecomposition (in LDS).
struct GevdScratch {
    double2 W[kMaxM * kMaxM];   // L^-1 (row-major, stride M)
    double2 T[kMaxM * kMaxM];   // L^-1 A (stride MP)
    double2 C[kMaxM * kMaxM];   // working Hermitian matrix (stride MP)
    double2 V[kMaxM * kMaxM];   // accumulated basis (stride MP)
    double4 prm[kMaxM];         // rotation of the pair containing index k: (c, g.re, g.im, t|h|)
};

template <int M> struct GevdShape {
    static constexpr int MP = M <= 1 ? 1 : M <= 2 ? 2 : M <= 4 ? 4 : 8;  // padded order
    static constexpr int LG = MP == 1 ? 0 : MP == 2 ? 1 : MP == 4 ? 2 : 3;
};

// sum_j log d_j of positive pivots: one log of the product unless it leaves
// the range where the product is exact enough.
template <int M>
__device__ __forceinline__ double log_pivots(const double (&d)[M]) {
    double prod = 1.0;
#pragma unroll
    for (int j = 0; j < M; ++j) prod *= d[j];
    if (prod > 1e-300 && prod < 1e300) return ::log(prod);
    double ld = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) ld += ::log(d[j]);
    return ld;
}

struct PairRot {
    double cc, th;
    double2 g;
    bool rot;
};
// Jacobi rotation of one pair (p, q), p < q, of a Hermitian matrix from
// C_pp = a, C_qq = b, C_pq = h (formulas at gevd_wave): skipped (identity)
// when |h|^2 <= eps2 |a b|. FastAngle: the angle in float (t = sign(d) /
// (u + sqrt(u^2 + 1)), u = |d| / (2|h|)); the cosine/sine pair stays
// consistent in double through the double rsqrt. Otherwise
// t = sign(d) 2|h| / (|d| + sqrt(d^2 + 4|h|^2)), d = b - a (no overflow,
// no division by |h|).
template <bool FastAngle>
__device__ __forceinline__ PairRot pair_rotation(double a, double b, double2 h, double eps2) {
    PairRot r{1.0, 0.0, make_double2(0.0, 0.0), false};
    const double hh = cabs2(h);
    r.rot = hh > eps2 * fabs(a * b) && hh > 1e-300;
    if (r.rot) {
        const double rh = rsqrt_nr(hh);
        const double habs = hh * rh;
        const double d = b - a;
        double t;
        if constexpr (FastAngle) {
            const float u = (float)fmin(fabs(d) * 0.5 * rh, 1e18);
            const float tf = __builtin_amdgcn_rcpf(u + __builtin_amdgcn_sqrtf(fmaf(u, u, 1.0f)));
            t = copysign((double)tf, d);
        } else {
            const double w2 = fma(d, d, 4.0 * hh);
            const double root = w2 * rsqrt_nr1(w2);
            t = copysign(2.0 * habs * rcp_nr1(fabs(d) + root), d);
        }
        r.cc = rsqrt_nr(fma(t, t, 1.0));
        const double sn = t * r.cc * rh;
        r.g = make_double2(sn * h.x, sn * h.y);
        r.th = t * habs;
    }
    return r;
}

// Generalized eigendecomposition of the Hermitian-definite pencil (A, B),
// folded into a basis update: Pnew = Pold Q with Q^H B Q = I and
// Q^H A Q = diag(lam); *dlogdet = -log det B = log|det Q|^2. This is the
// per-frequency step of the FastFCA iteration (eqs. GEVDeff5, updatePeff,
// updateLambdaeff); the Appendix theorem guarantees Q exists when B is
// positive definite.
//
// Called by all 64 lanes of ONE wavefront (uniform control flow). A, B, Pold
// are full M x M row-major in LDS (Hermitian inputs; the upper triangle of B
// is what the factorisation reads). Pnew and lam may be LDS or global.
// Returns FCA flag bits (0 on success); when a freezing flag is returned
// nothing is written. FastAngle computes each rotation angle in float (the
// rotation itself, its cosine/sine pair and its application stay in double):
// for the float bulk mode, where the angle's float accuracy is below the
// per-bin arithmetic's. PnewT and lamT (optional) receive Pnew and lam in
// the bulk precision Tb as well. Pnew may alias Pold (Pold is read before
// any output is written). With piv (optional, M doubles) the Cholesky pivots
// d_j (log det B = sum_j log d_j) are written there instead of computing
// *dlogdet, so that the caller can take the logarithm off this wave.
//
// Method: B = L L^H by Cholesky (computed redundantly by every lane, so it is
// uniform), W = L^-1; lane (i,k) of the MP x MP grid (M padded to a power of
// two with zero rows/columns) then holds C_ik of C = W A W^H and V_ik of
// V = Pold W^H. Jacobi rounds x = 1..MP-1 pair every index k with k XOR x;
// the MP/2 disjoint rotations of a round are applied together, so each
// sweep rotates every pair once. The rotation of (p,q), p < q, is
// G_pp = G_qq = c, G_pq = g = s e, G_qp = -conj(g), e = C_pq/|C_pq|,
// t = s/c = sign(tau)/(|tau| + sqrt(1+tau^2)), tau = (C_qq - C_pp)/(2|C_pq|):
// it zeroes C_pq and moves C_pp -= t|C_pq|, C_qq += t|C_pq|. Rotations are
// skipped when |C_pq|^2 <= eps2 |C_pp C_qq|, and sweeps stop once every
// off-diagonal entry passes that test. At the end C = diag(lam), V = Pold Q.
// (The Appendix proof whitens B by its eigendecomposition; a Cholesky factor
// gives the same eigenvalues and an equally valid Q.)
template <int M, bool FastAngle = false, typename Tb = double>
__device__ int gevd_wave(const double2* A, const double2* B, const double2* Pold, GevdScratch& ws,
                         double2* Pnew, double* lam, double* dlogdet, double eps2,
                         typename Vec2<Tb>::type* PnewT = nullptr, Tb* lamT = nullptr,
                         double* piv = nullptr) {
    constexpr int MP = GevdShape<M>::MP;
    constexpr int LG = GevdShape<M>::LG;
    const int lane = threadIdx.x & 63;
    const int i = lane >> LG, k = lane & (MP - 1);
    const bool act = lane < MP * MP;
    const bool in = act && i < M && k < M;

    // ---- Cholesky B = L L^H and W = L^-1, uniform across lanes
    double2 L[M][M];
    double pv[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double d = B[j * M + j].x;
#pragma unroll
        for (int q = 0; q < j; ++q) d -= cabs2(L[j][q]);
        if (!(d > 0.0) || !__builtin_isfinite(d)) return kFlagNotPD;
        pv[j] = d;
        const double inv = rsqrt_nr(d);
        L[j][j] = make_double2(d * inv, 0.0);
#pragma unroll
        for (int r = j + 1; r < M; ++r) {
            double2 s = cconj(B[j * M + r]);
#pragma unroll
            for (int q = 0; q < j; ++q) s = csub(s, cmulc(L[r][q], L[j][q]));
            L[r][j] = cscale(inv, s);
        }
    }
    // log det B = sum_j log d_j; with piv the pivots d_j go to the caller
    // instead (lane 0 writes them) and *dlogdet is left alone
    double ld = 0.0;
    if (piv) {
        if (lane == 0)
#pragma unroll
            for (int j = 0; j < M; ++j) piv[j] = pv[j];
    } else {
        ld = log_pivots<M>(pv);
    }
    if (lane == 0) {
        double2 Wr[M][M];
#pragma unroll
        for (int j = 0; j < M; ++j) Wr[j][j] = make_double2(rcp_nr(L[j][j].x), 0.0);
#pragma unroll
        for (int j = 0; j < M; ++j) {
#pragma unroll
            for (int r = j + 1; r < M; ++r) {
                double2 s = make_double2(0.0, 0.0);
#pragma unroll
                for (int q = j; q < r; ++q) s = cfma(L[r][q], Wr[q][j], s);
                Wr[r][j] = cscale(-Wr[r][r].x, s);
            }
        }
#pragma unroll
        for (int r = 0; r < M; ++r)
#pragma unroll
            for (int j = 0; j <= r; ++j) ws.W[r * M + j] = Wr[r][j];
    }
    wave_lds_sync();

    // ---- T = W A (row i of lane), then C = T W^H and V = Pold W^H
    if (in) {
        double2 t = make_double2(0.0, 0.0);
#pragma unroll
        for (int a = 0; a < M; ++a)
            if (a <= i) t = cfma(ws.W[i * M + a], A[a * M + k], t);
        ws.T[i * MP + k] = t;
    }
    wave_lds_sync();
    double2 c = make_double2(0.0, 0.0), v = make_double2(0.0, 0.0);
    if (in) {
#pragma unroll
        for (int b = 0; b < M; ++b) {
            if (b <= k) {
                const double2 w = ws.W[k * M + b];
                c = cfmac(ws.T[i * MP + b], w, c);
                v = cfmac(Pold[i * M + b], w, v);
            }
        }
        if (i == k) c.y = 0.0;
    }

    // ---- Jacobi sweeps
    int flag = 0;
    int sweep = 0;
    for (;; ++sweep) {
        // convergence test on the current matrix (before the first sweep the
        // matrix is essentially never diagonal: that sweep always runs, and
        // its rounds skip the rotations that are not needed)
        if (sweep > 0) {
            if (act) ws.C[lane] = c;
            wave_lds_sync();
            bool open = false;
            if (in && i < k) {
                const double a = ws.C[i * MP + i].x, b = ws.C[k * MP + k].x;
                const double hh = cabs2(c);
                open = hh > eps2 * fabs(a * b) && hh > 1e-300;
            }
            if (!__any(open)) break;
            if (sweep == kJacobiMaxSweeps) {
                flag |= kFlagSweeps;
                break;
            }
        }
#pragma unroll 1
        for (int x = 1; x < MP; ++x) {
            const int k2 = k ^ x, i2 = i ^ x;
            if (act) {
                ws.C[lane] = c;
                ws.V[lane] = v;
            }
            wave_lds_sync();
            PairRot r{1.0, 0.0, make_double2(0.0, 0.0), false};
            double2 cik2 = c, ci2k = c, ci2k2 = c, vik2 = v;
            if (act) {
                const int p = k < k2 ? k : k2, q = k ^ k2 ^ p;
                r = pair_rotation<FastAngle>(ws.C[p * MP + p].x, ws.C[q * MP + q].x, ws.C[p * MP + q], eps2);
                cik2 = ws.C[i * MP + k2];
                ci2k = ws.C[i2 * MP + k];
                ci2k2 = ws.C[i2 * MP + k2];
                vik2 = ws.V[i * MP + k2];
                if (i == 0) ws.prm[k] = make_double4(r.cc, r.g.x, r.g.y, r.th);
            }
            if (!__any(r.rot)) continue;   // no pair of this round rotates: C and V stay
            wave_lds_sync();
            if (act) {
                const double4 pr = ws.prm[i];   // the rotation of the pair containing i
                // column factor G_{k2,k} and conjugated row factor conj(G_{i2,i})
                const double cc = r.cc, th = r.th;
                const double2 gk = (k < k2) ? make_double2(-r.g.x, r.g.y) : r.g;
                const double2 gi = (i < i2) ? make_double2(-pr.y, -pr.z) : make_double2(pr.y, -pr.z);
                const double ci = pr.x;
                double2 cn = cadd(cscale(ci, cadd(cscale(cc, c), cmul(gk, cik2))),
                                  cmul(gi, cadd(cscale(cc, ci2k), cmul(gk, ci2k2))));
                if (k == i) cn = make_double2(c.x + ((i < i2) ? -th : th), 0.0);
                else if (k == i2 && th != 0.0) cn = make_double2(0.0, 0.0);
                v = cadd(cscale(cc, v), cmul(gk, vik2));
                c = cn;
            }
        }
    }

    bool finite = !in || (cfinite(v) && (i != k || __builtin_isfinite(c.x)));
    if (!__all(finite) || !__builtin_isfinite(ld)) flag |= kFlagNonFinite;
    if (in && !(flag & kFreezeMask)) {
        Pnew[i * M + k] = v;
        if (i == k) lam[i] = c.x;
        if (PnewT) PnewT[i * M + k] = make_vec2<Tb>((Tb)v.x, (Tb)v.y);
        if (lamT && i == k) lamT[i] = (Tb)c.x;
    }
    if (!piv) *dlogdet = -ld;
    return flag;
}

}  // namespace fca
