// fca_multi.hip -- the EM for J >= 2 sources by approximate joint
// diagonalisation (the extension the paper leaves as future work).
//
// Parameters per frequency: S_j = P^-H Lambda_j P^-1 with one basis P,
// Lambda_j diagonal, Lambda_J = I. Per bin, in the basis (exact for
// parameters of that form; for J = 2 Algorithm 1, steps 3-7):
//   y~ = P^H y, d_i = sum_j v_j lam_ji, r_i = 1 / d_i,
//   t_ji = r_i (v_j lam_ji e_i r_i + d_i - v_j lam_ji)  (e_i = |y~_i|^2),
//   v_j' = (v_j / M) sum_i t_ji,
//   S~_j: off the diagonal lam_ji lam_jk (v_j^2 / v_j') z_i conj(z_k)
//         with z = r y~; on it lam_ji (v_j / v_j') t_ji; summed over the
//         frames and divided by N,
//   log-likelihood -M log pi + log|det P|^2 - sum_i log d_i - sum_i e_i r_i.
// Per frequency (the approximate step): whiten by S~_J (Cholesky L, W =
// L^-1), C_j = W S~_j W^H (j < J), unitary Jacobi joint diagonalisation of
// the C_j with the Cardoso-Souloumiac angle of each pair (dominant
// eigenvector of G = sum_j h_j h_j^T, h_j = (C_pp - C_qq, 2 Re C_pq,
// -2 Im C_pq)), rounds of disjoint pairs (k, k XOR x); then P <- P W^H U,
// lam_ji = (U^H C_j U)_ii, log|det P|^2 -= log det S~_J. The off-diagonal
// remainder of U^H C_j U is dropped; for J = 2 there is none.
//
// One workgroup per frequency for all iterations of a call, frames in
// registers (N <= 2048), M <= 4 microphones, J <= 4 sources; the joint
// diagonalisation runs in FP64 on one wavefront (16 lanes: entry (i, k)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

#include "fca.h"
#include "fca_device.h"
#include "fca_internal.h"

namespace fca {
namespace {

constexpr int kMJ = 4;        // largest number of sources
constexpr int kMM = 4;        // largest number of microphones
constexpr int kMS = kMM * kMM;
constexpr int kMThreads = 256;
constexpr int kMRows = 128;   // iterations per launch (log-likelihood rows)
constexpr int kAjdMaxSweeps = 16;

// ---------------------------------------------------------------- dominant eigenvector of a 3x3
// Unit eigenvector (x, y, z), x >= 0, of the largest eigenvalue of the
// symmetric G = [[g0, g1, g2], [g1, g3, g4], [g2, g4, g5]] (the largest
// root of the characteristic cubic by monotone Newton steps, then the
// longest cross product of two rows of G - lambda I). False when no
// direction dominates (G a multiple of the identity, zero included, or a
// repeated largest eigenvalue).
__device__ bool dominant_eig3(const double (&g)[6], double& x, double& y, double& z) {
    const double m = (g[0] + g[3] + g[5]) * (1.0 / 3.0);
    const double a = g[0] - m, b = g[3] - m, c = g[5] - m;
    const double off = g[1] * g[1] + g[2] * g[2] + g[4] * g[4];
    const double p2 = a * a + b * b + c * c + 2.0 * off;
    const double scale = fabs(g[0]) + fabs(g[3]) + fabs(g[5]);
    if (!(p2 > 1e-28 * scale * scale) || !(scale > 1e-300)) return false;
    // the largest eigenvalue by Newton's method on the characteristic polynomial of the
    // shifted matrix B = G - m I, q(t) = det(t I - B) = t^3 - k1 t - k0 (trace 0), from an
    // upper bound of its largest root (the largest Gershgorin row sum): right of that root
    // q is increasing and convex, so the iterates decrease monotonically onto it
    const double k1 = 0.5 * p2;                        // sum of the squared entries / 2
    const double k0 = a * (b * c - g[4] * g[4]) - g[1] * (g[1] * c - g[4] * g[2]) + g[2] * (g[1] * g[4] - b * g[2]);
    double t = fmax(fabs(a) + fabs(g[1]) + fabs(g[2]), fmax(fabs(g[1]) + fabs(b) + fabs(g[4]), fabs(g[2]) + fabs(g[4]) + fabs(c)));
    for (int it = 0; it < 48; ++it) {
        const double q = (t * t - k1) * t - k0;
        const double dq = 3.0 * t * t - k1;
        if (!(q > 0.0) || !(dq > 0.0)) break;
        const double step = q * rcp_nr(dq);            // the step's rounding does not move the root
        t -= step;
        if (step <= 2e-16 * t) break;
    }
    const double lam = m + t;
    const double r0[3] = {g[0] - lam, g[1], g[2]}, r1[3] = {g[1], g[3] - lam, g[4]}, r2[3] = {g[2], g[4], g[5] - lam};
    double best[3] = {0.0, 0.0, 0.0}, bn = 0.0;
    auto consider = [&](const double (&u)[3], const double (&w)[3]) {
        const double cx = u[1] * w[2] - u[2] * w[1], cy = u[2] * w[0] - u[0] * w[2], cz = u[0] * w[1] - u[1] * w[0];
        const double n2 = cx * cx + cy * cy + cz * cz;
        if (n2 > bn) {
            bn = n2;
            best[0] = cx;
            best[1] = cy;
            best[2] = cz;
        }
    };
    consider(r0, r1);
    consider(r0, r2);
    consider(r1, r2);
    if (!(bn > 1e-28 * scale * scale * scale * scale)) return false;
    const double inv = (best[0] < 0.0 ? -1.0 : 1.0) * rsqrt_nr(bn);
    x = best[0] * inv;
    y = best[1] * inv;
    z = best[2] * inv;
    return true;
}

// ---------------------------------------------------------------- joint diagonalisation (one wave)
struct AjdScratch {
    double2 W[kMS];             // L^-1, stride M
    double2 T[kMJ - 1][kMS];    // W S~_j, stride 4
    double2 C[kMJ - 1][kMS];    // working matrices, stride 4
    double2 V[kMS];             // accumulated basis, stride 4
    double4 prm[kMM];           // rotation of the pair containing index k: (c, s.re, s.im, rotated)
};

// Called by all 64 lanes of one wave. S[j] full Hermitian M x M (stride M)
// for j < J (S[J-1] the whitening reference), Pold (stride M); on success
// writes Pnew (stride M, may alias Pold), lam (J rows of stride kMM; row
// J-1 = 1) and their bulk-precision copies when given; *dlogdet =
// -log det S~_J. Returns FCA flag bits; nothing is written on a freezing
// flag. tol: skip threshold of a pair (relative off-diagonal size, and |s|).
template <int M, int J, typename Tb>
__device__ int ajd_wave(const double2 (*S)[kMS], const double2* Pold, AjdScratch& ws, double2* Pnew, double* lam,
                        typename Vec2<Tb>::type* PnewT, Tb* lamT, double* dlogdet, double tol) {
    constexpr int MP = GevdShape<M>::MP;
    constexpr int LG = GevdShape<M>::LG;
    constexpr int NC = J - 1;
    const int lane = threadIdx.x & 63;
    const int i = lane >> LG, k = lane & (MP - 1);
    const bool act = lane < MP * MP;
    const bool in = act && i < M && k < M;
    const double2* B = S[J - 1];
    // ---- whitening by S~_J: uniform Cholesky, W = L^-1 on lane 0
    double2 L[M][M];
    double pivprod = 1.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double d = B[j * M + j].x;
#pragma unroll
        for (int q = 0; q < j; ++q) d -= cabs2(L[j][q]);
        if (!(d > 0.0) || !__builtin_isfinite(d)) return kFlagNotPD;
        pivprod *= d;
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
    double ld = 0.0;
    if (pivprod > 1e-300 && pivprod < 1e300) {
        ld = ::log(pivprod);
    } else {
#pragma unroll
        for (int j = 0; j < M; ++j) ld += 2.0 * ::log(L[j][j].x);
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
            for (int j = 0; j < M; ++j) ws.W[r * M + j] = j <= r ? Wr[r][j] : make_double2(0.0, 0.0);
    }
    wave_lds_sync();
    // ---- C_j = W S~_j W^H, V = Pold W^H (lane (i, k) holds entry (i, k))
    if (in) {
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            double2 t = make_double2(0.0, 0.0);
#pragma unroll
            for (int a = 0; a < M; ++a) t = cfma(ws.W[i * M + a], S[j][a * M + k], t);
            ws.T[j][i * MP + k] = t;
        }
    }
    wave_lds_sync();
    double2 c[NC], v = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < NC; ++j) c[j] = make_double2(0.0, 0.0);
    if (in) {
#pragma unroll
        for (int b = 0; b < M; ++b) {
            const double2 w = ws.W[k * M + b];
#pragma unroll
            for (int j = 0; j < NC; ++j) c[j] = cfmac(ws.T[j][i * MP + b], w, c[j]);
            v = cfmac(Pold[i * M + b], w, v);
        }
        if (i == k)
#pragma unroll
            for (int j = 0; j < NC; ++j) c[j].y = 0.0;
    }
    // ---- Jacobi sweeps over rounds of disjoint pairs (k, k XOR x)
    int flag = 0;
    const double tol2 = tol * tol;
    int sweep = 0;
    for (; sweep < kAjdMaxSweeps; ++sweep) {
        bool any_sweep = false;
#pragma unroll 1
        for (int x = 1; x < MP; ++x) {
            const int k2 = k ^ x, i2 = i ^ x;
            if (act) {
#pragma unroll
                for (int j = 0; j < NC; ++j) ws.C[j][lane] = c[j];
                ws.V[lane] = v;
            }
            wave_lds_sync();
            const int p = k < k2 ? k : k2, q = k ^ k2 ^ p;
            double cs = 1.0;
            double2 sn = make_double2(0.0, 0.0);
            bool rot = false;
            if (act) {
                double off = 0.0, dia = 0.0, g[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    const double a = ws.C[j][p * MP + p].x, b = ws.C[j][q * MP + q].x;
                    const double2 h = ws.C[j][p * MP + q];
                    off += cabs2(h);
                    dia += fabs(a * b);
                    const double h0 = a - b, h1 = 2.0 * h.x, h2 = -2.0 * h.y;
                    g[0] = fma(h0, h0, g[0]);
                    g[1] = fma(h0, h1, g[1]);
                    g[2] = fma(h0, h2, g[2]);
                    g[3] = fma(h1, h1, g[3]);
                    g[4] = fma(h1, h2, g[4]);
                    g[5] = fma(h2, h2, g[5]);
                }
                // A pair whose rotation is provably below tol is left alone without solving for it:
                // with the residual (0, g1, g2) of e1 as an eigenvector of G and the gap g0 - mu to
                // the rest of the spectrum (mu, the largest eigenvalue of G's lower 2 x 2 block,
                // bounds the others by interlacing), the dominant eigenvector u makes an angle phi
                // with e1 of sin phi <= |(g1, g2)| / (g0 - mu) (Davis-Kahan), and the rotation it
                // gives has |s|^2 = (1 - u0) / 2 <= sin^2 phi / 2. Skipped when that bound is below
                // tol^2 / 8: the eigenvector's own test would skip the pair too.
                const double hb = 0.5 * (g[3] - g[5]);
                const double gap = g[0] - (0.5 * (g[3] + g[5]) + sqrt(hb * hb + g[4] * g[4]));
                const bool tiny = gap > 0.0 && g[1] * g[1] + g[2] * g[2] <= 0.25 * tol2 * gap * gap;
                double ex, ey, ez;
                if (q < M && off > tol2 * dia && off > 1e-300 && !tiny && dominant_eig3(g, ex, ey, ez)) {
                    const double hc = 0.5 * (1.0 + ex), rc = rsqrt_nr(hc);   // hc >= 1/2
                    cs = hc * rc;
                    const double is2c = 0.5 * rc;
                    sn = make_double2(ey * is2c, ez * is2c);
                    rot = cabs2(sn) > tol2;
                    if (!rot) {
                        cs = 1.0;
                        sn = make_double2(0.0, 0.0);
                    }
                }
                if (i == 0) ws.prm[k] = make_double4(cs, sn.x, sn.y, rot ? 1.0 : 0.0);
            }
            if (!__any(rot)) continue;
            any_sweep = true;
            wave_lds_sync();
            if (act) {
                // the partner entries of this round (C and V as written at its start; the next
                // writes come after these reads in this wave's order)
                double2 cik2[NC], ci2k[NC], ci2k2[NC];
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    cik2[j] = ws.C[j][i * MP + k2];
                    ci2k[j] = ws.C[j][i2 * MP + k];
                    ci2k2[j] = ws.C[j][i2 * MP + k2];
                }
                const double2 vik2 = ws.V[i * MP + k2];
                // column factors of this lane's k (pair (k, k2)), row factors of i (pair (i, i2))
                const double2 gam = make_double2(cs, 0.0);
                const double2 del = (k < k2) ? sn : make_double2(-sn.x, sn.y);   // s or -conj(s)
                const double4 pr = ws.prm[i];
                const double2 al = make_double2(pr.x, 0.0);
                const double2 be = (i < i2) ? make_double2(pr.y, -pr.z) : make_double2(-pr.y, -pr.z);  // conj(s) or -s
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    const double2 own = cadd(cmul(gam, c[j]), cmul(del, cik2[j]));
                    const double2 oth = cadd(cmul(gam, ci2k[j]), cmul(del, ci2k2[j]));
                    c[j] = cadd(cmul(al, own), cmul(be, oth));
                    if (i == k) c[j].y = 0.0;
                }
                v = cadd(cmul(gam, v), cmul(del, vik2));
            }
        }
        if (!any_sweep) break;
    }
    if (sweep == kAjdMaxSweeps) flag |= kFlagSweeps;
    bool finite = !in || cfinite(v);
#pragma unroll
    for (int j = 0; j < NC; ++j) finite = finite && (!in || cfinite(c[j]));
    if (!__all(finite) || !__builtin_isfinite(ld)) flag |= kFlagNonFinite;
    if (in && !(flag & kFreezeMask)) {
        Pnew[i * M + k] = v;
        if (PnewT) PnewT[i * M + k] = make_vec2<Tb>((Tb)v.x, (Tb)v.y);
        if (i == k) {
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                lam[j * kMM + i] = c[j].x;
                if (lamT) lamT[j * kMM + i] = (Tb)c[j].x;
            }
            lam[(J - 1) * kMM + i] = 1.0;
            if (lamT) lamT[(J - 1) * kMM + i] = (Tb)1;
        }
    }
    *dlogdet = -ld;
    return flag;
}

// ---------------------------------------------------------------- EM kernel
template <int M, int J, typename T> struct MultiShared {
    static constexpr int NTH = kMThreads;
    using Tb = T;
    using T2 = typename Vec2<T>::type;
    static constexpr int MM = M * M;
    static constexpr int NV = J * MM;
    static constexpr int CH = NV < 32 ? NV : 32;
    static constexpr int NCH = (NV + CH - 1) / CH;
    static constexpr int NW = kMThreads / 64;
    double2 P[MM];
    T2 Pt[MM];
    double lam[J * kMM];
    T lamT[J * kMM];
    double logdet;
    int flag, bad;
    double2 S[J][kMS];
    T red[kMThreads * (CH + 1)];
    double wh[NW][64];
    double wp[NW][NV];
    double LL[NW];
    AjdScratch ws;
};

// One bin (see the file comment); `ok` masks padding frames.
template <int M, int J, typename T>
__device__ __forceinline__ void multi_bin(const T (&yr)[M], const T (&yi)[M], const T (&a)[J], const T* lmT,
                                          const typename Vec2<T>::type* Pt, bool ok, T (&acc)[J * M * M],
                                          double& llacc, T (&nvo)[J], bool& bad) {
    using T2 = typename Vec2<T>::type;
    using MT = Math<T>;
    constexpr int MM = M * M;
    T ytr[M], yti[M], e[M];
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
    T pw[J][M], d[M], r[M];
    T quad = T(0);
#pragma unroll
    for (int i = 0; i < M; ++i) {
        T s = T(0);
#pragma unroll
        for (int j = 0; j < J; ++j) {
            pw[j][i] = a[j] * lmT[j * kMM + i];
            s += pw[j][i];
        }
        d[i] = s;
        r[i] = MT::rcp(s);
        quad = fma(e[i], r[i], quad);
    }
    T logd = T(0);
    if constexpr (sizeof(T) == 4) {
        float l2 = 0.0f;
#pragma unroll
        for (int i = 0; i < M; ++i) l2 += __builtin_amdgcn_logf(d[i]);
        logd = l2 * 0.69314718055994531f;
    } else {
#pragma unroll
        for (int i = 0; i < M; i += 2) logd += MT::log((i + 1 < M) ? d[i] * d[i + 1] : d[i]);
    }
    if (ok) llacc += (double)(-logd - quad);
    T zr[M], zi[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        zr[i] = r[i] * ytr[i];
        zi[i] = r[i] * yti[i];
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        T t[M], s = T(0);
#pragma unroll
        for (int i = 0; i < M; ++i) {
            t[i] = r[i] * (fma(pw[j][i] * e[i], r[i], d[i]) - pw[j][i]);
            s += t[i];
        }
        T nv = a[j] * s * (T(1) / T(M));
        if (ok) bad = bad || !(nv > T(0)) || !isfinite(nv);
        if constexpr (sizeof(T) == 4) nv = fmaxf(nv, kPowerFloorF32);
        if (ok) nvo[j] = nv;
        const T kj = ok ? a[j] * MT::rcp(nv) : T(0);
        const T al = kj * a[j];
#pragma unroll
        for (int i = 0; i < M; ++i) acc[j * MM + i] = fma(kj, t[i], acc[j * MM + i]);
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int q = i + 1; q < M; ++q) {
                const int o = j * MM + M + 2 * pair_index(M, i, q);
                acc[o] = fma(al, fma(zr[i], zr[q], zi[i] * zi[q]), acc[o]);
                acc[o + 1] = fma(al, fma(zi[i], zr[q], -zr[i] * zi[q]), acc[o + 1]);
            }
    }
}

constexpr double kMultiTolFp64 = 1e-15;
constexpr double kMultiTolFp32 = 1e-8;

// Problem table entries: y_off, v_off (source j at + j v2_off), n, npad, pid.
// Register budget in float bulk with up to four frames per thread: three
// workgroups per CU for J = 2 (513 frequencies then run as one wave of
// workgroups on 256 CUs), two for J >= 3 (their J power sums would spill
// heavily at three); no cap otherwise (FP64 needs two workgroups' LDS per CU
// anyway).
template <int M, int J, typename T, int FPT>
constexpr int multi_waves_per_eu() {
    return (sizeof(T) == 4 && FPT <= 4) ? (J >= 3 ? 2 : 3) : 1;
}

template <int M, int J, typename T, int FPT>
__global__ __launch_bounds__(kMThreads) __attribute__((amdgpu_waves_per_eu(multi_waves_per_eu<M, J, T, FPT>()))) void em_multi_kernel(
    const EmProblem* __restrict__ probs, const typename Vec2<T>::type* __restrict__ y, T* __restrict__ v,
    double2* __restrict__ Pg, double* __restrict__ lamg, double* __restrict__ logdetg, int* __restrict__ flagsg,
    double* __restrict__ ll, int64_t ll_stride, int iters, int it_base) {
    using T2 = typename Vec2<T>::type;
    constexpr int MM = M * M;
    __shared__ MultiShared<M, J, T> sh;
    const EmProblem pr = probs[blockIdx.x];
    const int tid = threadIdx.x;
    const int nf = pr.n, npad = pr.npad, pid = pr.pid;
    const double tol = sizeof(T) == 8 ? kMultiTolFp64 : kMultiTolFp32;
    if (tid < MM) {
        sh.P[tid] = Pg[(int64_t)pid * kMS + tid];
        sh.Pt[tid] = make_vec2<T>((T)sh.P[tid].x, (T)sh.P[tid].y);
    }
    if (tid < J * kMM) {
        sh.lam[tid] = lamg[(int64_t)pid * kMJ * kMM + tid];
        sh.lamT[tid] = (T)sh.lam[tid];
    }
    if (tid == 0) {
        sh.logdet = logdetg[pid];
        sh.flag = flagsg[pid];
        sh.bad = 0;
    }
    T yr[FPT][M], yi[FPT][M], vv[FPT][J];
    const T2* __restrict__ yb = y + pr.y_off;
#pragma unroll
    for (int f = 0; f < FPT; ++f) {
        const int n = f * kMThreads + tid;
        const bool ok = n < nf;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            T2 val;
            if (ok) val = yb[(int64_t)m * npad + n];
            else { val.x = T(0); val.y = T(0); }
            yr[f][m] = val.x;
            yi[f][m] = val.y;
        }
#pragma unroll
        for (int j = 0; j < J; ++j) vv[f][j] = ok ? v[pr.v_off + j * pr.v2_off + n] : T(1);
    }
    __syncthreads();
    const bool frozen_at_entry = (sh.flag & kFreezeMask) != 0;
    const int passes = (iters > 0 && !frozen_at_entry) ? iters : 1;
    const int ll_count = iters > 0 ? iters : 1;
    for (int it = 0; it < passes; ++it) {
        T acc[J * MM];
#pragma unroll
        for (int q = 0; q < J * MM; ++q) acc[q] = T(0);
        double llacc = 0.0;
        bool bad = false;
        T vn[FPT][J];
#pragma unroll
        for (int f = 0; f < FPT; ++f) {
#pragma unroll
            for (int j = 0; j < J; ++j) vn[f][j] = vv[f][j];
            if (f * kMThreads >= nf) continue;
            multi_bin<M, J, T>(yr[f], yi[f], vv[f], sh.lamT, sh.Pt, (f * kMThreads + tid) < nf, acc, llacc, vn[f],
                               bad);
        }
        if (bad) sh.bad = 1;
        wg_reduce_sums<M, J>(sh, acc, llacc, nf, tid, sh.lam, kMM);
        if (tid < 64) {
            double tot = 0.0;
#pragma unroll
            for (int w = 0; w < MultiShared<M, J, T>::NW; ++w) tot += sh.LL[w];
            tot += (double)nf * (-(double)M * kLogPi + sh.logdet);
            const bool last = (iters == 0) || frozen_at_entry;
            if (last) {
                if (tid == 0)
                    for (int l = it; l < ll_count; ++l) ll[(int64_t)l * ll_stride + pid] = tot;
            } else {
                if (tid == 0) ll[(int64_t)it * ll_stride + pid] = tot;
                int flag = sh.bad ? kFlagNonFinite : 0;
                double dld = 0.0;
                __builtin_amdgcn_s_setprio(3);
                if (!flag) flag = ajd_wave<M, J, T>(sh.S, sh.P, sh.ws, sh.P, sh.lam, sh.Pt, sh.lamT, &dld, tol);
                __builtin_amdgcn_s_setprio(0);
                if (flag & kFreezeMask) {
                    if (tid == 0)
                        for (int l = it + 1; l < ll_count; ++l) ll[(int64_t)l * ll_stride + pid] = tot;
                    flag |= (it_base + it + 1) << kFlagIterShift;
                } else if (tid == 0) {
                    sh.logdet += dld;
                }
                if (tid == 0) sh.flag |= flag;
            }
        }
        __syncthreads();
        if (iters == 0 || frozen_at_entry || (sh.flag & kFreezeMask)) break;
#pragma unroll
        for (int f = 0; f < FPT; ++f)
#pragma unroll
            for (int j = 0; j < J; ++j) vv[f][j] = vn[f][j];
    }
    if (iters > 0 && !frozen_at_entry) {
#pragma unroll
        for (int f = 0; f < FPT; ++f) {
            const int n = f * kMThreads + tid;
            if (n < nf)
#pragma unroll
                for (int j = 0; j < J; ++j) v[pr.v_off + j * pr.v2_off + n] = vv[f][j];
        }
        if (tid < MM) Pg[(int64_t)pid * kMS + tid] = sh.P[tid];
        if (tid < J * kMM) lamg[(int64_t)pid * kMJ * kMM + tid] = sh.lam[tid];
        if (tid == 0) {
            logdetg[pid] = sh.logdet;
            flagsg[pid] = sh.flag;
        }
    }
}

// Initial basis of every frequency: S_j^(0) (R0, [J][F][M][M]) projected by
// the same whitening and joint diagonalisation (from P = I). One wave per
// frequency.
template <int M, int J>
__global__ __launch_bounds__(64) void multi_project_kernel(const double2* __restrict__ R0, int F, double2* __restrict__ Pg,
                                                           double* __restrict__ lamg, double* __restrict__ logdetg,
                                                           int* __restrict__ flagsg) {
    __shared__ double2 S[J][kMS];
    __shared__ double2 Id[kMS];
    __shared__ double2 Pn[kMS];
    __shared__ double lam[J * kMM];
    __shared__ AjdScratch ws;
    const int f = blockIdx.x, tid = threadIdx.x;
    constexpr int MM = M * M;
    if (tid < J * kMM) lam[tid] = 1.0;
    if (tid < MM) {
        const int r = tid / M, c = tid % M;
        Id[tid] = make_double2(r == c ? 1.0 : 0.0, 0.0);
#pragma unroll
        for (int j = 0; j < J; ++j) {
            // Hermitian from the upper triangle
            const double2 val = (r <= c) ? R0[((int64_t)j * F + f) * MM + r * M + c]
                                         : cconj(R0[((int64_t)j * F + f) * MM + c * M + r]);
            S[j][tid] = (r == c) ? make_double2(val.x, 0.0) : val;
        }
    }
    __syncthreads();
    double dld = 0.0;
    const int flag = ajd_wave<M, J, double>(S, Id, ws, Pn, lam, nullptr, nullptr, &dld, kMultiTolFp64);
    wave_lds_sync();
    const bool ok = !(flag & kFreezeMask);
    if (tid < MM) Pg[(int64_t)f * kMS + tid] = ok ? Pn[tid] : Id[tid];
    if (tid < J * kMM) lamg[(int64_t)f * kMJ * kMM + tid] = ok ? lam[tid] : 1.0;
    if (tid == 0) {
        logdetg[f] = ok ? dld : 0.0;
        flagsg[f] = flag & kFreezeMask;
    }
}

// R_j = P^-H Lambda_j P^-1 of every frequency, [J][F][M][M]; and P^-1.
template <int M, int J>
__global__ void multi_recover_kernel(const double2* __restrict__ Pg, const double* __restrict__ lamg, int F,
                                     double2* __restrict__ R, double2* __restrict__ Pinv) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double2 X[M][M];
    invert<M>(Pg + (int64_t)f * kMS, X);
    if (Pinv)
        for (int a = 0; a < M; ++a)
            for (int b = 0; b < M; ++b) Pinv[(int64_t)f * kMS + a * M + b] = X[a][b];
    if (!R) return;
    for (int j = 0; j < J; ++j) {
        const double* lj = lamg + (int64_t)f * kMJ * kMM + j * kMM;
        for (int a = 0; a < M; ++a)
            for (int b = 0; b < M; ++b) {
                double2 s = make_double2(0.0, 0.0);
                for (int q = 0; q < M; ++q) s = cadd(s, cscale(lj[q], cmulc(X[q][b], X[q][a])));
                if (a == b) s.y = 0.0;
                R[(((int64_t)j * F + f) * M + a) * M + b] = s;
            }
    }
}

// MMSE images x_j = P^-H mu~_j, [J][F][N][M]; one thread per bin.
template <int M, int J, typename T>
__global__ void multi_separate_kernel(const typename Vec2<T>::type* __restrict__ y, const T* __restrict__ v,
                                      const double2* __restrict__ Pg, const double2* __restrict__ Pinv,
                                      const double* __restrict__ lamg, int F, int N, int npad,
                                      typename Vec2<T>::type* __restrict__ x) {
    using T2 = typename Vec2<T>::type;
    const int f = blockIdx.y;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    T yr[M], yi[M];
    for (int m = 0; m < M; ++m) {
        const T2 val = y[((int64_t)f * M + m) * npad + n];
        yr[m] = val.x;
        yi[m] = val.y;
    }
    double ytr[M], yti[M];
    for (int i = 0; i < M; ++i) {
        double sr = 0.0, si = 0.0;
        for (int m = 0; m < M; ++m) {
            const double2 p = Pg[(int64_t)f * kMS + m * M + i];
            sr += p.x * yr[m] + p.y * yi[m];
            si += p.x * yi[m] - p.y * yr[m];
        }
        ytr[i] = sr;
        yti[i] = si;
    }
    const double* lf = lamg + (int64_t)f * kMJ * kMM;
    double pw[J][M], d[M];
    for (int i = 0; i < M; ++i) {
        d[i] = 0.0;
        for (int j = 0; j < J; ++j) {
            pw[j][i] = (double)v[((int64_t)j * F + f) * npad + n] * lf[j * kMM + i];
            d[i] += pw[j][i];
        }
    }
    for (int j = 0; j < J; ++j) {
        double mr[M], mi[M];
        for (int i = 0; i < M; ++i) {
            const double g = pw[j][i] / d[i];
            mr[i] = g * ytr[i];
            mi[i] = g * yti[i];
        }
        for (int m = 0; m < M; ++m) {
            // (P^-H mu~)_m = sum_i conj(Pinv[i][m]) mu~_i
            double sr = 0.0, si = 0.0;
            for (int i = 0; i < M; ++i) {
                const double2 q = Pinv[(int64_t)f * kMS + i * M + m];
                sr += q.x * mr[i] + q.y * mi[i];
                si += q.x * mi[i] - q.y * mr[i];
            }
            T2 o;
            o.x = (T)sr;
            o.y = (T)si;
            x[(((int64_t)j * F + f) * N + n) * M + m] = o;
        }
    }
}

template <int M, int J, typename T>
hipError_t launch_multi_em(int fpt, const EmProblem* probs, int F, const void* y, void* v, double2* P, double* lam,
                           double* logdet, int* flags, double* ll, int iters, int it_base, hipStream_t s) {
    using T2 = typename Vec2<T>::type;
    const T2* yy = static_cast<const T2*>(y);
    T* vv = static_cast<T*>(v);
    switch (fpt) {
        case 1: em_multi_kernel<M, J, T, 1><<<F, kMThreads, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, F, iters, it_base); break;
        case 2: em_multi_kernel<M, J, T, 2><<<F, kMThreads, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, F, iters, it_base); break;
        case 4: em_multi_kernel<M, J, T, 4><<<F, kMThreads, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, F, iters, it_base); break;
        case 8: em_multi_kernel<M, J, T, 8><<<F, kMThreads, 0, s>>>(probs, yy, vv, P, lam, logdet, flags, ll, F, iters, it_base); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Dispatch over (M, J) for one of the templated launchers.
template <template <int, int> class Op, typename... A>
hipError_t dispatch_mj(int M, int J, A... args) {
#define FCA_MJ(MM_, JJ_) \
    if (M == MM_ && J == JJ_) return Op<MM_, JJ_>::run(args...);
    FCA_MJ(1, 2) FCA_MJ(1, 3) FCA_MJ(1, 4) FCA_MJ(2, 2) FCA_MJ(2, 3) FCA_MJ(2, 4)
    FCA_MJ(3, 2) FCA_MJ(3, 3) FCA_MJ(3, 4) FCA_MJ(4, 2) FCA_MJ(4, 3) FCA_MJ(4, 4)
#undef FCA_MJ
    return hipErrorInvalidValue;
}

template <int M, int J> struct OpEm {
    static hipError_t run(bool fp64, int fpt, const EmProblem* probs, int F, const void* y, void* v, double2* P,
                          double* lam, double* logdet, int* flags, double* ll, int iters, int it_base, hipStream_t s) {
        return fp64 ? launch_multi_em<M, J, double>(fpt, probs, F, y, v, P, lam, logdet, flags, ll, iters, it_base, s)
                    : launch_multi_em<M, J, float>(fpt, probs, F, y, v, P, lam, logdet, flags, ll, iters, it_base, s);
    }
};
template <int M, int J> struct OpProject {
    static hipError_t run(const double2* R0, int F, double2* P, double* lam, double* logdet, int* flags, hipStream_t s) {
        multi_project_kernel<M, J><<<F, 64, 0, s>>>(R0, F, P, lam, logdet, flags);
        return hipGetLastError();
    }
};
template <int M, int J> struct OpRecover {
    static hipError_t run(const double2* P, const double* lam, int F, double2* R, double2* Pinv, hipStream_t s) {
        multi_recover_kernel<M, J><<<(F + 63) / 64, 64, 0, s>>>(P, lam, F, R, Pinv);
        return hipGetLastError();
    }
};
template <int M, int J> struct OpSeparate {
    static hipError_t run(bool fp64, const void* y, const void* v, const double2* P, const double2* Pinv,
                          const double* lam, int F, int N, int npad, void* x, hipStream_t s) {
        const dim3 grid((N + 127) / 128, F);
        if (fp64)
            multi_separate_kernel<M, J, double><<<grid, 128, 0, s>>>(static_cast<const double2*>(y),
                                                                      static_cast<const double*>(v), P, Pinv, lam, F, N,
                                                                      npad, static_cast<double2*>(x));
        else
            multi_separate_kernel<M, J, float><<<grid, 128, 0, s>>>(static_cast<const float2*>(y),
                                                                     static_cast<const float*>(v), P, Pinv, lam, F, N,
                                                                     npad, static_cast<float2*>(x));
        return hipGetLastError();
    }
};

bool on_device(const void* p) {
    hipPointerAttribute_t a;
    if (!p || hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged || a.isManaged;
}

}  // namespace
}  // namespace fca

struct fca_mctx {
    int M = 0, F = 0, N = 0, npad = 0, J = 0, fpt = 1;
    bool fp64 = false;
    int esz = 8, rsz = 4;
    hipStream_t stream = nullptr;
    void* y = nullptr;          // [F][M][npad] complex
    void* v = nullptr;          // [J][F][npad] real
    double2* P = nullptr;       // [F][16]
    double2* Pinv = nullptr;    // [F][16]
    double* lam = nullptr;      // [F][J max][4]
    double* logdet = nullptr;   // [F]
    int* flags = nullptr;       // [F]
    double* ll = nullptr;       // [128][F]
    double* ll_tot = nullptr;   // [128]
    double* fsum = nullptr;     // [F + 1]
    double2* R0 = nullptr;      // [J][F][M][M]
    fca::EmProblem* probs = nullptr;
    int* flag_sum = nullptr;    // 5 ints
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // created by the first fca_multi_timing(enable != 0)
    bool timing = false;
    double em_ms = 0.0;
    int64_t em_launches = 0;
    std::string err;
};

namespace {

using fca::EmProblem;

// Whether the Hermitian matrix with the upper triangle of A (M x M,
// row-major) is positive definite: a Cholesky factorisation in double.
bool hermitian_pd(const double2* A, int M) {
    double Lr[4][4] = {}, Li[4][4] = {};
    for (int j = 0; j < M; ++j) {
        double d = A[j * M + j].x;
        for (int q = 0; q < j; ++q) d -= Lr[j][q] * Lr[j][q] + Li[j][q] * Li[j][q];
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        const double l = std::sqrt(d);
        Lr[j][j] = l;
        for (int r = j + 1; r < M; ++r) {
            // A_rj = conj(A_jr); L_rj = (A_rj - sum_q L_rq conj(L_jq)) / L_jj
            double sr = A[j * M + r].x, si = -A[j * M + r].y;
            for (int q = 0; q < j; ++q) {
                sr -= Lr[r][q] * Lr[j][q] + Li[r][q] * Li[j][q];
                si -= Li[r][q] * Lr[j][q] - Lr[r][q] * Li[j][q];
            }
            Lr[r][j] = sr / l;
            Li[r][j] = si / l;
        }
    }
    return true;
}

void mfree(fca_mctx* c) {
    void* ptrs[] = {c->y, c->v, c->P, c->Pinv, c->lam, c->logdet, c->flags, c->ll, c->ll_tot, c->fsum, c->R0, c->probs,
                    c->flag_sum};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
}

template <typename Q>
bool malloc_dev(Q** p, size_t bytes) {
    void* q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    *p = static_cast<Q*>(q);
    return true;
}

fca_status merr(fca_mctx* c, fca_status st, const char* fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else fca::set_global_error(buf);
    return st;
}

#define MHIP(c, call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) return merr((c), FCA_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Flags summary: FCA_E_NOT_PD / FCA_E_NONFINITE as the two-source calls.
fca_status mcheck(fca_mctx* c) {
    int host[5] = {0, 0, 0, 0, 0};
    MHIP(c, fca::launch_flag_summary(c->flags, c->F, c->flag_sum, c->stream));
    MHIP(c, hipMemcpyAsync(host, c->flag_sum, sizeof host, hipMemcpyDeviceToHost, c->stream));
    MHIP(c, hipStreamSynchronize(c->stream));
    if (host[1] < c->F) return merr(c, FCA_E_NOT_PD, "frequency %d lost positive definiteness in iteration %d of the call", host[1], host[3]);
    if (host[2] < c->F) return merr(c, FCA_E_NONFINITE, "frequency %d produced a non-finite value in iteration %d of the call", host[2], host[4]);
    return FCA_OK;
}

}  // namespace

extern "C" {

fca_status fca_multi_init(const fca_problem* p, int32_t J, const double* R0, const void* v0, fca_mctx** out) {
    using namespace fca;
    if (!out) return merr(nullptr, FCA_E_ARG, "fca_multi_init: out is NULL");
    *out = nullptr;
    if (!p || J < 2 || J > kMJ || p->M < 1 || p->M > kMM || p->F < 1 || p->N < 1 || p->N > kMaxFrames ||
        (p->prec != FCA_FP64 && p->prec != FCA_FP32_BULK) || !p->y)
        return merr(nullptr, FCA_E_ARG, "fca_multi_init: need 2 <= J <= 4, 1 <= M <= 4, F >= 1, 1 <= N <= 2048, a "
                                        "known precision and y");
    if (p->R0 || p->v0)
        return merr(nullptr, FCA_E_ARG, "fca_multi_init: give the J-source R0 and v0 as arguments (problem R0, v0 NULL)");
    if (p->y_stride_f < 0 || p->y_stride_n < 0 || p->y_stride_m < 0)
        return merr(nullptr, FCA_E_ARG, "fca_multi_init: negative y stride");
    fca_mctx* c = new (std::nothrow) fca_mctx();
    if (!c) return merr(nullptr, FCA_E_NOMEM, "fca_multi_init: out of host memory");
    c->M = p->M;
    c->F = p->F;
    c->N = p->N;
    c->J = J;
    c->npad = (p->N + 63) / 64 * 64;
    c->fp64 = p->prec == FCA_FP64;
    c->esz = c->fp64 ? 16 : 8;
    c->rsz = c->fp64 ? 8 : 4;
    c->stream = static_cast<hipStream_t>(p->stream);
    while (c->fpt * kMThreads < c->N) c->fpt *= 2;
    const int F = c->F, M = c->M;
    bool ok = malloc_dev(&c->y, (size_t)F * M * c->npad * c->esz) && malloc_dev(&c->v, (size_t)J * F * c->npad * c->rsz) &&
              malloc_dev(&c->P, (size_t)F * kMS * sizeof(double2)) && malloc_dev(&c->Pinv, (size_t)F * kMS * sizeof(double2)) &&
              malloc_dev(&c->lam, (size_t)F * kMJ * kMM * sizeof(double)) && malloc_dev(&c->logdet, (size_t)F * sizeof(double)) &&
              malloc_dev(&c->flags, (size_t)F * sizeof(int)) && malloc_dev(&c->ll, (size_t)kMRows * F * sizeof(double)) &&
              malloc_dev(&c->ll_tot, (size_t)kMRows * sizeof(double)) && malloc_dev(&c->fsum, (size_t)(F + 1) * sizeof(double)) &&
              malloc_dev(&c->R0, (size_t)J * F * M * M * sizeof(double2)) &&
              malloc_dev(&c->probs, (size_t)F * sizeof(EmProblem)) && malloc_dev(&c->flag_sum, 5 * sizeof(int));
    if (!ok) {
        mfree(c);
        delete c;
        return merr(nullptr, FCA_E_NOMEM, "fca_multi_init: device allocation failed");
    }
    const hipStream_t s = c->stream;
    auto fail = [&](fca_status st, const char* what) {
        (void)hipGetLastError();
        mfree(c);
        delete c;
        return merr(nullptr, st, "fca_multi_init: %s", what);
    };
    // y in the EM layout (host y goes through a temporary device copy)
    {
        const int64_t extent = (int64_t)(F - 1) * p->y_stride_f + (int64_t)(p->N - 1) * p->y_stride_n +
                               (int64_t)(M - 1) * p->y_stride_m + 1;
        const void* src = p->y;
        void* tmp = nullptr;
        if (!on_device(p->y)) {
            if (!malloc_dev(&tmp, extent * c->esz)) return fail(FCA_E_NOMEM, "device allocation failed");
            if (hipMemcpyAsync(tmp, p->y, extent * c->esz, hipMemcpyHostToDevice, s) != hipSuccess) {
                (void)hipFree(tmp);
                return fail(FCA_E_DEVICE, "copy of y failed");
            }
            src = tmp;
        }
        const hipError_t e = launch_ingest(c->fp64, src, p->y_stride_f, p->y_stride_n, p->y_stride_m, M, F, c->N,
                                           c->npad, c->y, s);
        if (tmp) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(tmp);
        }
        if (e != hipSuccess) return fail(FCA_E_DEVICE, "ingest failed");
    }
    // problem table
    {
        std::vector<EmProblem> tab(F);
        for (int f = 0; f < F; ++f)
            tab[f] = EmProblem{(int64_t)f * M * c->npad, (int64_t)f * c->npad, (int64_t)F * c->npad, c->N, c->npad, f, M};
        if (hipMemcpy(c->probs, tab.data(), F * sizeof(EmProblem), hipMemcpyHostToDevice) != hipSuccess)
            return fail(FCA_E_DEVICE, "copy of the problem table failed");
    }
    // powers: given [J][F][N], or the plain start (||y||^2 / M, floored) for every source
    if (v0) {
        for (int j = 0; j < J; ++j)
            if (hipMemcpy2DAsync(static_cast<char*>(c->v) + (size_t)j * F * c->npad * c->rsz, c->npad * c->rsz,
                                 static_cast<const char*>(v0) + (size_t)j * F * c->N * c->rsz, c->N * c->rsz,
                                 c->N * c->rsz, F, hipMemcpyDefault, s) != hipSuccess)
                return fail(FCA_E_DEVICE, "copy of v0 failed");
    } else {
        if (launch_power_sums(c->fp64, c->y, M, F, c->N, c->npad, c->fsum, s) != hipSuccess ||
            launch_default_v(c->fp64, c->y, c->fsum, M, F, c->N, c->npad, c->v, s) != hipSuccess)
            return fail(FCA_E_DEVICE, "plain start failed");
        for (int j = 2; j < J; ++j)
            if (hipMemcpyAsync(static_cast<char*>(c->v) + (size_t)j * F * c->npad * c->rsz, c->v,
                               (size_t)F * c->npad * c->rsz, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return fail(FCA_E_DEVICE, "plain start failed");
    }
    // spatial covariances: given (every R_j(f) checked positive definite by a
    // Cholesky factorisation of the Hermitian matrix its upper triangle
    // defines), or the plain start S_j = I + 0.5 (j-1)/(J-1) e1 e1^H
    if (R0) {
        std::vector<double2> h((size_t)J * F * M * M);
        if (hipMemcpy(h.data(), R0, h.size() * sizeof(double2), hipMemcpyDefault) != hipSuccess)
            return fail(FCA_E_DEVICE, "copy of R0 failed");
        for (int j = 0; j < J; ++j)
            for (int f = 0; f < F; ++f)
                if (!hermitian_pd(h.data() + ((size_t)j * F + f) * M * M, M)) {
                    char what[96];
                    snprintf(what, sizeof what, "R0 of source %d at frequency %d is not positive definite", j + 1, f);
                    return fail(FCA_E_ARG, what);
                }
        if (hipMemcpyAsync(c->R0, h.data(), h.size() * sizeof(double2), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(FCA_E_DEVICE, "copy of R0 failed");
    } else {
        std::vector<double2> h((size_t)J * F * M * M, make_double2(0.0, 0.0));
        for (int j = 0; j < J; ++j)
            for (int f = 0; f < F; ++f) {
                double2* S = h.data() + ((size_t)j * F + f) * M * M;
                for (int m = 0; m < M; ++m) S[m * M + m] = make_double2(1.0, 0.0);
                S[0].x += 0.5 * j / (J - 1);
            }
        if (hipMemcpy(c->R0, h.data(), h.size() * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess)
            return fail(FCA_E_DEVICE, "copy of the plain R0 failed");
    }
    if (hipMemsetAsync(c->lam, 0, (size_t)F * kMJ * kMM * sizeof(double), s) != hipSuccess ||
        dispatch_mj<OpProject>(M, J, (const double2*)c->R0, F, c->P, c->lam, c->logdet, c->flags, s) != hipSuccess)
        return fail(FCA_E_DEVICE, "initial decomposition failed");
    c->err.clear();
    const fca_status st = mcheck(c);
    if (st != FCA_OK) {
        const std::string why = c->err;
        mfree(c);
        delete c;
        return merr(nullptr, FCA_E_ARG, "fca_multi_init: R0 is not positive definite (%s)", why.c_str());
    }
    *out = c;
    return FCA_OK;
}

fca_status fca_multi_em_step(fca_mctx* c, int32_t iters, double* loglik, double* R_out, void* v_out) {
    using namespace fca;
    if (!c) return FCA_E_ARG;
    if (iters < 0) return merr(c, FCA_E_ARG, "iters < 0");
    const hipStream_t s = c->stream;
    int done = 0;
    do {
        const int chunk = iters == 0 ? 0 : std::min(kMRows, iters - done);
        const int rows = chunk > 0 ? chunk : 1;
        if (c->timing) MHIP(c, hipEventRecord(c->ev0, s));
        MHIP(c, dispatch_mj<OpEm>(c->M, c->J, c->fp64, c->fpt, (const EmProblem*)c->probs, c->F, (const void*)c->y,
                                  c->v, c->P, c->lam, c->logdet, c->flags, c->ll, chunk, done, s));
        if (c->timing) {
            MHIP(c, hipEventRecord(c->ev1, s));
            MHIP(c, hipEventSynchronize(c->ev1));
            float ms = 0.f;
            MHIP(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
            c->em_ms += ms;
            ++c->em_launches;
        }
        if (loglik) {
            MHIP(c, launch_ll_reduce(c->ll, c->F, rows, 1, c->F, c->ll_tot, s));
            MHIP(c, hipMemcpyAsync(loglik + done, c->ll_tot, rows * sizeof(double), hipMemcpyDefault, s));
        }
        done += chunk;
    } while (done < iters);
    if (R_out) {
        const bool dev = on_device(R_out);
        double2* dst = dev ? reinterpret_cast<double2*>(R_out) : c->R0;   // R0 is free after init
        MHIP(c, dispatch_mj<OpRecover>(c->M, c->J, (const double2*)c->P, (const double*)c->lam, c->F, dst,
                                       (double2*)nullptr, s));
        if (!dev)
            MHIP(c, hipMemcpyAsync(R_out, c->R0, (size_t)c->J * c->F * c->M * c->M * sizeof(double2),
                                   hipMemcpyDeviceToHost, s));
    }
    if (v_out)
        for (int j = 0; j < c->J; ++j)
            MHIP(c, hipMemcpy2DAsync(static_cast<char*>(v_out) + (size_t)j * c->F * c->N * c->rsz, c->N * c->rsz,
                                     static_cast<char*>(c->v) + (size_t)j * c->F * c->npad * c->rsz, c->npad * c->rsz,
                                     c->N * c->rsz, c->F, hipMemcpyDefault, s));
    return mcheck(c);
}

fca_status fca_multi_separate(fca_mctx* c, void* x_out) {
    using namespace fca;
    if (!c || !x_out) return FCA_E_ARG;
    if (!on_device(x_out)) return merr(c, FCA_E_ARG, "fca_multi_separate: x_out must be a device pointer");
    const hipStream_t s = c->stream;
    MHIP(c, dispatch_mj<OpRecover>(c->M, c->J, (const double2*)c->P, (const double*)c->lam, c->F, (double2*)nullptr,
                                   c->Pinv, s));
    MHIP(c, dispatch_mj<OpSeparate>(c->M, c->J, c->fp64, (const void*)c->y, (const void*)c->v, (const double2*)c->P,
                                    (const double2*)c->Pinv, (const double*)c->lam, c->F, c->N, c->npad, x_out, s));
    MHIP(c, hipStreamSynchronize(s));
    return FCA_OK;
}

fca_status fca_multi_timing(fca_mctx* c, int32_t enable, double* em_kernel_ms, int64_t* em_launches) {
    using namespace fca;
    if (!c) return FCA_E_ARG;
    if (enable && !c->ev0) {
        MHIP(c, hipEventCreate(&c->ev0));
        MHIP(c, hipEventCreate(&c->ev1));
    }
    if (em_kernel_ms) *em_kernel_ms = c->em_ms;
    if (em_launches) *em_launches = c->em_launches;
    c->em_ms = 0.0;
    c->em_launches = 0;
    c->timing = enable != 0;
    return FCA_OK;
}

const char* fca_multi_last_error(const fca_mctx* c) { return c ? c->err.c_str() : fca_last_error(nullptr); }

void fca_multi_destroy(fca_mctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    mfree(c);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
}

}  // extern "C"
