/*
 * fca_oracle.c -- CPU oracle for the two-source FCA EM. TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library. The product path (the HIP library) never calls it
 * and shares no code, header, table or helper with it.
 *
 * What it computes: the conventional EM of full-rank spatial covariance
 * analysis exactly as stated in Section 2 of Ito, Araki & Nakatani,
 * "FastFCA: a joint diagonalization based fast algorithm for audio source
 * separation using a full-rank spatial covariance model" (arXiv:1805.06572):
 *
 *   likelihood   eq. (like):        p(y) = CN(y; 0, v1 S1 + v2 S2)
 *   E-step       eq. (MMSE):        mu_j = v_j S_j (v1 S1 + v2 S2)^-1 y
 *                eq. (postquadexp): Phi_j = mu_j mu_j^H
 *                                         + v1 S1 (v1 S1 + v2 S2)^-1 v2 S2
 *   M-step       eq. (vupdate):     v_j' = tr(S_j^-1 Phi_j) / M   (old S_j)
 *                eq. (Supdate):     S_j' = (1/N) sum_n Phi_j / v_j'  (new v)
 *
 * The paper states that FastFCA (Section 3, Algorithm 1) produces exactly
 * these iterates, so this frame-wise definition -- with per-bin Cholesky
 * solves and no generalized eigendecomposition -- is the reference the GPU
 * FastFCA path is compared with.  Everything is double precision, summation
 * over frames is sequential in n, and frequencies are independent problems
 * (parallelised with OpenMP, which does not change any result).
 *
 * Readings where the paper is silent:
 *  - Rounding can make a computed Hermitian matrix slightly non-Hermitian;
 *    the posterior term and the new S_j are symmetrised as (A + A^H)/2 with
 *    a real diagonal.
 *  - The paper's S_j is this library's R_j (the spatial covariance).
 *  - A frequency whose computation breaks down (a covariance that is not
 *    positive definite, a non-finite or non-positive power) is frozen at its
 *    last complete iterate and flagged; its later log-likelihood entries are
 *    NaN.
 *
 * Layouts (complex = two doubles, real then imaginary, row-major):
 *   y  [F][N][M] complex        S [2][F][M][M] complex      v [2][F][N]
 *   ll [L+1][F]  per-frequency log-likelihood of theta^(0..L)
 *   x  [2][F][N][M] complex     MMSE source images
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORACLE_MAX_M 16

enum { ORACLE_FLAG_NOT_PD = 1, ORACLE_FLAG_NONFINITE = 2 };

/* Cholesky factor of a Hermitian positive definite A = L L^H (L lower with a
 * positive real diagonal). Returns 0 on success, -1 if A is not numerically
 * positive definite. */
static int cholesky(int M, const cplx *A, cplx *L)
{
    memset(L, 0, sizeof(cplx) * M * M);
    for (int j = 0; j < M; ++j) {
        double d = creal(A[j * M + j]);
        for (int k = 0; k < j; ++k)
            d -= creal(L[j * M + k] * conj(L[j * M + k]));
        if (!(d > 0.0) || !isfinite(d))
            return -1;
        double ljj = sqrt(d);
        L[j * M + j] = ljj;
        for (int i = j + 1; i < M; ++i) {
            cplx s = A[i * M + j];
            for (int k = 0; k < j; ++k)
                s -= L[i * M + k] * conj(L[j * M + k]);
            L[i * M + j] = s / ljj;
        }
    }
    return 0;
}

/* Solve L z = b (forward substitution). */
static void lower_solve(int M, const cplx *L, const cplx *b, cplx *z)
{
    for (int i = 0; i < M; ++i) {
        cplx s = b[i];
        for (int k = 0; k < i; ++k)
            s -= L[i * M + k] * z[k];
        z[i] = s / L[i * M + i];
    }
}

/* Solve L^H x = z (backward substitution). */
static void upper_h_solve(int M, const cplx *L, const cplx *z, cplx *x)
{
    for (int i = M - 1; i >= 0; --i) {
        cplx s = z[i];
        for (int k = i + 1; k < M; ++k)
            s -= conj(L[k * M + i]) * x[k];
        x[i] = s / L[i * M + i];
    }
}

/* x = A^-1 b with A = L L^H. */
static void chol_solve(int M, const cplx *L, const cplx *b, cplx *x)
{
    cplx z[ORACLE_MAX_M];
    lower_solve(M, L, b, z);
    upper_h_solve(M, L, z, x);
}

/* Inverse of a Hermitian positive definite matrix, column by column. */
static int hpd_inverse(int M, const cplx *A, cplx *Ainv)
{
    cplx L[ORACLE_MAX_M * ORACLE_MAX_M], e[ORACLE_MAX_M], col[ORACLE_MAX_M];
    if (cholesky(M, A, L))
        return -1;
    for (int c = 0; c < M; ++c) {
        for (int i = 0; i < M; ++i)
            e[i] = (i == c) ? 1.0 : 0.0;
        chol_solve(M, L, e, col);
        for (int i = 0; i < M; ++i)
            Ainv[i * M + c] = col[i];
    }
    return 0;
}

static void hermitian_part(int M, cplx *A)
{
    for (int i = 0; i < M; ++i) {
        A[i * M + i] = creal(A[i * M + i]);
        for (int k = i + 1; k < M; ++k) {
            cplx h = 0.5 * (A[i * M + k] + conj(A[k * M + i]));
            A[i * M + k] = h;
            A[k * M + i] = conj(h);
        }
    }
}

/* Log-likelihood of one bin, eq. (like): -M log(pi) - log det R - y^H R^-1 y,
 * with R = L L^H, so log det R = 2 sum_i log L_ii and
 * y^H R^-1 y = || L^-1 y ||^2. */
static double bin_loglik(int M, const cplx *L, const cplx *y)
{
    cplx z[ORACLE_MAX_M];
    lower_solve(M, L, y, z);
    double q = 0.0, ld = 0.0;
    for (int i = 0; i < M; ++i) {
        q += creal(z[i] * conj(z[i]));
        ld += log(creal(L[i * M + i]));
    }
    return -M * log(M_PI) - 2.0 * ld - q;
}

/* R = v1 S1 + v2 S2 (the mixture covariance of one bin, eq. like). */
static void mixture_cov(int M, double v1, const cplx *S1, double v2, const cplx *S2, cplx *R)
{
    for (int i = 0; i < M * M; ++i)
        R[i] = v1 * S1[i] + v2 * S2[i];
}

/* Log-likelihood of frequency f under (S, v): sum over frames of eq. (like).
 * Returns NaN if some mixture covariance is not positive definite. */
static double freq_loglik(int M, int N, const cplx *yf, const cplx *S1, const cplx *S2,
                          const double *v1, const double *v2)
{
    cplx R[ORACLE_MAX_M * ORACLE_MAX_M], L[ORACLE_MAX_M * ORACLE_MAX_M];
    double ll = 0.0;
    for (int n = 0; n < N; ++n) {
        mixture_cov(M, v1[n], S1, v2[n], S2, R);
        if (cholesky(M, R, L))
            return NAN;
        ll += bin_loglik(M, L, yf + (size_t)n * M);
    }
    return ll;
}

/* One conventional EM iteration for one frequency (E-step eqs. MMSE and
 * postquadexp, then M-step eqs. vupdate and Supdate). On success S1, S2, v1,
 * v2 hold theta^(l+1) and *ll the log-likelihood of theta^(l). On failure the
 * inputs are left untouched and a flag is returned. */
static int em_iteration_freq(int M, int N, const cplx *yf, cplx *S1, cplx *S2,
                             double *v1, double *v2, double *v1n, double *v2n, double *ll)
{
    const int MM = M * M;
    cplx S1inv[ORACLE_MAX_M * ORACLE_MAX_M], S2inv[ORACLE_MAX_M * ORACLE_MAX_M];
    cplx A1[ORACLE_MAX_M * ORACLE_MAX_M], A2[ORACLE_MAX_M * ORACLE_MAX_M];
    cplx R[ORACLE_MAX_M * ORACLE_MAX_M], L[ORACLE_MAX_M * ORACLE_MAX_M];
    cplx X[ORACLE_MAX_M * ORACLE_MAX_M], C[ORACLE_MAX_M * ORACLE_MAX_M];
    cplx Phi1[ORACLE_MAX_M * ORACLE_MAX_M], Phi2[ORACLE_MAX_M * ORACLE_MAX_M];
    cplx w[ORACLE_MAX_M], mu1[ORACLE_MAX_M], mu2[ORACLE_MAX_M];
    cplx col[ORACLE_MAX_M], sol[ORACLE_MAX_M];

    /* S_j^(l)^-1 for eq. (vupdate): the M-step for v uses the old S_j. */
    if (hpd_inverse(M, S1, S1inv) || hpd_inverse(M, S2, S2inv))
        return ORACLE_FLAG_NOT_PD;
    memset(A1, 0, sizeof(cplx) * MM);
    memset(A2, 0, sizeof(cplx) * MM);
    double llsum = 0.0;

    for (int n = 0; n < N; ++n) {
        const cplx *y = yf + (size_t)n * M;
        const double a = v1[n], b = v2[n];
        mixture_cov(M, a, S1, b, S2, R);
        if (cholesky(M, R, L))
            return ORACLE_FLAG_NOT_PD;
        llsum += bin_loglik(M, L, y);

        /* eq. (MMSE): mu_j = v_j S_j R^-1 y */
        chol_solve(M, L, y, w);
        for (int i = 0; i < M; ++i) {
            cplx s1 = 0.0, s2 = 0.0;
            for (int k = 0; k < M; ++k) {
                s1 += S1[i * M + k] * w[k];
                s2 += S2[i * M + k] * w[k];
            }
            mu1[i] = a * s1;
            mu2[i] = b * s2;
        }

        /* eq. (postquadexp), second term: C = v1 S1 R^-1 (v2 S2).
         * X = R^-1 (v2 S2) column by column, then C = v1 S1 X. */
        for (int c = 0; c < M; ++c) {
            for (int i = 0; i < M; ++i)
                col[i] = b * S2[i * M + c];
            chol_solve(M, L, col, sol);
            for (int i = 0; i < M; ++i)
                X[i * M + c] = sol[i];
        }
        for (int i = 0; i < M; ++i)
            for (int c = 0; c < M; ++c) {
                cplx s = 0.0;
                for (int k = 0; k < M; ++k)
                    s += S1[i * M + k] * X[k * M + c];
                C[i * M + c] = a * s;
            }
        hermitian_part(M, C);

        /* Phi_j = mu_j mu_j^H + C */
        for (int i = 0; i < M; ++i)
            for (int k = 0; k < M; ++k) {
                Phi1[i * M + k] = mu1[i] * conj(mu1[k]) + C[i * M + k];
                Phi2[i * M + k] = mu2[i] * conj(mu2[k]) + C[i * M + k];
            }

        /* eq. (vupdate): v_j' = Re tr(S_j^-1 Phi_j) / M */
        double t1 = 0.0, t2 = 0.0;
        for (int i = 0; i < M; ++i)
            for (int k = 0; k < M; ++k) {
                t1 += creal(S1inv[i * M + k] * Phi1[k * M + i]);
                t2 += creal(S2inv[i * M + k] * Phi2[k * M + i]);
            }
        const double nv1 = t1 / M, nv2 = t2 / M;
        if (!(nv1 > 0.0) || !(nv2 > 0.0) || !isfinite(nv1) || !isfinite(nv2))
            return ORACLE_FLAG_NONFINITE;
        v1n[n] = nv1;
        v2n[n] = nv2;

        /* eq. (Supdate) numerator: sum_n Phi_j / v_j' (uses the new v) */
        for (int i = 0; i < MM; ++i) {
            A1[i] += Phi1[i] / nv1;
            A2[i] += Phi2[i] / nv2;
        }
    }

    for (int i = 0; i < MM; ++i) {
        A1[i] /= N;
        A2[i] /= N;
    }
    hermitian_part(M, A1);
    hermitian_part(M, A2);
    for (int i = 0; i < MM; ++i) {
        if (!isfinite(creal(A1[i])) || !isfinite(cimag(A1[i])) ||
            !isfinite(creal(A2[i])) || !isfinite(cimag(A2[i])))
            return ORACLE_FLAG_NONFINITE;
    }
    memcpy(S1, A1, sizeof(cplx) * MM);
    memcpy(S2, A2, sizeof(cplx) * MM);
    memcpy(v1, v1n, sizeof(double) * N);
    memcpy(v2, v2n, sizeof(double) * N);
    *ll = llsum;
    return 0;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Run L conventional EM iterations from (S0, v0).
 * Outputs S_out, v_out = theta^(L); ll_out[l][f] = log-likelihood of
 * theta^(l) at frequency f for l = 0..L (the last entry needs one extra
 * evaluation pass); flags[f] = 0 or an ORACLE_FLAG_* bitmask.
 * Returns 0, or -1 for invalid sizes. */
int fca_oracle_em(int M, int F, int N, const double *y, const double *S0, const double *v0,
                  int L, int nthreads, double *S_out, double *v_out, double *ll_out, int *flags)
{
    if (M < 1 || M > ORACLE_MAX_M || F < 1 || N < 1 || L < 0)
        return -1;
    const cplx *Y = (const cplx *)y;
    const cplx *SS0 = (const cplx *)S0;
    cplx *SS = (cplx *)S_out;
    const size_t MM = (size_t)M * M;
    set_threads(nthreads);

#pragma omp parallel for schedule(dynamic, 1)
    for (int f = 0; f < F; ++f) {
        const cplx *yf = Y + (size_t)f * N * M;
        cplx *S1 = SS + (size_t)f * MM;
        cplx *S2 = SS + ((size_t)F + f) * MM;
        double *v1 = v_out + (size_t)f * N;
        double *v2 = v_out + ((size_t)F + f) * N;
        memcpy(S1, SS0 + (size_t)f * MM, sizeof(cplx) * MM);
        memcpy(S2, SS0 + ((size_t)F + f) * MM, sizeof(cplx) * MM);
        memcpy(v1, v0 + (size_t)f * N, sizeof(double) * N);
        memcpy(v2, v0 + ((size_t)F + f) * N, sizeof(double) * N);
        hermitian_part(M, S1);
        hermitian_part(M, S2);
        double *v1n = (double *)malloc(sizeof(double) * N);
        double *v2n = (double *)malloc(sizeof(double) * N);
        int flag = 0;
        for (int l = 0; l < L; ++l) {
            double ll = NAN;
            if (!flag)
                flag = em_iteration_freq(M, N, yf, S1, S2, v1, v2, v1n, v2n, &ll);
            ll_out[(size_t)l * F + f] = flag ? NAN : ll;
        }
        ll_out[(size_t)L * F + f] = flag ? NAN : freq_loglik(M, N, yf, S1, S2, v1, v2);
        flags[f] = flag;
        free(v1n);
        free(v2n);
    }
    return 0;
}

/* MMSE source images under (S, v), eq. (MMSE): x_j = v_j S_j R^-1 y.
 * Returns 0, -1 for invalid sizes, or 1 if some bin's R is not PD (its
 * outputs are then NaN). */
int fca_oracle_mmse(int M, int F, int N, const double *y, const double *S, const double *v,
                    int nthreads, double *x_out)
{
    if (M < 1 || M > ORACLE_MAX_M || F < 1 || N < 1)
        return -1;
    const cplx *Y = (const cplx *)y;
    const cplx *SS = (const cplx *)S;
    cplx *X = (cplx *)x_out;
    const size_t MM = (size_t)M * M;
    int bad = 0;
    set_threads(nthreads);

#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int f = 0; f < F; ++f) {
        const cplx *S1 = SS + (size_t)f * MM, *S2 = SS + ((size_t)F + f) * MM;
        cplx R[ORACLE_MAX_M * ORACLE_MAX_M], L[ORACLE_MAX_M * ORACLE_MAX_M], w[ORACLE_MAX_M];
        for (int n = 0; n < N; ++n) {
            const cplx *yb = Y + ((size_t)f * N + n) * M;
            const double a = v[(size_t)f * N + n], b = v[((size_t)F + f) * N + n];
            cplx *x1 = X + ((size_t)f * N + n) * M;
            cplx *x2 = X + (((size_t)F + f) * N + n) * M;
            mixture_cov(M, a, S1, b, S2, R);
            if (cholesky(M, R, L)) {
                for (int i = 0; i < M; ++i)
                    x1[i] = x2[i] = NAN;
                bad = 1;
                continue;
            }
            chol_solve(M, L, yb, w);
            for (int i = 0; i < M; ++i) {
                cplx s1 = 0.0, s2 = 0.0;
                for (int k = 0; k < M; ++k) {
                    s1 += S1[i * M + k] * w[k];
                    s2 += S2[i * M + k] * w[k];
                }
                x1[i] = a * s1;
                x2[i] = b * s2;
            }
        }
    }
    return bad ? 1 : 0;
}

/* Per-frequency log-likelihood of (S, v) under eq. (like): ll[f]. */
int fca_oracle_loglik(int M, int F, int N, const double *y, const double *S, const double *v,
                      int nthreads, double *ll)
{
    if (M < 1 || M > ORACLE_MAX_M || F < 1 || N < 1)
        return -1;
    const cplx *Y = (const cplx *)y;
    const cplx *SS = (const cplx *)S;
    const size_t MM = (size_t)M * M;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int f = 0; f < F; ++f)
        ll[f] = freq_loglik(M, N, Y + (size_t)f * N * M, SS + (size_t)f * MM,
                            SS + ((size_t)F + f) * MM, v + (size_t)f * N, v + ((size_t)F + f) * N);
    return 0;
}

/* The plain start used when no initial values are given: R1 = I,
 * R2 = I + 0.5 e1 e1^H, and for both sources v_j(n,f) = ||y(n,f)||^2 / M,
 * floored at 1e-12 times the mean of ||y||^2 / M over all bins (1 if that
 * mean is zero). */
int fca_oracle_default_init(int M, int F, int N, const double *y, double *S0_out, double *v0_out)
{
    if (M < 1 || M > ORACLE_MAX_M || F < 1 || N < 1)
        return -1;
    const cplx *Y = (const cplx *)y;
    cplx *S = (cplx *)S0_out;
    const size_t MM = (size_t)M * M;
    for (int j = 0; j < 2; ++j)
        for (int f = 0; f < F; ++f) {
            cplx *Sf = S + ((size_t)j * F + f) * MM;
            for (size_t i = 0; i < MM; ++i)
                Sf[i] = 0.0;
            for (int i = 0; i < M; ++i)
                Sf[i * M + i] = 1.0;
            if (j == 1)
                Sf[0] += 0.5;
        }
    double mean = 0.0;
    for (size_t b = 0; b < (size_t)F * N; ++b) {
        double p = 0.0;
        for (int m = 0; m < M; ++m)
            p += creal(Y[b * M + m] * conj(Y[b * M + m]));
        v0_out[b] = p / M;
        mean += p / M;
    }
    mean /= (double)F * N;
    const double floor_v = mean > 0.0 ? 1e-12 * mean : 1.0;
    for (size_t b = 0; b < (size_t)F * N; ++b) {
        if (!(v0_out[b] >= floor_v))
            v0_out[b] = floor_v;
        v0_out[(size_t)F * N + b] = v0_out[b];
    }
    return 0;
}
