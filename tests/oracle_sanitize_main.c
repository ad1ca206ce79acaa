/* Drives every entry point of the C oracle (oracle/fca_oracle.c) on small
 * inputs under AddressSanitizer and UndefinedBehaviorSanitizer: a random
 * mixture, one microphone, one frame, a silent mixture, and invalid sizes.
 * Inputs come from a fixed linear congruential generator; this program checks
 * return codes and that outputs are finite, not values (the values are
 * pinned by the other oracle tests). Built and run by
 * tests/test_oracle_sanitizers.py. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int fca_oracle_em(int M, int F, int N, const double *y, const double *S0, const double *v0, int L, int nthreads,
                  double *S_out, double *v_out, double *ll_out, int *flags);
int fca_oracle_mmse(int M, int F, int N, const double *y, const double *S, const double *v, int nthreads,
                    double *x_out);
int fca_oracle_loglik(int M, int F, int N, const double *y, const double *S, const double *v, int nthreads,
                      double *ll);
int fca_oracle_default_init(int M, int F, int N, const double *y, double *S0_out, double *v0_out);

static unsigned long long state = 12345;
static double uniform(void)
{
    state = state * 6364136223846793005ULL + 1442695040888963407ULL;
    return ((state >> 11) + 0.5) / 9007199254740992.0;
}

static int all_finite(const double *a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i]))
            return 0;
    return 1;
}

/* one case: returns 0 on success */
static int run_case(int M, int F, int N, int L, int silent)
{
    const size_t ny = (size_t)2 * F * N * M, nS = (size_t)2 * 2 * F * M * M, nv = (size_t)2 * F * N;
    double *y = malloc(sizeof(double) * ny), *S0 = malloc(sizeof(double) * nS), *v0 = malloc(sizeof(double) * nv);
    double *S = malloc(sizeof(double) * nS), *v = malloc(sizeof(double) * nv);
    double *ll = malloc(sizeof(double) * (size_t)(L + 1) * F), *llf = malloc(sizeof(double) * F);
    double *x = malloc(sizeof(double) * 2 * ny);
    int *flags = malloc(sizeof(int) * F);
    for (size_t i = 0; i < ny; ++i)
        y[i] = silent ? 0.0 : 2.0 * uniform() - 1.0;
    int bad = 0;
    bad |= fca_oracle_default_init(M, F, N, y, S0, v0) != 0;
    bad |= fca_oracle_em(M, F, N, y, S0, v0, L, 1, S, v, ll, flags) != 0;
    bad |= fca_oracle_loglik(M, F, N, y, S, v, 1, llf) != 0;
    bad |= fca_oracle_mmse(M, F, N, y, S, v, 1, x) != 0;
    for (int f = 0; f < F; ++f)
        bad |= flags[f] != 0;
    bad |= !all_finite(S, nS) || !all_finite(v, nv) || !all_finite(ll, (size_t)(L + 1) * F) ||
           !all_finite(llf, F) || !all_finite(x, 2 * ny);
    free(y); free(S0); free(v0); free(S); free(v); free(ll); free(llf); free(x); free(flags);
    if (bad)
        printf("case M=%d F=%d N=%d L=%d silent=%d failed\n", M, F, N, L, silent);
    return bad;
}

int main(void)
{
    int bad = 0;
    bad |= run_case(3, 2, 5, 3, 0);
    bad |= run_case(8, 1, 4, 2, 0);
    bad |= run_case(1, 3, 6, 4, 0);
    bad |= run_case(2, 2, 1, 2, 0);
    bad |= run_case(2, 2, 4, 2, 1);
    bad |= run_case(4, 1, 7, 0, 0);
    /* invalid sizes are refused without touching the (absent) buffers */
    bad |= fca_oracle_em(0, 1, 1, NULL, NULL, NULL, 1, 1, NULL, NULL, NULL, NULL) != -1;
    bad |= fca_oracle_em(2, 1, 1, NULL, NULL, NULL, -1, 1, NULL, NULL, NULL, NULL) != -1;
    bad |= fca_oracle_default_init(2, 0, 1, NULL, NULL, NULL) != -1;
    bad |= fca_oracle_loglik(2, 1, 0, NULL, NULL, NULL, 1, NULL) != -1;
    bad |= fca_oracle_mmse(99, 1, 1, NULL, NULL, NULL, 1, NULL) != -1;
    printf(bad ? "FAILED\n" : "ok\n");
    return bad;
}
