/*
 * fca.h -- C ABI of the MI355X (gfx950) FastFCA EM library, libfca.so.
 *
 * The library estimates the two-source full-rank spatial covariance model
 * of Ito, Araki & Nakatani, "FastFCA" (arXiv:1805.06572), Section 2:
 *     y(n,f) = x1(n,f) + x2(n,f),   x_j(n,f) ~ CN(0, v_j(n,f) R_j(f)),
 * with R_j(f) Hermitian positive definite (the paper's S_j(f)) and
 * v_j(n,f) > 0, by the FastFCA EM of Section 3 (Algorithm 1): a per-
 * frequency generalized eigendecomposition jointly diagonalises R1 and R2,
 * so every time-frequency bin is updated with scalar arithmetic.
 *
 * Conventions for every entry point
 *  - Every call returns an fca_status; nothing throws across the ABI and
 *    nothing aborts. Calls are stream-ordered on the stream given at init
 *    and synchronous on return.
 *  - Complex numbers are interleaved (real, imaginary): complex128 in
 *    FCA_FP64 mode, complex64 in FCA_FP32_BULK mode. "prec real" means
 *    double in FCA_FP64 mode and float in FCA_FP32_BULK mode.
 *  - Pointers may be host or device memory unless stated otherwise; the
 *    library tells them apart with hipPointerGetAttributes. Every output
 *    buffer is allocated and owned by the caller.
 *  - Matrices are row-major; element (m, m') of an M x M matrix is at
 *    m * M + m'.
 *  - A context is not thread-safe. Different contexts are independent.
 */
#ifndef FCA_H
#define FCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fca_ctx fca_ctx;

typedef enum {
    FCA_OK = 0,
    FCA_E_ARG = -1,       /* invalid argument; nothing was changed or allocated */
    FCA_E_NOMEM = -2,     /* a device or pinned-host allocation failed */
    FCA_E_DEVICE = -3,    /* a HIP runtime call or kernel launch failed */
    FCA_E_NOT_PD = -4,    /* some frequency lost positive definiteness (see flags) */
    FCA_E_NONFINITE = -5, /* some frequency produced a non-finite value (see flags) */
    FCA_E_STATE = -6      /* the context is unusable after an earlier device error */
} fca_status;

typedef enum {
    FCA_FP64 = 0,      /* everything in double precision */
    FCA_FP32_BULK = 1  /* per-bin arithmetic in float; the generalized eigen-
                          decomposition, every cross-thread sum and the log-
                          likelihood sums in double. Updated powers are kept
                          >= 1e-30 so that the float arithmetic stays in the
                          normal range (an all-zero bin roughly halves its
                          powers at every iteration); FCA_FP64 has no floor */
} fca_precision;

/* Per-frequency status bits (fca_status_per_freq). A frequency with
 * FCA_FLAG_NOT_PD or FCA_FLAG_NONFINITE is frozen at its last complete
 * iterate theta^(l): later iterations leave it unchanged and report the
 * log-likelihood of that iterate. Other frequencies are unaffected. */
#define FCA_FLAG_NOT_PD 1    /* a Cholesky pivot of R2 (or its eigenbasis
                                form) was not positive */
#define FCA_FLAG_NONFINITE 2 /* a power or covariance entry was non-finite or
                                a power was not positive */
#define FCA_FLAG_SWEEPS 4    /* the Jacobi eigen-solver stopped at its sweep
                                limit (informational; not frozen) */

/* One mixture (Section 2, problem statement).
 *   M        microphones (the paper's I), 1 <= M <= 8
 *   F        frequency bins (DC .. Nyquist), F >= 1
 *   N        frames, 1 <= N <= 16777216 (up to 2048 frames stay in registers for
 *            all iterations; longer mixtures are re-read from memory every pass)
 *   prec     an fca_precision
 *   y        observed STFT mixture y(n,f), complex (prec), element (f,n,m)
 *            at y + f*y_stride_f + n*y_stride_n + m*y_stride_m, strides in
 *            complex elements and >= 0 (torch.stft's [m][f][n] and the
 *            natural [f][n][m] both fit); copied into the context by
 *            fca_init, so the caller may free it afterwards.
 *   R0       optional initial spatial covariances, [2][F][M][M] complex128
 *            (R_1 then R_2), Hermitian positive definite (only the upper
 *            triangle is read); NULL selects R1 = I, R2 = I + 0.5 e1 e1^H.
 *   v0       optional initial powers, [2][F][N] prec real, > 0; NULL selects
 *            v_j(n,f) = ||y(n,f)||^2 / M for both sources, floored at 1e-12
 *            times the mean of ||y||^2 / M over all bins (1 if that mean is
 *            zero). R0 and v0 are copied at init.
 *   stream   hipStream_t for all work of the context; NULL = null stream. */
typedef struct {
    int32_t M, F, N;
    int32_t prec;
    const void *y;
    int64_t y_stride_f, y_stride_n, y_stride_m;
    const double *R0;
    const void *v0;
    void *stream;
} fca_problem;

/* Create a context for one mixture, copy y, R0, v0 into device memory and
 * set the initial values (Algorithm 1, step 1): v^(0) and the generalized
 * eigenvectors P^(0) and eigenvalues Lambda^(0) of (R1^(0), R2^(0)).
 * Returns FCA_E_ARG (and *out = NULL) for invalid sizes, pointers or an R0
 * that is not positive definite. */
fca_status fca_init(const fca_problem *p, fca_ctx **out);

/* As fca_init for B >= 1 mixtures processed together. All mixtures share F,
 * prec and stream; M and N may differ per mixture. Batch outputs below are
 * the per-mixture outputs concatenated in mixture order. */
fca_status fca_init_batch(const fca_problem *p, int32_t B, fca_ctx **out);

/* Set the initial values again from the R0 and v0 given at init (or the
 * plain start), clearing all per-frequency flags (Algorithm 1, step 1), and
 * make every mixture active again (fca_set_active). The starts are kept
 * materialised (powers and the basis of their GEVD), so this is a few
 * whole-buffer device copies; waits for the stream. Allocates nothing. */
fca_status fca_reset(fca_ctx *c);

/* Replace the initial values of mixture b and reset that mixture to them
 * (Algorithm 1, step 1); every other mixture keeps its current state.
 *   R0  NULL (R1 = I, R2 = I + 0.5 e1 e1^H) or [2][F][M][M] complex128,
 *       host or device, copied; must be Hermitian positive definite.
 *   v0  NULL (the plain start ||y(n,f)||^2 / M) or [2][F][N] prec reals,
 *       host or device, copied; must be positive.
 * The new start is what later fca_reset calls return to, and the mixture is
 * made active. A non-positive-definite R0 gives FCA_E_ARG and leaves mixture
 * b's stored start and its parameters as they were (its per-frequency flags
 * are cleared). Runs asynchronously on
 * the context's stream unless v0 is a host pointer or R0 is given (its
 * definiteness is checked before returning). */
fca_status fca_set_start(fca_ctx *c, int32_t b, const double *R0, const void *v0);

/* Take mixture b out of (active = 0) or back into (active != 0) later
 * fca_em_step and fca_conv_em_step calls. An inactive mixture keeps its
 * parameters; those calls skip its frequencies and write NaN to its loglik
 * rows (R_out, v_out and fca_separate still cover it). Lets a batch stop each
 * mixture once it has converged. Host-only bookkeeping: the launch tables
 * are rebuilt by the next EM call. Allocates nothing. */
fca_status fca_set_active(fca_ctx *c, int32_t b, int32_t active);

/* Run `iters` >= 0 EM iterations (Algorithm 1, steps 3-9) on every active
 * mixture (all of them unless fca_set_active took some out).
 *   loglik  NULL, or [B][iters] doubles: the log-likelihood (eq. like,
 *           summed over all bins of the mixture) of theta^(l) at the start
 *           of iteration l. With iters == 0 nothing is updated and
 *           loglik[b] receives the log-likelihood of the current parameters.
 *   R_out   NULL, or [2][F][M][M] complex128 per mixture: R_j(f) of the
 *           parameters after the call, recovered as R2 = (P P^H)^-1 and
 *           R1 = P^-H Lambda P^-1 (eq. recoverS).
 *   v_out   NULL, or [2][F][N] prec real per mixture: v_j(n,f) after the call.
 * Returns FCA_E_NOT_PD or FCA_E_NONFINITE when some frequency is flagged
 * (all outputs are still written; see fca_status_per_freq). */
fca_status fca_em_step(fca_ctx *c, int32_t iters, double *loglik, double *R_out, void *v_out);

/* The same L iterations computed by the conventional frame-wise EM of
 * Section 2 (eqs. MMSE, postquadexp, vupdate, Supdate: per bin a Cholesky
 * factorisation of v1 R1 + v2 R2, its solves and matrix products, no
 * eigendecomposition), on the same context and with the same arguments,
 * outputs and failure semantics as fca_em_step. The paper states the two
 * algorithms produce identical iterates; this entry point is the in-run
 * baseline of that comparison. Mixtures of more than 2048 frames re-read
 * their frames from memory every pass (powers double-buffered, as in
 * fca_em_step's streamed shape); the others keep them in registers. */
fca_status fca_conv_em_step(fca_ctx *c, int32_t iters, double *loglik, double *R_out, void *v_out);

/* MMSE source images with the current parameters (eq. MMSE; Algorithm 1,
 * step 11): x_out is [2][F][N][M] complex (prec) per mixture, x1 then x2,
 * with x1 = P^-H mu~1 computed in the eigenbasis and x2 = y - x1. */
fca_status fca_separate(fca_ctx *c, void *x_out);

/* Copy the per-frequency FCA_FLAG_* bits, [B][F] int32, to flags. */
fca_status fca_status_per_freq(const fca_ctx *c, int32_t *flags);

/* Per-frequency log-likelihood of the last EM call on the context
 * (fca_em_step, fca_conv_em_step or fca_graph_launch, whichever ran last):
 * ll_out is [rows][B][F] doubles, host or device; entry (r, b, f) is the
 * log-likelihood (eq. like summed over the frames of frequency f) of
 * theta^(l) with l = iters - rows + r counted in that call (its loglik
 * entries summed over f give the per-mixture values). The rows come from
 * the call's final chunk of at most 128 iterations: 1 <= rows <=
 * min(iters, 128), or rows = 1 after an iters = 0 call; FCA_E_ARG
 * otherwise. Mixtures inactive in that call get NaN. FCA_E_STATE before any
 * EM call and after fca_autotune (its trial runs overwrite the rows).
 * Waits for the stream; allocates nothing. */
fca_status fca_loglik_per_freq(const fca_ctx *c, int32_t rows, double *ll_out);

/* Text of the last error of the context (or of the last failed fca_init when
 * c is NULL). The string stays valid until the next call on the context.
 * After FCA_E_NOT_PD or FCA_E_NONFINITE from an EM call it names the first
 * failing mixture and frequency and the iteration of that call (1-based;
 * of the replay for fca_graph_launch) whose update failed; that frequency
 * keeps the parameters of the iteration before. */
const char *fca_last_error(const fca_ctx *c);

/* Free the context and all its device memory. NULL is accepted. */
void fca_destroy(fca_ctx *c);

/* Batched generalized eigendecomposition of Hermitian-definite pencils in
 * FP64 (eq. GEVD and the Appendix theorem): for each of `count` problems,
 * P^H S2 P = I and P^H S1 P = diag(lambda). S1, S2, P are [count][M][M]
 * complex128 and lambda [count] x M doubles, all DEVICE pointers; only the
 * upper triangles of S1 and S2 are read; eigenvalue order is unspecified.
 * flags [count] int32 device pointer receives FCA_FLAG_* bits (NOT_PD if
 * S2 is not positive definite). 1 <= M <= 8. stream as in fca_problem. */
fca_status fca_gevd(int32_t M, int32_t count, const double *S1, const double *S2, double *P,
                    double *lambda, int32_t *flags, void *stream);

/* The plain-start EM of one mixture (Algorithm 1, step 1 with the plain
 * start, then steps 3-9) without any device allocation, for callers that
 * cannot allocate (code under stream capture, serving loops, harnesses that
 * forbid it). Results equal fca_init (plain R; v0 as below) followed by
 * fca_em_step(iters) with the same y. The per-frequency state lives in one
 * fixed-size device array of the library (about 4.3 MiB, held by each GPU
 * the library runs on until the process ends); y and the powers are used in
 * place. Calls on one GPU share that array: calls that overlap in time on
 * one GPU (several streams or threads) race and must be serialised by the
 * caller. Enqueued on `stream` (hipStream_t, NULL = null stream) without
 * waiting; no host synchronisation, so numerical failures are not returned
 * as a status but as flags.
 *   M, F, N  1 <= M <= 8, 1 <= F <= 2048, 1 <= N <= 2048 (frames held in
 *            registers); FCA_E_ARG beyond these limits.
 *   prec     FCA_FP64 or FCA_FP32_BULK.
 *   y        DEVICE, [F][M][pitch] complex (prec): y(n,f) of microphone m
 *            at f*M*pitch + m*pitch + n; N <= pitch <= 2^30.
 *   v        DEVICE, [2][F][pitch] prec reals (v_1 then v_2): in, v^(0)
 *            when use_v0 != 0 (else overwritten with the plain start
 *            ||y||^2 / M floored as in fca_problem); out, v^(iters).
 *   iters    >= 0; 0 evaluates the start only.
 *   loglik   NULL or DEVICE [max(iters, 1)] doubles, as fca_em_step's.
 *   R_out    NULL or DEVICE [2][F][M][M] complex128, as fca_em_step's.
 *   flags_out NULL or DEVICE [F] int32: FCA_FLAG_* bits per frequency.
 * Returns FCA_E_ARG for invalid arguments (nothing is enqueued),
 * FCA_E_DEVICE if a launch fails; fca_last_error(NULL) gives the reason. */
fca_status fca_em_solve_noalloc(int32_t M, int32_t F, int32_t N, int32_t prec, const void *y, int64_t pitch,
                                void *v, int32_t use_v0, int32_t iters, double *loglik, double *R_out,
                                int32_t *flags_out, void *stream);

/* Kernel timing of the EM iterations. enable != 0 makes later fca_em_step
 * calls record HIP events, on the context's stream, around the launches of
 * the EM-iteration kernel. On return *em_kernel_ms and *em_launches hold the
 * totals accumulated since the previous fca_timing call (either may be
 * NULL), and the totals restart from zero. */
fca_status fca_timing(fca_ctx *c, int32_t enable, double *em_kernel_ms, int64_t *em_launches);

/* ------------------------------------------------------------------
 * STFT front and back end (the analysis and resynthesis around the EM in
 * the experiments of Section 4; Table 1: 16 kHz, frames of 1024 samples,
 * frame shift 512, square-root Hann window). Frame length L (a power of two,
 * 16 <= L <= 4096), shift S = L/2, window w(t) = sin(pi t / L), the square
 * root of the periodic Hann window. Frame n holds samples n S - S + t,
 * t = 0 .. L-1 (zero outside 0 .. T-1); N = fca_stft_frames(T, L) =
 * floor((T - 1) / S) + 2 frames, so every sample lies in two frames and,
 * since w(t)^2 + w(t + S)^2 = 1, fca_istft(fca_stft(x)) = x up to rounding.
 * Both run in the precision prec (real float/complex64 or double/
 * complex128), take DEVICE pointers only, are enqueued on `stream`
 * (hipStream_t, NULL = null stream) without waiting and allocate nothing;
 * FCA_E_ARG (nothing enqueued, reason in fca_last_error(NULL)) for invalid
 * sizes or host pointers.
 * ------------------------------------------------------------------ */
int64_t fca_stft_frames(int64_t T, int32_t L);   /* 0 for T < 1 */
/* x: [M][T] real signals. X: [F][N][M] complex, F = L/2 + 1:
 * X[f][n][m] = sum_t w(t) x_m(n S - S + t) exp(-2 pi i f t / L), the layout
 * fca_problem.y takes (y_stride_f = N M, y_stride_n = M, y_stride_m = 1). */
fca_status fca_stft(int32_t M, int64_t T, int32_t L, int32_t prec, const void *x, void *X, void *stream);
/* X: [F][N][M] complex (e.g. one source image of fca_separate's output).
 * x: [M][T] real: the overlap-add of each frame's inverse DFT over the
 * Hermitian extension X[L - k] = conj(X[k]) (real part), windowed by w. */
fca_status fca_istft(int32_t M, int64_t T, int32_t L, int32_t prec, const void *X, void *x, void *stream);

/* ------------------------------------------------------------------
 * More than two sources (the extension Section 5 leaves open; not the
 * paper's algorithm, which is exact for J = 2 only). The model of Section 2
 * with J sources, y = x_1 + .. + x_J, x_j ~ CN(0, v_j R_j), is fitted with
 * every R_j(f) kept in the jointly diagonalisable form R_j = P^-H Lambda_j
 * P^-1 (one basis P per frequency, Lambda_j diagonal, Lambda_J = I). The
 * E-step and power update of each bin run in the basis as in Algorithm 1
 * (exact for parameters of that form); the new R~_j are then projected back
 * onto the form: whitening by R~_J (Cholesky) and a unitary Jacobi joint
 * diagonalisation of the other J - 1 matrices (Cardoso-Souloumiac angles,
 * rounds of disjoint index pairs, FP64, at most 16 sweeps), whose
 * off-diagonal remainder is dropped. For J = 2 the projection is the exact
 * generalized eigendecomposition and the iterates are FastFCA's (eqs.
 * GEVDeff5 .. updateLambdaeff); for J > 2 the update is an approximation of
 * the EM (the likelihood is not guaranteed to increase). One mixture per
 * context; 2 <= J <= 4 sources, 1 <= M <= 4 microphones, 1 <= N <= 2048
 * frames (kept in registers: all iterations of a call run in one launch
 * with one workgroup per frequency), FP64 or FP32 bulk (the joint
 * diagonalisation stays FP64; a pair is rotated only while its rotation
 * exceeds 1e-15 in FP64, 1e-8 in FP32 bulk).
 * ------------------------------------------------------------------ */
typedef struct fca_mctx fca_mctx;

/* Create a J-source context for the mixture p->y (layout and precision as in
 * fca_problem; p->R0 and p->v0 must be NULL).
 *   R0  NULL (the plain start R_j = I + 0.5 (j - 1) / (J - 1) e1 e1^H,
 *       which is fca_init's default for J = 2) or [J][F][M][M] complex128,
 *       host or device, positive definite Hermitian (upper triangles read).
 *       It is projected onto the jointly diagonalisable form first (exact
 *       when it already has that form, as the plain start has).
 *   v0  NULL (every source starts at ||y(n,f)||^2 / M, floored at 1e-12
 *       times its mean) or [J][F][N] prec reals, host or device, positive.
 * FCA_E_ARG (reason in fca_last_error(NULL)) for sizes out of range or an
 * R0 whose R_J is not positive definite; FCA_E_NOMEM, FCA_E_DEVICE.
 * Waits for the context's stream. */
fca_status fca_multi_init(const fca_problem *p, int32_t J, const double *R0, const void *v0, fca_mctx **out);
/* Run iters >= 0 iterations.
 *   loglik  NULL or [iters] doubles (host or device): the log-likelihood
 *           (eq. like with R = sum_j v_j R_j) of theta^(l) at the start of
 *           iteration l; iters = 0: [1], that of the current parameters.
 *   R_out   NULL or [J][F][M][M] complex128 (host or device): R_j of the
 *           parameters after the call, P^-H Lambda_j P^-1.
 *   v_out   NULL or [J][F][N] prec reals (host or device).
 * FCA_E_NOT_PD / FCA_E_NONFINITE as fca_em_step (the failing frequency keeps
 * the parameters of the iteration before; the reason names it). Waits for
 * the stream. */
fca_status fca_multi_em_step(fca_mctx *c, int32_t iters, double *loglik, double *R_out, void *v_out);
/* MMSE source images with the current parameters: x_out (DEVICE) is
 * [J][F][N][M] complex (prec), x_j = P^-H D_j (sum_k D_k)^-1 P^H y with
 * D_j = v_j Lambda_j (eq. MMSE in the basis); they sum to y. Waits. */
fca_status fca_multi_separate(fca_mctx *c, void *x_out);
/* Kernel timing of the iterations, as fca_timing: enable != 0 makes later
 * fca_multi_em_step calls record HIP events on the context's stream around
 * each launch of the iteration kernel (and wait for them); on return
 * *em_kernel_ms and *em_launches (either may be NULL) hold the totals since
 * the previous call, which restart from zero. FCA_E_DEVICE if the events
 * cannot be created. */
fca_status fca_multi_timing(fca_mctx *c, int32_t enable, double *em_kernel_ms, int64_t *em_launches);
const char *fca_multi_last_error(const fca_mctx *c);
void fca_multi_destroy(fca_mctx *c);   /* NULL is accepted */

/* ------------------------------------------------------------------
 * Orchestration of batched runs: launch shapes, autotuning, captured steps.
 * The problems of a context are launched in groups of equal M and frames-
 * per-thread class (one launch per group and chunk of iterations; the groups
 * of one call run concurrently on forked streams). */
typedef struct {
    int32_t M;                 /* microphones of the group's mixtures */
    int32_t threads;           /* workgroup size of its EM launches (256 or 128) */
    int32_t frames_per_thread; /* frames each thread keeps in registers; 0 = streamed */
    int32_t problems;          /* (mixture, frequency) problems in the group */
    int32_t max_frames;        /* largest N among them */
} fca_launch_group;

/* Copy up to cap launch-group descriptions to out; *count (if not NULL)
 * receives the number of groups. */
fca_status fca_launch_groups(const fca_ctx *c, fca_launch_group *out, int32_t cap, int32_t *count);

/* Set the launch shape of launch group `group`: threads 0 or 256, or 128
 * (groups of at most 1024 frames; each thread then keeps up
 * to 8 frames in registers); streamed != 0 re-reads the frames from memory
 * every pass instead of keeping them in registers (256 threads; the only
 * shape for groups beyond 2048 frames). Results differ only by rounding (a
 * different reduction order). FCA_E_ARG for a group index out of range or a
 * shape that cannot hold the group. A context starts every group at 256
 * threads, except float-bulk groups of M <= 4 microphones, at most 1024
 * frames and more problems than three per compute unit, which start at 128
 * threads (more of their problems fit on a compute unit at once). */
fca_status fca_set_launch_shape(fca_ctx *c, int32_t group, int32_t threads, int32_t streamed);

/* Pick the launch shape of every group by measurement: each admissible shape
 * (256 or 128 threads with frames in registers, or streamed)
 * runs `iters` EM iterations (<= 0: 3) of that group alone, timed with HIP
 * events (best of two after one warm run), and the fastest is kept. The
 * parameters are saved before and restored after the trials, so the state
 * of the context is unchanged. Allocates a temporary copy of v, P, Lambda,
 * log|det P|^2 and the flags. */
fca_status fca_autotune(fca_ctx *c, int32_t iters);

/* Capture one whole step into a HIP graph owned by the context: optionally
 * (with_reset != 0) the reset of every mixture to its start as fca_reset
 * does (without its host-side definiteness check, already done when the
 * start was set), `iters` EM iterations of the active mixtures, then the
 * requested outputs, laid out as for fca_em_step and fca_separate: loglik
 * [B][iters] (iters = 0: [B][1]), R_out, v_out, x_out. Every output must be
 * a DEVICE pointer (or NULL) and stay valid while the graph is used. Nothing
 * runs at capture. A new capture replaces the previous graph. */
fca_status fca_graph_capture(fca_ctx *c, int32_t iters, int32_t with_reset, double *loglik, double *R_out,
                             void *v_out, void *x_out);

/* Replay the captured step `count` >= 1 times back to back on the context's
 * stream and wait for them; returns FCA_E_NOT_PD / FCA_E_NONFINITE as
 * fca_em_step does. FCA_E_STATE when nothing is captured or when the active
 * mixtures, launch shapes or kinds of start changed since the capture. */
fca_status fca_graph_launch(fca_ctx *c, int32_t count);

/* ------------------------------------------------------------------
 * Learned initial powers (optional; not part of the paper's method).
 * A per-bin MLP predicts r = v1 / (v1 + v2) from features of y(n,f):
 * log(|y_m|^2 + 1e-20) for each microphone, cos and sin of the phase of y_m
 * relative to microphone 1 (m = 2..M), and f / (F - 1) (IN = 3M - 1 values,
 * zero-padded to 32). Three hidden layers of width H (32, 64, 128 or 256) with
 * GELU, one sigmoid output; BF16 weights and activations into MFMA, FP32
 * accumulation, FP32 master weights, AdamW; loss = mean binary cross-
 * entropy against soft targets. The learned start is
 * v_j^(0) = (r, 1 - r) * 2 ||y||^2 / M (r = 1/2 gives the plain start) and
 * reaches the EM only through fca_problem.v0. The forward GELU is
 * max(x, 0) - t P(t), t = min(|x|, 4), with P a fitted degree-6 polynomial
 * (|error| <= 2.1e-4 against x Phi(x)); the backward uses the exact GELU's
 * derivative. The network costs about 2 (32 H + 2 H^2 + H) flop and 3 H
 * GELUs per bin: at M = 4 the EM spends about 500 flop per bin and
 * iteration, so H = 256 costs as much as tens of EM iterations, H = 64
 * about ten times less and H = 32 about half of H = 64.
 * Parameter vector (fp32, flat): for each hidden layer l = 1..3 its weight
 * [H][in_l] (in_1 = 32, the padded input; in_2 = in_3 = H) then its bias
 * [H]; then the output weight [H] and bias [1].
 * Every array argument below is a DEVICE pointer unless marked host; y of
 * fca_mlp_forward/backward is [n][M] complex64, fpos/target/r are [n] float.
 * ------------------------------------------------------------------ */
typedef struct fca_mlp fca_mlp;

/* max_batch: largest n of one forward/backward call, a multiple of 64.
 * 2 <= M <= 8; hidden (H) is 32, 64, 128 or 256, else FCA_E_ARG. Weights are
 * initialised from seed. All work runs on `stream`. */
fca_status fca_mlp_create(int32_t M, int32_t hidden, uint64_t seed, int32_t max_batch, void *stream, fca_mlp **out);
void fca_mlp_destroy(fca_mlp *m);
int64_t fca_mlp_num_params(const fca_mlp *m);
const char *fca_mlp_last_error(const fca_mlp *m);
/* host params [num_params] */
fca_status fca_mlp_get_params(fca_mlp *m, float *params);
fca_status fca_mlp_set_params(fca_mlp *m, const float *params);
/* r_out[b] = sigmoid(network(features(y[b], fpos[b]))), 1 <= n <= max_batch */
fca_status fca_mlp_forward(fca_mlp *m, const float *y, const float *fpos, int32_t n, float *r_out);
/* forward + backward of the mean loss; keeps the gradient for fca_mlp_adamw;
 * loss (host, may be NULL) and grads_out (host [num_params], may be NULL).
 * n a multiple of 64, 64 <= n <= max_batch. */
fca_status fca_mlp_backward(fca_mlp *m, const float *y, const float *fpos, const float *target, int32_t n,
                            double *loss, float *grads_out);
/* one AdamW step with the last gradient (bias-corrected moments) */
fca_status fca_mlp_adamw(fca_mlp *m, float lr, float beta1, float beta2, float eps, float weight_decay);
/* Learned starts straight from the mixtures a context already holds: for
 * each listed mixture (mixtures = NULL: mixtures 0..count-1) the network's
 * v_j^(0) becomes its stored start (as fca_set_start with that v0 and the
 * plain R would make it), and the mixture is reset to it and made active.
 * One inference launch reads the context's copy of y and writes the stored
 * and the working powers; enqueued on the context's stream (after the
 * network's stream). FCA_E_ARG for an FP64 context, a mixture index out of
 * range or a mixture whose M differs from the network's. */
fca_status fca_set_learned_starts(fca_ctx *c, fca_mlp *m, int32_t count, const int32_t *mixtures);
/* Initial spatial covariances from time-frequency masks (the experiments of
 * Section 4 start from covariances estimated with masks; the paper gives no
 * formula, this is the plain mask-weighted estimate). For each listed
 * mixture (mixtures: host array of count indices, or NULL for mixtures
 * 0..count-1) the masks come from its
 * stored powers v_j^(0) (e.g. a learned start): r = v1 / (v1 + v2) (1/2
 * where both are 0), sharpened to r^p / (r^p + (1 - r)^p) with p = sharpen,
 * w_1 = r, w_2 = 1 - r. Then A_j(f) = sum_n w_j y y^H (FP64 sums) and
 * R_j^(0)(f) = M A_j / tr(A_j) + load I ((1 + load) I where tr(A_j) = 0).
 * These become the stored R start (the powers stay), the initial
 * decomposition is recomputed, and the mixture is reset and made active.
 * With one microphone R_j^(0) = 1 + load for both sources. A listed mixture
 * whose stored powers are the plain start (equal powers: every mask would be
 * 1/2, so R1 = R2, a fixed point of the EM) gives FCA_E_ARG; its powers must
 * come from v0, fca_set_start or fca_set_learned_starts.
 * 1 <= sharpen <= 64, 0 < load <= 1e6, else FCA_E_ARG. If a decomposition
 * fails (FCA_E_NOT_PD) every listed mixture gets the default R back and is
 * still reset. Waits for the context's stream. A later fca_set_start without
 * R0, or fca_set_learned_starts, puts the default R back. */
fca_status fca_set_mask_covariances(fca_ctx *c, int32_t count, const int32_t *mixtures, double sharpen, double load);
/* learned start for a mixture y [F][N][M] complex64 (contiguous, device):
 * v0_out [2][F][N] float (device), usable as fca_problem.v0. One fused
 * kernel, enqueued on the network's stream without waiting: v0_out is
 * complete in that stream's order (a context created on the same stream
 * may take it at once; other users synchronise first). */
fca_status fca_mlp_init_powers(fca_mlp *m, const float *y, int32_t F, int32_t N, float *v0_out);
/* the same for `count` mixtures in one launch (a fixed number of bins per
 * workgroup, so many small mixtures fill the GPU as one large one does):
 * ys[i] (device, [F][Ns[i]][M] complex64) gives v0s[i] (device,
 * [2][F][Ns[i]] float). ys, Ns and v0s are host arrays of length count; the
 * call copies them, so they may be reused once it returns. Enqueued on the
 * network's stream like fca_mlp_init_powers; FCA_E_ARG on count < 1, F < 1,
 * a null buffer or Ns[i] < 1. */
fca_status fca_mlp_init_powers_batch(fca_mlp *m, int32_t count, const float *const *ys, int32_t F,
                                     const int32_t *Ns, float *const *v0s);

#ifdef __cplusplus
}
#endif

#endif /* FCA_H */
