// fca_internal.h -- declarations shared by the kernel translation unit and
// the host runtime of libfca (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fca.h"

namespace fca {

// Per-frequency status bits (the FCA_FLAG_* values of fca.h).
constexpr int kFlagNotPD = 1;
constexpr int kFlagNonFinite = 2;
constexpr int kFlagSweeps = 4;
constexpr int kFreezeMask = kFlagNotPD | kFlagNonFinite;
// Bits from kFlagIterShift up of a problem's flag word hold the iteration of
// the EM call (1-based, counted over the call's chunks) whose update froze
// the problem; the status bits exported to callers are the low byte.
constexpr int kFlagIterShift = 8;
constexpr int kFlagBitsMask = 0xFF;

// Largest microphone count; per-frequency state is stored with this stride.
constexpr int kMaxM = 8;
// Smallest power the float bulk mode keeps after an M-step: an all-zero bin
// roughly halves its powers at every iteration, and below this value the
// float d_i, their reciprocals and logarithms would leave the normal range
// (FLT_MIN is 1.2e-38). Double precision has no floor.
constexpr float kPowerFloorF32 = 1e-30f;

// Threads per workgroup of the per-frequency EM kernel, and the largest
// number of frames each thread keeps in registers.
constexpr int kEmThreads = 256;
constexpr int kMaxFramesPerThread = 8;
constexpr int kMaxFrames = kEmThreads * kMaxFramesPerThread;  // resident limit
// Frames per thread per chunk of the streaming EM kernel (more frames than
// kMaxFrames); such problems use frames-per-thread code 0 in a launch group.
constexpr int kStreamFramesPerThread = 2;
// Largest frame count accepted.
constexpr int kMaxFramesStream = 1 << 24;

// One EM problem = one (mixture, frequency) pair. All offsets are element
// offsets into the context's device arrays.
struct EmProblem {
    int64_t y_off;   // complex elements: start of y_int[f][m][0]; rows of npad
    int64_t v_off;   // prec reals: start of v1[f][0]; v2 follows at +v2_off
    int64_t v2_off;  // distance (elements) from v1 to v2 of the same bin
    int32_t n;       // frames
    int32_t npad;    // row pitch of y_int and v (>= n)
    int32_t pid;     // problem index into P, lam, logdet, flags, ll
    int32_t m;       // microphones (checked against the kernel's template M)
};

// Launchers. All return hipSuccess or the launch error. Every pointer is a
// device pointer.
// The EM-iteration kernels (fca_em.h), instantiated for workgroup sizes NT =
// kEmThreads (every problem) and 128 (resident problems of at most
// 128 * kMaxFramesPerThread frames). fpt: frames per thread of the resident
// kernel (1, 2, 4, 8; fpt * NT >= frames), or 0 for the streaming kernel
// (NT = kEmThreads only), whose second power buffer starts at v + v_alt.
template <int NT>
hipError_t launch_em_nt(int M, bool fp64, int fpt, const EmProblem* probs, int count, const void* y, void* v,
                        int64_t v_alt, double2* P, double* lam, double* logdet, int* flags, double* ll,
                        int64_t ll_stride, int iters, int it_base, hipStream_t s);

// Dispatch on nt (kEmThreads or 128); defined in fca_api.hip, which sees only
// the declaration above, so each instantiation lives in its own translation unit.
hipError_t launch_em(int M, bool fp64, int nt, int fpt, const EmProblem* probs, int count, const void* y,
                     void* v, int64_t v_alt, double2* P, double* lam, double* logdet, int* flags, double* ll,
                     int64_t ll_stride, int iters, int it_base, hipStream_t s);

// The conventional frame-wise EM (fca_conv.h; resident frames only, fpt in
// 1, 2, 4, 8, kEmThreads threads): per (M, T) launcher, instantiated in
// fca_conv_lo.hip and fca_conv_m5.hip .. fca_conv_m8.hip, and the dispatch
// on M and precision (fca_api.hip).
template <int M, typename T>
hipError_t launch_conv_fpt(int fpt, const EmProblem* probs, int count, const void* y, void* v, int64_t v_alt,
                           double2* P, double* lam, double* logdet, int* flags, double* ll, int64_t ll_stride,
                           int iters, int it_base, hipStream_t s);

// fpt 0: frames streamed (the powers double-buffered at v + v_alt elements).
hipError_t launch_conv_em(int M, bool fp64, int fpt, const EmProblem* probs, int count, const void* y,
                          void* v, int64_t v_alt, double2* P, double* lam, double* logdet, int* flags, double* ll,
                          int64_t ll_stride, int iters, int it_base, hipStream_t s);

// Support kernels (fca_kernels.hip).
// p[i] = val for count 32-bit words (a kernel, not a memset: graph-capturable).
hipError_t launch_fill_u32(void* p, uint32_t val, int64_t count, hipStream_t s);

// Segments of 32-bit words for launch_multi_copy: segment k copies
// end[k] - end[k-1] words from src[k] to dst[k] (src null: writes zeros);
// unused trailing segments repeat the last end.
struct WordSegs {
    static constexpr int kMax = 5;
    const uint32_t* src[kMax];
    uint32_t* dst[kMax];
    int64_t end[kMax];
};
// launch_multi_copy's split of the segments into 16-byte or 4-byte units
struct WordSegUnits {
    int64_t end[WordSegs::kMax];
    int vec[WordSegs::kMax];
};
hipError_t launch_multi_copy(const WordSegs& segs, hipStream_t s);

// One mixture of a fused learned-start inference (fca_mlp.hip): y element
// (f, n, microphone m) at y[f y_sf + n y_sn + m y_sm] (complex64); v_j(n,f)
// written to out[j o_sj + f o_sf + n] and, if out2 is not null, to out2 at
// the same offset. Its workgroups are [tile0, tile0 + ceil(F N / 128)).
struct MlpInferJob {
    const float2* y;
    float* out;
    float* out2;
    int64_t y_sf, y_sn, y_sm, o_sj, o_sf;
    int64_t tile0;
    int F, N;
};
// Enqueues the fused inference of network m for `count` jobs (host array,
// tile0 filled in here) on stream s, after the network's own stream.
hipError_t mlp_infer_jobs(fca_mlp* m, MlpInferJob* jobs, int count, hipStream_t s, const char** err);
int mlp_microphones(const fca_mlp* m);

// Text returned by fca_last_error(NULL) (calls without a context).
void set_global_error(const char* msg);

// NaN in base[r row_stride + list[i] b_stride + e] for r < rows, e < len and
// the `count` entries of the device index list (one launch).
hipError_t launch_nan_rows(double* base, int64_t row_stride, int rows, int64_t b_stride, int len, const int* list,
                           int count, hipStream_t s);

// out[0] = OR of flags[0..count), out[1] / out[2] = first index flagged
// kFlagNotPD / kFlagNonFinite, count if none (out: 3 device ints).
hipError_t launch_flag_summary(const int* flags, int count, int* out, hipStream_t s);

hipError_t launch_ingest(bool fp64, const void* src, int64_t sf, int64_t sn, int64_t sm, int M,
                         int F, int N, int npad, void* dst, hipStream_t s);

hipError_t launch_power_sums(bool fp64, const void* y, int M, int F, int N, int npad,
                             double* fsum, hipStream_t s);

// fsum holds F per-frequency power sums followed by one slot for the floor.
hipError_t launch_default_v(bool fp64, const void* y, double* fsum, int M, int F, int N,
                            int npad, void* v, hipStream_t s);

hipError_t launch_copy_v_in(bool fp64, const void* v0, int F, int N, int npad, void* v,
                            hipStream_t s);

hipError_t launch_gevd(int M, int count, const double2* A, const double2* B, int64_t stride_a,
                       int64_t stride_b, double2* P, int64_t stride_p, double* lam, int64_t stride_l,
                       double* logdet, int* flags, hipStream_t s);

// As launch_gevd for runs of `per` pencils: pencil i reads its inputs at
// (i / per) outer + (i % per) stride_a (stride_b) and writes P, lam, logdet,
// flags at index i.
hipError_t launch_gevd_runs(int M, int count, int per, int64_t outer, const double2* A, const double2* B,
                            int64_t stride_a, int64_t stride_b, double2* P, int64_t stride_p, double* lam,
                            int64_t stride_l, double* logdet, int* flags, hipStream_t s);

hipError_t launch_default_R(int M, int F, double2* R, hipStream_t s);

// Mask-weighted initial covariances (mask_cov_kernel) of `count` mixtures of
// M microphones (device table `mix`): y_int of a mixture at y_base (complex
// elements, [f][m][npad]), its stored powers at v_base (reals, [j][f][npad]),
// R_1 at R_base and R_2 at R_base + F M M (complex128, [f][M][M]).
struct MaskCovMix {
    int64_t y_base, v_base, R_base;
    int32_t N, npad;
};
hipError_t launch_mask_cov(bool fp64, int M, const MaskCovMix* mix, int count, int F, const void* y, const void* v,
                           double2* R, double p, double load, hipStream_t s);

hipError_t launch_ll_reduce(const double* ll, int64_t ll_stride, int iters, int B, int F,
                            double* out, hipStream_t s);

hipError_t launch_recover_R(int M, int count, const double2* P, const double* lam, double2* R1,
                            double2* R2, hipStream_t s);

// P^-1 of `count` problems (one wavefront each; stride kMaxM^2 like P) and,
// when R1 != NULL, R2 = (P P^H)^-1, R1 = P^-H Lambda P^-1 ([count][M][M]).
// Pinv may be NULL.
hipError_t launch_pinv(int M, int count, const double2* P, const double* lam, double2* Pinv, double2* R1,
                       double2* R2, hipStream_t s);

// MMSE images; Pinv holds P^-1 of every problem (launch_pinv).
hipError_t launch_separate(int M, bool fp64, const EmProblem* probs, int count, int max_n,
                           const void* y, const void* v, const double2* P, const double* lam,
                           const double2* Pinv, void* x, const int64_t* x_off, hipStream_t s);

}  // namespace fca
