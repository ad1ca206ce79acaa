// fca_noalloc.hip -- fca_em_solve_noalloc: the plain-start EM of one mixture
// (Algorithm 1, steps 1 and 3-9) without any device allocation.
//
// fca_init + fca_em_step keep the per-frequency state (the basis P and the
// eigenvalues, log|det P|^2, status flags, the per-problem log-likelihood
// rows, the problem table) in buffers the context allocates. This variant
// keeps the same state in one file-scope device array, `scratch`, of fixed
// size, and reads y and the powers in place from the caller's buffers, so a
// caller that cannot allocate (a captured stream, a serving loop) can run
// the iterations. The kernels are the context path's: the results equal
// fca_init (plain R) + fca_em_step for the same y, start and launch shape.
//
// Each device holds its own copy of the array; its address is taken once
// per device with hipGetSymbolAddress (in host code the array's name is not
// a device address). Calls on one device share the array: calls that overlap
// in time on one GPU (two streams, two threads) race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "fca.h"
#include "fca_internal.h"

namespace fca {
namespace {

constexpr int kNaMaxF = 2048;      // frequencies per call
constexpr int kNaRows = 128;       // iterations per launch (log-likelihood rows)
constexpr int kNaMaxDevices = 64;

// Carving of the array into the per-call state (byte offsets, 256-aligned).
constexpr int64_t al(int64_t x) { return (x + 255) / 256 * 256; }
constexpr int64_t kOffP = 0;                                                           // double2 [F][kMaxM^2]
constexpr int64_t kOffLam = al(kOffP + (int64_t)kNaMaxF * kMaxM * kMaxM * 16);        // double [F][kMaxM]
constexpr int64_t kOffLogdet = al(kOffLam + (int64_t)kNaMaxF * kMaxM * 8);            // double [F]
constexpr int64_t kOffFlags = al(kOffLogdet + (int64_t)kNaMaxF * 8);                  // int [F]
constexpr int64_t kOffLL = al(kOffFlags + (int64_t)kNaMaxF * 4);                      // double [kNaRows][F]
constexpr int64_t kOffLLTot = al(kOffLL + (int64_t)kNaRows * kNaMaxF * 8);            // double [kNaRows]
constexpr int64_t kOffFsum = al(kOffLLTot + (int64_t)kNaRows * 8);                    // double [F + 1]
constexpr int64_t kOffR0 = al(kOffFsum + (int64_t)(kNaMaxF + 1) * 8);                 // double2 [2][M][M]
constexpr int64_t kOffProbs = al(kOffR0 + 2 * kMaxM * kMaxM * 16);                    // EmProblem [F]
constexpr int64_t kScratchBytes = al(kOffProbs + (int64_t)kNaMaxF * sizeof(EmProblem));

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
unsigned char* g_ptr[kNaMaxDevices] = {};

// The device address of this device's scratch array (taken once per device).
hipError_t scratch_ptr(unsigned char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNaMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

// The problem table of one mixture in the caller's layout: y[f][m][pitch],
// powers [j][f][pitch].
__global__ void na_problems_kernel(EmProblem* __restrict__ probs, int F, int M, int N, int pitch) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    EmProblem p;
    p.y_off = (int64_t)f * M * pitch;
    p.v_off = (int64_t)f * pitch;
    p.v2_off = (int64_t)F * pitch;
    p.n = N;
    p.npad = pitch;
    p.pid = f;
    p.m = M;
    probs[f] = p;
}

// The exported status bits (low byte) of every frequency.
__global__ void na_flags_out_kernel(const int* __restrict__ flags, int F, int32_t* __restrict__ out) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < F) out[f] = flags[f] & kFlagBitsMask;
}

bool on_device(const void* p) {
    hipPointerAttribute_t a;
    if (!p || hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged || a.isManaged;
}

fca_status arg_error(const char* msg) {
    set_global_error(msg);
    return FCA_E_ARG;
}

}  // namespace
}  // namespace fca

extern "C" fca_status fca_em_solve_noalloc(int32_t M, int32_t F, int32_t N, int32_t prec, const void* y,
                                           int64_t pitch, void* v, int32_t use_v0, int32_t iters,
                                           double* loglik, double* R_out, int32_t* flags_out, void* stream) {
    using namespace fca;
    if (M < 1 || M > kMaxM) return arg_error("fca_em_solve_noalloc: need 1 <= M <= 8");
    if (F < 1 || F > kNaMaxF) return arg_error("fca_em_solve_noalloc: need 1 <= F <= 2048 (the scratch limit)");
    if (N < 1 || N > kMaxFrames)
        return arg_error("fca_em_solve_noalloc: need 1 <= N <= 2048 (frames held in registers)");
    if (prec != FCA_FP64 && prec != FCA_FP32_BULK) return arg_error("fca_em_solve_noalloc: unknown precision");
    if (pitch < N || pitch > (1 << 30)) return arg_error("fca_em_solve_noalloc: need N <= pitch <= 2^30");
    if (iters < 0) return arg_error("fca_em_solve_noalloc: iters < 0");
    if (!on_device(y) || !on_device(v)) return arg_error("fca_em_solve_noalloc: y and v must be device pointers");
    if ((loglik && !on_device(loglik)) || (R_out && !on_device(R_out)) || (flags_out && !on_device(flags_out)))
        return arg_error("fca_em_solve_noalloc: outputs must be device pointers (or NULL)");
    unsigned char* base = nullptr;
    hipError_t e = scratch_ptr(&base);
    if (e != hipSuccess) {
        set_global_error("fca_em_solve_noalloc: hipGetSymbolAddress failed");
        return FCA_E_DEVICE;
    }
    double2* P = reinterpret_cast<double2*>(base + kOffP);
    double* lam = reinterpret_cast<double*>(base + kOffLam);
    double* logdet = reinterpret_cast<double*>(base + kOffLogdet);
    int* flags = reinterpret_cast<int*>(base + kOffFlags);
    double* ll = reinterpret_cast<double*>(base + kOffLL);
    double* ll_tot = reinterpret_cast<double*>(base + kOffLLTot);
    double* fsum = reinterpret_cast<double*>(base + kOffFsum);
    double2* R0 = reinterpret_cast<double2*>(base + kOffR0);
    EmProblem* probs = reinterpret_cast<EmProblem*>(base + kOffProbs);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const bool fp64 = prec == FCA_FP64;
    const int64_t mm = (int64_t)M * M;
    int fpt = 1;
    while (fpt * kEmThreads < N) fpt *= 2;

#define NA_HIP(call)                                                                   \
    do {                                                                               \
        if ((e = (call)) != hipSuccess) {                                              \
            set_global_error("fca_em_solve_noalloc: " #call " failed");                \
            return FCA_E_DEVICE;                                                       \
        }                                                                              \
    } while (0)
    // step 1: plain start (R1 = I, R2 = I + 0.5 e1 e1^H; v = ||y||^2 / M
    // floored, unless the caller's v holds v0), one pencil for every frequency
    na_problems_kernel<<<(F + 255) / 256, 256, 0, s>>>(probs, F, M, N, (int)pitch);
    NA_HIP(hipGetLastError());
    if (!use_v0) {
        NA_HIP(launch_power_sums(fp64, y, M, F, N, (int)pitch, fsum, s));
        NA_HIP(launch_default_v(fp64, y, fsum, M, F, N, (int)pitch, v, s));
    }
    NA_HIP(launch_default_R(M, 1, R0, s));
    NA_HIP(launch_gevd(M, F, R0, R0 + mm, 0, 0, P, kMaxM * kMaxM, lam, kMaxM, logdet, flags, s));
    NA_HIP(launch_fill_u32(flags, 0u, F, s));  // the plain start's decomposition cannot fail
    // steps 3-9 in launches of at most kNaRows iterations
    int done = 0;
    do {
        const int chunk = iters == 0 ? 0 : std::min(kNaRows, iters - done);
        const int rows = chunk > 0 ? chunk : 1;
        NA_HIP(launch_em(M, fp64, kEmThreads, fpt, probs, F, y, v, 0, P, lam, logdet, flags, ll, F, chunk, done,
                         s));
        if (loglik) {
            NA_HIP(launch_ll_reduce(ll, F, rows, 1, F, ll_tot, s));
            NA_HIP(hipMemcpyAsync(loglik + done, ll_tot, rows * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        done += chunk;
    } while (done < iters);
    if (R_out) NA_HIP(launch_recover_R(M, F, P, lam, reinterpret_cast<double2*>(R_out),
                                       reinterpret_cast<double2*>(R_out) + F * mm, s));
    if (flags_out) {
        na_flags_out_kernel<<<(F + 255) / 256, 256, 0, s>>>(flags, F, flags_out);
        NA_HIP(hipGetLastError());
    }
#undef NA_HIP
    return FCA_OK;
}
