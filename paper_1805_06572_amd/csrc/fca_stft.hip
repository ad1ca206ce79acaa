// fca_stft.hip -- STFT analysis and overlap-add synthesis (the front and
// back end of the separation experiments of Section 4: frames of L samples,
// frame shift L/2, square-root Hann window; Table 1 uses L = 1024 at
// 16 kHz).
//
// Frame n of a signal of T samples holds samples n S - S + t (S = L/2,
// t = 0 .. L-1, zero outside the signal), weighted by w(t) = sin(pi t / L),
// the square root of the periodic Hann window; N = floor((T - 1) / S) + 2
// frames, so every sample lies in two frames and, since
// w(t)^2 + w(t + S)^2 = 1, synthesis with the same window reconstructs the
// signal exactly.
//
// One workgroup transforms one frame of one channel: the windowed samples
// are loaded in bit-reversed order into LDS and an in-place radix-2 FFT
// (twiddles exp(-2 pi i k / L) tabulated once per workgroup with sincospi)
// gives bins 0 .. L/2. Synthesis: one workgroup per block of S output
// samples and channel computes the inverse FFTs of the two frames that
// cover the block (over the Hermitian extension of bins 0 .. L/2, real part)
// and adds their windowed halves: deterministic, no atomics.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "fca.h"
#include "fca_internal.h"

namespace fca {
namespace {

constexpr int kStftThreads = 256;
constexpr int kStftMinL = 16, kStftMaxL = 4096;

template <typename T> struct C2;
template <> struct C2<float> { using t = float2; };
template <> struct C2<double> { using t = double2; };

template <typename T> __device__ __forceinline__ void sincospi_t(T x, T* s, T* c);
template <> __device__ __forceinline__ void sincospi_t<float>(float x, float* s, float* c) { sincospif(x, s, c); }
template <> __device__ __forceinline__ void sincospi_t<double>(double x, double* s, double* c) { sincospi(x, s, c); }

template <typename T> __device__ __forceinline__ T sinpi_t(T x);
template <> __device__ __forceinline__ float sinpi_t<float>(float x) { return sinpif(x); }
template <> __device__ __forceinline__ double sinpi_t<double>(double x) { return sinpi(x); }

__device__ __forceinline__ int bitrev(int i, int lg) { return (int)(__brev((unsigned)i) >> (32 - lg)); }

// tw[k] = exp(sign 2 pi i k / L), k < L/2
template <typename T>
__device__ void twiddles(typename C2<T>::t* tw, int L, T sign) {
    for (int k = threadIdx.x; k < L / 2; k += kStftThreads) {
        T s, c;
        sincospi_t<T>((T)(2 * k) / (T)L, &s, &c);
        tw[k].x = c;
        tw[k].y = sign * s;
    }
}

// In-place iterative radix-2 FFT of buf (input in bit-reversed order) with
// the twiddle table tw; __syncthreads between stages (and after the last).
template <typename T>
__device__ void fft_inplace(typename C2<T>::t* buf, const typename C2<T>::t* tw, int L) {
    using V = typename C2<T>::t;
    for (int len = 2; len <= L; len <<= 1) {
        const int half = len >> 1, step = L / len;
        for (int j = threadIdx.x; j < L / 2; j += kStftThreads) {
            const int g = j / half, pos = j - g * half;
            const int i0 = g * len + pos, i1 = i0 + half;
            const V w = tw[pos * step];
            const V u = buf[i0], v = buf[i1];
            V t;
            t.x = v.x * w.x - v.y * w.y;
            t.y = v.x * w.y + v.y * w.x;
            V a, b;
            a.x = u.x + t.x;
            a.y = u.y + t.y;
            b.x = u.x - t.x;
            b.y = u.y - t.y;
            buf[i0] = a;
            buf[i1] = b;
        }
        __syncthreads();
    }
}

// X[f][n][m] = sum_t w(t) x_m(n S - S + t) exp(-2 pi i f t / L), f <= L/2
template <typename T>
__global__ __launch_bounds__(kStftThreads) void stft_kernel(const T* __restrict__ x, int64_t T_len, int M, int L,
                                                            int lg, int N, typename C2<T>::t* __restrict__ X) {
    using V = typename C2<T>::t;
    extern __shared__ __align__(16) unsigned char smem[];
    V* buf = reinterpret_cast<V*>(smem);
    V* tw = buf + L;
    const int n = blockIdx.x, m = blockIdx.y, S = L / 2;
    twiddles<T>(tw, L, (T)-1);
    const T* xm = x + (int64_t)m * T_len;
    for (int t = threadIdx.x; t < L; t += kStftThreads) {
        const int64_t s = (int64_t)n * S - S + t;
        V v;
        v.x = (s >= 0 && s < T_len) ? sinpi_t<T>((T)t / (T)L) * xm[s] : (T)0;
        v.y = (T)0;
        buf[bitrev(t, lg)] = v;
    }
    __syncthreads();
    fft_inplace<T>(buf, tw, L);
    const int F = S + 1;
    for (int f = threadIdx.x; f < F; f += kStftThreads) X[((int64_t)f * N + n) * M + m] = buf[f];
}

// Output samples j S .. j S + S - 1 of channel m: the second half of frame j
// and the first half of frame j + 1, each the real part of the inverse DFT
// of the frame's Hermitian-extended spectrum, windowed.
template <typename T>
__global__ __launch_bounds__(kStftThreads) void istft_kernel(const typename C2<T>::t* __restrict__ X, int64_t T_len,
                                                             int M, int L, int lg, int N, T* __restrict__ x) {
    using V = typename C2<T>::t;
    extern __shared__ __align__(16) unsigned char smem[];
    V* buf = reinterpret_cast<V*>(smem);
    V* tw = buf + L;
    T* acc = reinterpret_cast<T*>(tw + L / 2);   // the block's S samples (each thread its own)
    const int j = blockIdx.x, m = blockIdx.y, S = L / 2, F = S + 1;
    twiddles<T>(tw, L, (T)1);
    const T inv = (T)1 / (T)L;
    for (int h = 0; h < 2; ++h) {
        const int n = j + 1 - h;    // h = 0: frame j + 1 (its first half); h = 1: frame j (its second half)
        __syncthreads();            // the previous transform is read out
        for (int k = threadIdx.x; k < L; k += kStftThreads) {
            V v;
            if (k < F) {
                v = X[((int64_t)k * N + n) * M + m];
            } else {
                v = X[((int64_t)(L - k) * N + n) * M + m];
                v.y = -v.y;
            }
            buf[bitrev(k, lg)] = v;
        }
        __syncthreads();
        fft_inplace<T>(buf, tw, L);
        const int off = h == 0 ? 0 : S;
        for (int u = threadIdx.x; u < S; u += kStftThreads) {
            const int t = u + off;
            const T part = sinpi_t<T>((T)t / (T)L) * buf[t].x * inv;
            acc[u] = h == 0 ? part : acc[u] + part;
        }
    }
    T* xm = x + (int64_t)m * T_len;
    for (int u = threadIdx.x; u < S; u += kStftThreads) {
        const int64_t s = (int64_t)j * S + u;
        if (s < T_len) xm[s] = acc[u];
    }
}

bool on_dev(const void* p) {
    hipPointerAttribute_t a;
    if (!p || hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged || a.isManaged;
}

fca_status check_args(const char* who, int32_t M, int64_t T, int32_t L, int32_t prec, const void* in, const void* out,
                      int* lg) {
    char msg[160];
    if (M < 1 || T < 1 || L < kStftMinL || L > kStftMaxL || (L & (L - 1)) || (prec != FCA_FP64 && prec != FCA_FP32_BULK)) {
        snprintf(msg, sizeof msg, "%s: need M >= 1, T >= 1, L a power of two in [16, 4096] and a known precision", who);
        set_global_error(msg);
        return FCA_E_ARG;
    }
    const int64_t N = (T - 1) / (L / 2) + 2;
    if (N > (int64_t)1 << 30) {
        snprintf(msg, sizeof msg, "%s: too many frames", who);
        set_global_error(msg);
        return FCA_E_ARG;
    }
    if (!on_dev(in) || !on_dev(out)) {
        snprintf(msg, sizeof msg, "%s: input and output must be device pointers", who);
        set_global_error(msg);
        return FCA_E_ARG;
    }
    int g = 0;
    while ((1 << g) < L) ++g;
    *lg = g;
    return FCA_OK;
}

// Allow `lds` bytes of dynamic LDS (above 64 KiB for FP64 at L = 4096).
template <typename K>
hipError_t allow_lds(K kernel, size_t lds) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

}  // namespace
}  // namespace fca

extern "C" {

int64_t fca_stft_frames(int64_t T, int32_t L) {
    if (T < 1 || L < 2) return 0;
    return (T - 1) / (L / 2) + 2;
}

fca_status fca_stft(int32_t M, int64_t T, int32_t L, int32_t prec, const void* x, void* X, void* stream) {
    using namespace fca;
    int lg = 0;
    fca_status st = check_args("fca_stft", M, T, L, prec, x, X, &lg);
    if (st != FCA_OK) return st;
    const int N = (int)fca_stft_frames(T, L);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 grid(N, M);
    hipError_t e;
    if (prec == FCA_FP64) {
        const size_t lds = (size_t)(L + L / 2) * sizeof(double2);
        e = allow_lds(stft_kernel<double>, lds);
        if (e == hipSuccess) {
            stft_kernel<double><<<grid, kStftThreads, lds, s>>>(static_cast<const double*>(x), T, M, L, lg, N,
                                                               static_cast<double2*>(X));
            e = hipGetLastError();
        }
    } else {
        const size_t lds = (size_t)(L + L / 2) * sizeof(float2);
        e = allow_lds(stft_kernel<float>, lds);
        if (e == hipSuccess) {
            stft_kernel<float><<<grid, kStftThreads, lds, s>>>(static_cast<const float*>(x), T, M, L, lg, N,
                                                              static_cast<float2*>(X));
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess) {
        set_global_error("fca_stft: launch failed");
        return FCA_E_DEVICE;
    }
    return FCA_OK;
}

fca_status fca_istft(int32_t M, int64_t T, int32_t L, int32_t prec, const void* X, void* x, void* stream) {
    using namespace fca;
    int lg = 0;
    fca_status st = check_args("fca_istft", M, T, L, prec, X, x, &lg);
    if (st != FCA_OK) return st;
    const int N = (int)fca_stft_frames(T, L);
    const int blocks = (int)((T + L / 2 - 1) / (L / 2));
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 grid(blocks, M);
    hipError_t e;
    if (prec == FCA_FP64) {
        const size_t lds = (size_t)(L + L / 2) * sizeof(double2) + (size_t)(L / 2) * sizeof(double);
        e = allow_lds(istft_kernel<double>, lds);
        if (e == hipSuccess) {
            istft_kernel<double><<<grid, kStftThreads, lds, s>>>(static_cast<const double2*>(X), T, M, L, lg, N,
                                                                static_cast<double*>(x));
            e = hipGetLastError();
        }
    } else {
        const size_t lds = (size_t)(L + L / 2) * sizeof(float2) + (size_t)(L / 2) * sizeof(float);
        e = allow_lds(istft_kernel<float>, lds);
        if (e == hipSuccess) {
            istft_kernel<float><<<grid, kStftThreads, lds, s>>>(static_cast<const float2*>(X), T, M, L, lg, N,
                                                               static_cast<float*>(x));
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess) {
        set_global_error("fca_istft: launch failed");
        return FCA_E_DEVICE;
    }
    return FCA_OK;
}

}  // extern "C"
