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
// L = 1024, the experiments' frame length, has the register-resident path
// of the fft1024 section below. Other frame lengths: one workgroup
// transforms one frame of one channel: the windowed samples
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

// ------------------------------------------------------------ L = 1024
// The frame length of the experiments takes a register-resident path. The
// 1024-point DFT is split as 32 x 32: with t = l + 32 k' and bin
// k = k1 + 32 k2, X[k] = sum_l W32^(l k2) W1024^(l k1) sum_k' z[l + 32 k'] W32^(k' k1),
// so 32 lanes each run a 32-point DFT in registers over k' (one lane per l),
// scale by W1024^(l k1), exchange through LDS and run the 32-point DFTs over
// l. Two real frames a, b share one complex transform of z = a + i b:
// A[f] = (Z[f] + conj Z[L - f]) / 2, B[f] = (Z[f] - conj Z[L - f]) / (2i);
// synthesis packs Z = A + i B over the Hermitian extension the same way and
// takes a and b as the real and imaginary parts of one inverse transform.
//
// A workgroup owns kQ transforms (kQ x complex size = 128 B) that are
// consecutive in the flattened (frame, channel) index q = n M + m, the
// fastest index of the spectrum layout X[f][q]: every bin row it reads or
// writes is one contiguous 128-byte segment.
namespace fft1024 {

constexpr int kL = 1024, kS = 512, kF = 513;
constexpr int kRegion = 1060;      // complex elements of LDS per transform pair (32 x 33 exchange; 8 dwords of bank offset)
constexpr int kStage = 516;        // complex elements per staged spectrum (synthesis)

template <typename T>
struct alignas(2 * sizeof(T)) Cx {
    T x, y;
};

// kQ transforms per block, kThreads = 32 per transform pair; kLdsTw: the
// 32 x 32 inter-pass roots are copied to LDS once per workgroup (FP32; in
// FP64 the 16 KiB would halve the resident workgroups, so they are read from
// the constant table)
template <typename T> struct Shape;
// kPrefetchSyn: synthesis loads the next block's bins into registers while
// the current one is transformed (FP32; in FP64 the registers do not
// suffice; analysis measured faster without). kWaves: waves per SIMD that
// the LDS lets reside (two workgroups per CU), the register budget.
template <> struct Shape<float> {
    static constexpr int kQ = 16, kThreads = 256, kWaves = 2;
    static constexpr bool kLdsTw = true, kPrefetchSyn = true;
};
template <> struct Shape<double> {
    static constexpr int kQ = 8, kThreads = 128, kWaves = 1;
    static constexpr bool kLdsTw = false, kPrefetchSyn = false;
};

constexpr double kPi = 3.141592653589793238462643383279502884;

// sin and cos of |x| <= pi/4 from their Taylor series (the x^31 term is below 1e-35)
constexpr void sincos_small(double x, double& s, double& c) {
    const double x2 = x * x;
    double t = x, acc = 0.0;
    for (int n = 1; n < 32; n += 2) {
        acc += t;
        t *= -x2 / (double)((n + 1) * (n + 2));
    }
    s = acc;
    t = 1.0;
    acc = 0.0;
    for (int n = 0; n < 32; n += 2) {
        acc += t;
        t *= -x2 / (double)((n + 1) * (n + 2));
    }
    c = acc;
}

// exp(-2 pi i k / n), 0 <= k < n, n divisible by 8: the angle is reduced to
// [0, pi/4] exactly by the symmetries of the quadrants and the octant.
constexpr void root(int k, int n, double& re, double& im) {
    const int q = 4 * k / n, r = k - q * (n / 4);
    double s = 0.0, c = 0.0;
    if (8 * r <= n) {
        sincos_small(2.0 * kPi * r / n, s, c);
    } else {
        sincos_small(2.0 * kPi * (n / 4 - r) / n, c, s);
    }
    for (int i = 0; i < q; ++i) {      // a quarter turn: (cos, sin) -> (-sin, cos)
        const double t = c;
        c = -s;
        s = t;
    }
    re = c;
    im = -s;
}

template <typename T>
struct Tables {
    Cx<T> w[kL];      // exp(-2 pi i k / 1024)
    Cx<T> tw[32][32]; // tw[k1][l] = exp(-2 pi i l k1 / 1024): lane l reads row k1 contiguously
    T win[kL];        // sin(pi t / 1024) = -Im exp(-2 pi i t / 2048)
};

template <typename T>
constexpr Tables<T> make_tables() {
    Tables<T> t{};
    for (int k = 0; k < kL; ++k) {
        double re = 0.0, im = 0.0;
        root(k, kL, re, im);
        t.w[k].x = (T)re;
        t.w[k].y = (T)im;
        root(k, 2 * kL, re, im);
        t.win[k] = (T)(-im);
        root((k >> 5) * (k & 31), kL, re, im);
        t.tw[k >> 5][k & 31].x = (T)re;
        t.tw[k >> 5][k & 31].y = (T)im;
    }
    return t;
}

template <typename T> __device__ constexpr Tables<T> kTab = make_tables<T>();

template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> w) {
    return Cx<T>{a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x};
}

// exp(-+ 2 pi i k / 1024): forward (Inv = false) or inverse root
template <bool Inv, typename T>
__device__ __forceinline__ Cx<T> rt(int k) {
    const Cx<T> w = kTab<T>.w[k];
    return Inv ? Cx<T>{w.x, -w.y} : w;
}

__device__ __forceinline__ constexpr int br5(int k) {
    return ((k & 1) << 4) | ((k & 2) << 2) | (k & 4) | ((k & 8) >> 2) | ((k & 16) >> 4);
}

// In-register 32-point DFT, decimation in frequency: natural-order input
// d[k], output bin k in d[br5(k)]. Every root index is a compile-time
// constant after unrolling (read from the table at compile time).
template <bool Inv, typename T>
__device__ __forceinline__ void dft32(Cx<T> (&d)[32]) {
#pragma unroll
    for (int h = 16; h >= 1; h >>= 1) {
#pragma unroll
        for (int g = 0; g < 32; g += 2 * h) {
#pragma unroll
            for (int j = 0; j < h; ++j) {
                const Cx<T> a = d[g + j], b = d[g + j + h];
                d[g + j] = Cx<T>{a.x + b.x, a.y + b.y};
                const Cx<T> e{a.x - b.x, a.y - b.y};
                const int k = j * (kS / h);           // W_{2h}^j = root j * 1024 / (2h)
                if (k == 0) {
                    d[g + j + h] = e;
                } else if (k == kL / 4) {              // -i (forward) or +i (inverse)
                    d[g + j + h] = Inv ? Cx<T>{-e.y, e.x} : Cx<T>{e.y, -e.x};
                } else {
                    d[g + j + h] = cmul(e, rt<Inv, T>(k));
                }
            }
        }
    }
}

// d holds z[l + 32 k'] (k' = 0..31) of this lane's transform; on return the
// lane (as r = l) holds Z[r + 32 k2] in d[br5(k2)]. E: the pair's exchange
// region; twl: the roots in LDS (LdsTw) laid out as [k1][l]. All lanes of
// the workgroup take part (two __syncthreads).
template <bool Inv, bool LdsTw, typename T>
__device__ __forceinline__ void fft1024(Cx<T> (&d)[32], Cx<T>* E, const Cx<T>* twl, const Tables<T>* tab, int l) {
    dft32<Inv, T>(d);
#pragma unroll
    for (int k1 = 0; k1 < 32; ++k1) {
        const Cx<T> v = d[br5(k1)];
        const Cx<T> w = LdsTw ? twl[k1 * 32 + l] : tab->tw[k1][l];
        E[k1 * 33 + l] = k1 == 0 ? v : cmul(v, Inv ? Cx<T>{w.x, -w.y} : w);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 32; ++j) d[j] = E[l * 33 + j];
    dft32<Inv, T>(d);
    __syncthreads();                                   // the exchange region is read out
}

template <typename T>
constexpr size_t lds_bytes() {
    return ((size_t)(Shape<T>::kQ / 2) * kRegion + (Shape<T>::kLdsTw ? 1024 : 0)) * sizeof(Cx<T>);
}

// Persistent workgroups in an XCD-aware order: workgroup w runs on XCD w % 8
// (round-robin dispatch), so the blocks are cut into 8 contiguous shares and
// the workgroups of one XCD walk their share side by side: the blocks in
// flight on one XCD are neighbours (shared frame edges hit its L2; the bin
// rows are written and read as long contiguous runs). gridDim.x is a
// multiple of 8.
struct Share {
    int64_t begin, end, step;
};
__device__ __forceinline__ Share xcd_share(int64_t nblk) {
    const int64_t per = (nblk + 7) / 8;
    const int64_t b = (int64_t)(blockIdx.x & 7) * per;
    const int64_t e = b + per < nblk ? b + per : nblk;
    return Share{b + (blockIdx.x >> 3), e, (int64_t)(gridDim.x >> 3)};
}

// The constant tables, seen as a fresh pointer in every block iteration so
// that their loads stay next to their uses (not hoisted out of the loop into
// registers that the FP64 transform needs).
template <typename T>
__device__ __forceinline__ const Tables<T>* tables() {
    const Tables<T>* t = &kTab<T>;
    asm volatile("" : "+s"(t));
    return t;
}

__device__ __forceinline__ int64_t div_small(int64_t a, int M, bool narrow) {
    return narrow ? (int64_t)((uint32_t)a / (uint32_t)M) : a / M;
}

template <typename T, bool LdsTw>
__device__ __forceinline__ void copy_roots(Cx<T>* twl) {
    if (LdsTw)
        for (int k = threadIdx.x; k < 1024; k += Shape<T>::kThreads) twl[k] = kTab<T>.tw[k >> 5][k & 31];
}

// X[f][q] for blocks of kQ transforms q = n M + m (nq = N M), f <= 512.
template <typename T>
__global__ __launch_bounds__(Shape<T>::kThreads) __attribute__((amdgpu_waves_per_eu(Shape<T>::kWaves))) void stft1024_kernel(const T* __restrict__ x, int64_t T_len, int M,
                                                                      int64_t nq, Cx<T>* __restrict__ X) {
    constexpr int kQ = Shape<T>::kQ, kThreads = Shape<T>::kThreads;
    constexpr bool kLdsTw = Shape<T>::kLdsTw;
    extern __shared__ __align__(16) unsigned char smem[];
    Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
    Cx<T>* twl = lds + (kQ / 2) * kRegion;
    const Share sh = xcd_share((nq + kQ - 1) / kQ);
    if (sh.begin >= sh.end) return;                    // the whole workgroup
    const int p = threadIdx.x >> 5, l = threadIdx.x & 31;
    const bool narrow = nq <= 0xffffffffLL;
    copy_roots<T, kLdsTw>(twl);
    __syncthreads();                                   // roots in LDS
    // edge frames: loads from clamped indices, unconditionally; samples outside the signal count as zero
    auto clamp = [&](int64_t s1) { return s1 < 0 ? 0 : (s1 < T_len ? s1 : T_len - 1); };
    const T half = (T)0.5;
    const int oi = threadIdx.x % kQ;                   // output transform of this thread (kThreads is a multiple of kQ)
    const bool odd = oi & 1;
    constexpr int kFStep = kThreads / kQ;
    for (int64_t blk = sh.begin; blk < sh.end; blk += sh.step) {
        const Tables<T>* tab = tables<T>();
        // real part: transform q0 + 2p, imaginary part: q0 + 2p + 1
        const int64_t qa = blk * kQ + 2 * p, qb = qa + 1;
        const int64_t ca = qa < nq ? qa : nq - 1, cb = qb < nq ? qb : nq - 1;
        const int64_t na = div_small(ca, M, narrow), nb = div_small(cb, M, narrow);
        const T* xa = x + (ca - na * M) * T_len;
        const T* xb = x + (cb - nb * M) * T_len;
        const int64_t sa = na * kS - kS, sb = nb * kS - kS;
        Cx<T> d[32];
        if (qb < nq && sa >= 0 && sa + kL <= T_len && sb >= 0 && sb + kL <= T_len) {   // both frames inside
            const T* pa = xa + sa + l;
            const T* pb = xb + sb + l;
#pragma unroll
            for (int k = 0; k < 32; ++k) {
                const T w = tab->win[l + 32 * k];
                d[k].x = w * pa[32 * k];
                d[k].y = w * pb[32 * k];
            }
        } else {
            const bool va = qa < nq, vb = qb < nq;
#pragma unroll
            for (int k = 0; k < 32; ++k) {
                const int64_t s1 = sa + l + 32 * k, s2 = sb + l + 32 * k;
                const bool in1 = va && s1 >= 0 && s1 < T_len, in2 = vb && s2 >= 0 && s2 < T_len;
                const T w = tab->win[l + 32 * k];
                const T y1 = xa[clamp(s1)], y2 = xb[clamp(s2)];
                d[k].x = in1 ? w * y1 : (T)0;
                d[k].y = in2 ? w * y2 : (T)0;
            }
        }
        Cx<T>* E = lds + p * kRegion;
        fft1024<false, kLdsTw, T>(d, E, twl, tab, l);
#pragma unroll
        for (int k2 = 0; k2 < 32; ++k2) E[l + 32 * k2] = d[br5(k2)];
        __syncthreads();
        // A = (Z[f] + conj Z[L - f]) / 2 (even oi), B = (Z[f] - conj Z[L - f]) / (2i) (odd oi)
        const int64_t q = blk * kQ + oi;
        if (q < nq) {
            const Cx<T>* Z = lds + (oi >> 1) * kRegion;
            Cx<T>* out = X + (int64_t)(threadIdx.x / kQ) * nq + q;
            const int64_t stride = (int64_t)kFStep * nq;
            for (int f = threadIdx.x / kQ; f < kF; f += kFStep, out += stride) {
                const Cx<T> zf = Z[f], zc = Z[(kL - f) & (kL - 1)];
                const T p1 = odd ? zf.y : zf.x, p2 = odd ? zc.y : zc.x;
                const T p3 = odd ? zc.x : zf.y, p4 = odd ? zf.x : zc.y;
                *out = Cx<T>{(p1 + p2) * half, (p3 - p4) * half};
            }
        }
        __syncthreads();                                 // the spectra are read out
    }
}

// Output blocks of QB consecutive q = j M + m (samples j S .. j S + S - 1
// of channel m: frame j's second half plus frame j + 1's first half, i.e.
// the transforms q and q + M). Local transforms of a block starting at b0:
// [b0, b0 + kQ) when M <= kQ/2 (QB = kQ - M), else [b0, b0 + kQ/2) and
// [b0 + M, b0 + M + kQ/2) (QB = kQ/2). The next block's bins are loaded
// while the current one is transformed.
template <typename T>
__global__ __launch_bounds__(Shape<T>::kThreads) __attribute__((amdgpu_waves_per_eu(Shape<T>::kWaves))) void istft1024_kernel(const Cx<T>* __restrict__ X, int64_t T_len,
                                                                       int M, int64_t nq, T* __restrict__ x) {
    constexpr int kQ = Shape<T>::kQ, kThreads = Shape<T>::kThreads;
    constexpr bool kLdsTw = Shape<T>::kLdsTw, kPrefetch = Shape<T>::kPrefetchSyn;
    constexpr int kPer = (kQ * kF + kThreads - 1) / kThreads;   // staged bins per thread
    constexpr int kOut = kS / kThreads;                          // output samples per thread and block
    extern __shared__ __align__(16) unsigned char smem[];
    Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
    Cx<T>* twl = lds + (kQ / 2) * kRegion;
    const bool split = M > kQ / 2;
    const int QB = split ? kQ / 2 : kQ - M;
    const int64_t nb = nq - M;                           // output blocks: j = 0 .. N - 2
    const Share sh = xcd_share((nb + QB - 1) / QB);
    if (sh.begin >= sh.end) return;
    const int p = threadIdx.x >> 5, l = threadIdx.x & 31;
    copy_roots<T, kLdsTw>(twl);
    T wlo[kOut], whi[kOut];
#pragma unroll
    for (int r = 0; r < kOut; ++r) {
        wlo[r] = kTab<T>.win[threadIdx.x + r * kThreads];
        whi[r] = kTab<T>.win[kS + threadIdx.x + r * kThreads];
    }
    // staged bins: this thread's transform si and bins f = sf + kFStep r
    constexpr int kFStep = kThreads / kQ;
    const int si = threadIdx.x % kQ, sf = threadIdx.x / kQ;
    auto local_q = [&](int64_t b0) -> int64_t { return split && si >= QB ? b0 + M + (si - QB) : b0 + si; };
    Cx<T> st[kPrefetch ? kPer : 1];
    auto issue = [&](int64_t blk) {
        const int64_t q = local_q(blk * QB);
        const Cx<T>* src = X + (int64_t)sf * nq + (q < nq ? q : nq - 1);
#pragma unroll
        for (int r = 0; r < kPer; ++r)
            if (sf + kFStep * r < kF) st[r] = src[(int64_t)kFStep * r * nq];
    };
    const T inv = (T)1 / (T)kL;
    int64_t blk = sh.begin;
    if (kPrefetch) issue(blk);
    for (;;) {
        const int64_t b0 = blk * QB;
        {
            const int64_t q = local_q(b0);
            const bool valid = q < nq;
            const Cx<T>* src = X + (int64_t)sf * nq + (valid ? q : nq - 1);
            Cx<T>* dst = lds + si * kStage + sf;
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                if (sf + kFStep * r < kF) {
                    const Cx<T> v = kPrefetch ? st[r] : src[(int64_t)kFStep * r * nq];
                    dst[kFStep * r] = valid ? v : Cx<T>{(T)0, (T)0};
                }
            }
        }
        __syncthreads();                                 // staged spectra (and, the first time, the roots)
        const int64_t nxt = blk + sh.step;
        const bool more = nxt < sh.end;
        if (kPrefetch && more) issue(nxt);
        Cx<T> d[32];
        {
            const Cx<T>* A = lds + (2 * p) * kStage;
            const Cx<T>* B = A + kStage;
#pragma unroll
            for (int k = 0; k < 32; ++k) {
                const int f = l + 32 * k;
                if (f <= kS) {                           // Z[f] = A[f] + i B[f]; DC and Nyquist taken real
                    Cx<T> a = A[f], b = B[f];
                    if (f == 0 || f == kS) {
                        a.y = (T)0;
                        b.y = (T)0;
                    }
                    d[k] = Cx<T>{a.x - b.y, a.y + b.x};
                } else {                                 // Z[f] = conj A[L - f] + i conj B[L - f]
                    const Cx<T> a = A[kL - f], b = B[kL - f];
                    d[k] = Cx<T>{a.x + b.y, b.x - a.y};
                }
            }
        }
        __syncthreads();                                 // the staged spectra are read out
        Cx<T>* E = lds + p * kRegion;
        fft1024<true, kLdsTw, T>(d, E, twl, tables<T>(), l);
#pragma unroll
        for (int k2 = 0; k2 < 32; ++k2) E[l + 32 * k2] = d[br5(k2)];
        __syncthreads();
        // block b0 + b: j = j0 + (m0 + b) / M without a division per block
        int64_t j = b0 / M;
        int m = (int)(b0 - j * M);
        for (int b = 0; b < QB; ++b) {
            if (b0 + b >= nb) break;
            const int i2 = split ? QB + b : b + M;       // local index of transform q + M (frame j + 1)
            const Cx<T>* Z1 = lds + (b >> 1) * kRegion;
            const Cx<T>* Z2 = lds + (i2 >> 1) * kRegion;
            T* xm = x + (int64_t)m * T_len;
#pragma unroll
            for (int r = 0; r < kOut; ++r) {
                const int u = threadIdx.x + r * kThreads;
                const int64_t s = j * kS + u;
                if (s < T_len) {
                    const Cx<T> z1 = Z1[kS + u], z2 = Z2[u];
                    const T a1 = (b & 1) ? z1.y : z1.x, a2 = (i2 & 1) ? z2.y : z2.x;
                    xm[s] = (whi[r] * a1 + wlo[r] * a2) * inv;
                }
            }
            if (++m == M) {
                m = 0;
                ++j;
            }
        }
        if (!more) break;
        __syncthreads();                                 // the time signals are read out
        blk = nxt;
    }
}

}  // namespace fft1024

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

// The L = 1024 path: persistent workgroups, as many as are resident at once
// (a multiple of 8, at most one per block rounded up to 8).
template <typename K>
hipError_t persistent_grid(K kernel, int threads, size_t lds, int64_t nblk, unsigned* grid) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds);
    if (e != hipSuccess) return e;
    int64_t g = (int64_t)(per_cu > 0 ? per_cu : 1) * cus;
    g = g / 8 * 8;
    const int64_t need = (nblk + 7) / 8 * 8;
    *grid = (unsigned)(g < 8 ? 8 : (g < need ? g : need));
    return hipSuccess;
}

template <typename T>
hipError_t launch_stft1024(const T* x, int64_t T_len, int M, int64_t N, void* X, hipStream_t s) {
    using namespace fft1024;
    const int64_t nq = N * M;
    const size_t lds = lds_bytes<T>();
    unsigned grid = 0;
    hipError_t e = allow_lds(stft1024_kernel<T>, lds);
    if (e == hipSuccess)
        e = persistent_grid(stft1024_kernel<T>, Shape<T>::kThreads, lds, (nq + Shape<T>::kQ - 1) / Shape<T>::kQ, &grid);
    if (e != hipSuccess) return e;
    stft1024_kernel<T><<<grid, Shape<T>::kThreads, lds, s>>>(x, T_len, M, nq, static_cast<Cx<T>*>(X));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_istft1024(const void* X, int64_t T_len, int M, int64_t N, T* x, hipStream_t s) {
    using namespace fft1024;
    constexpr int kQ = Shape<T>::kQ;
    const int64_t nq = N * M;
    const int QB = M > kQ / 2 ? kQ / 2 : kQ - M;
    const size_t lds = lds_bytes<T>();
    unsigned grid = 0;
    hipError_t e = allow_lds(istft1024_kernel<T>, lds);
    if (e == hipSuccess) e = persistent_grid(istft1024_kernel<T>, Shape<T>::kThreads, lds, (nq - M + QB - 1) / QB, &grid);
    if (e != hipSuccess) return e;
    istft1024_kernel<T><<<grid, Shape<T>::kThreads, lds, s>>>(static_cast<const Cx<T>*>(X), T_len, M, nq, x);
    return hipGetLastError();
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
    hipError_t e = hipSuccess;
    if (L == 1024) {
        e = prec == FCA_FP64 ? launch_stft1024<double>(static_cast<const double*>(x), T, M, N, X, s)
                             : launch_stft1024<float>(static_cast<const float*>(x), T, M, N, X, s);
    } else if (prec == FCA_FP64) {
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
    hipError_t e = hipSuccess;
    if (L == 1024) {
        e = prec == FCA_FP64 ? launch_istft1024<double>(X, T, M, N, static_cast<double*>(x), s)
                             : launch_istft1024<float>(X, T, M, N, static_cast<float*>(x), s);
    } else if (prec == FCA_FP64) {
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
