// fca_kernels.hip -- gfx950 support kernels of the FastFCA EM library: input
// ingest, the plain start of v, the batched FP64 generalized eigendecomposition
// (initial values and fca_gevd), log-likelihood totals, recovery of R_j and
// the MMSE separation. The EM-iteration kernels are in fca_em.h.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fca_device.h"
#include "fca_internal.h"

namespace fca {

// ============================================================== ingest
// dst[f][m][n] (row pitch npad, zero padded) from the caller's strided y.
template <typename T2>
__global__ void ingest_kernel(const T2* __restrict__ src, int64_t sf, int64_t sn, int64_t sm, int M,
                              int F, int N, int npad, T2* __restrict__ dst) {
    const int64_t total = (int64_t)F * M * npad;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int n = (int)(i % npad);
        const int64_t fm = i / npad;
        const int m = (int)(fm % M);
        const int f = (int)(fm / M);
        T2 val;
        if (n < N) val = src[f * sf + n * sn + m * sm];
        else { val.x = 0; val.y = 0; }
        dst[i] = val;
    }
}

static unsigned grid_for(int64_t total, int block) {
    int64_t g = (total + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

hipError_t launch_ingest(bool fp64, const void* src, int64_t sf, int64_t sn, int64_t sm, int M,
                         int F, int N, int npad, void* dst, hipStream_t s) {
    const unsigned g = grid_for((int64_t)F * M * npad, 256);
    if (fp64)
        ingest_kernel<double2><<<g, 256, 0, s>>>(static_cast<const double2*>(src), sf, sn, sm, M, F, N, npad, static_cast<double2*>(dst));
    else
        ingest_kernel<float2><<<g, 256, 0, s>>>(static_cast<const float2*>(src), sf, sn, sm, M, F, N, npad, static_cast<float2*>(dst));
    return hipGetLastError();
}

// ============================================================== fill
// p[i] = val for i < count (32-bit words). Clears flags and marks log-
// likelihood rows with a kernel rather than a memset node, so that the same
// sequence can be captured into a HIP graph.
__global__ void fill_u32_kernel(uint32_t* __restrict__ p, uint32_t val, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

// Up to WordSegs::kMax copies of 32-bit words (src null: fill with zero) in
// one launch. Each segment is cut into units of 4 words (16-byte accesses)
// when both its addresses are 16-byte aligned, else of 1 word; the units of
// all segments form one index space.
__global__ void multi_copy_kernel(WordSegs segs, WordSegUnits u) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < u.end[WordSegs::kMax - 1]; i += stride) {
        int k = 0;
        while (i >= u.end[k]) ++k;
        const int64_t j = i - (k ? u.end[k - 1] : 0);
        const uint32_t* src = segs.src[k];
        uint32_t* dst = segs.dst[k];
        const int64_t n = segs.end[k] - (k ? segs.end[k - 1] : 0);
        if (u.vec[k]) {
            const int64_t w = 4 * j;
            if (w + 4 <= n) {
                const uint4 val = src ? *reinterpret_cast<const uint4*>(src + w) : make_uint4(0u, 0u, 0u, 0u);
                *reinterpret_cast<uint4*>(dst + w) = val;
            } else {
                for (int64_t q = w; q < n; ++q) dst[q] = src ? src[q] : 0u;
            }
        } else {
            dst[j] = src ? src[j] : 0u;
        }
    }
}

hipError_t launch_multi_copy(const WordSegs& segs, hipStream_t s) {
    WordSegUnits u{};
    int64_t acc = 0, prev = 0;
    for (int k = 0; k < WordSegs::kMax; ++k) {
        const int64_t n = segs.end[k] - prev;
        prev = segs.end[k];
        const bool al = (reinterpret_cast<uintptr_t>(segs.dst[k]) % 16 == 0) &&
                        (!segs.src[k] || reinterpret_cast<uintptr_t>(segs.src[k]) % 16 == 0);
        u.vec[k] = al ? 1 : 0;
        acc += al ? (n + 3) / 4 : n;
        u.end[k] = acc;
    }
    if (acc <= 0) return hipSuccess;
    const int64_t g = std::min<int64_t>((acc + 255) / 256, 8192);
    multi_copy_kernel<<<(unsigned)g, 256, 0, s>>>(segs, u);
    return hipGetLastError();
}

hipError_t launch_fill_u32(void* p, uint32_t val, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t g = std::min<int64_t>((count + 255) / 256, 4096);
    fill_u32_kernel<<<(unsigned)g, 256, 0, s>>>(static_cast<uint32_t*>(p), val, count);
    return hipGetLastError();
}

// Summary of the per-problem status flags: out[0] = their bitwise OR,
// out[1] / out[2] = the first problem flagged kFlagNotPD / kFlagNonFinite
// (count if none); out[3] / out[4] = the iteration recorded in their flag
// words (0 if none). One workgroup of kFlagThreads threads.
constexpr int kFlagThreads = 1024;
__global__ __launch_bounds__(kFlagThreads) void flag_summary_kernel(const int* __restrict__ flags, int count,
                                                                    int* __restrict__ out) {
    __shared__ int s_or[kFlagThreads], s_np[kFlagThreads], s_nf[kFlagThreads];
    const int t = threadIdx.x;
    int o = 0, np = count, nf = count;
    for (int i = t; i < count; i += kFlagThreads) {  // ascending: the first hit per thread is its minimum
        const int f = flags[i];
        o |= f;
        if ((f & kFlagNotPD) && np == count) np = i;
        if ((f & kFlagNonFinite) && nf == count) nf = i;
    }
    s_or[t] = o;
    s_np[t] = np;
    s_nf[t] = nf;
    __syncthreads();
    for (int w = kFlagThreads / 2; w >= 1; w >>= 1) {
        if (t < w) {
            s_or[t] |= s_or[t + w];
            s_np[t] = min(s_np[t], s_np[t + w]);
            s_nf[t] = min(s_nf[t], s_nf[t + w]);
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = s_or[0] & kFlagBitsMask;
        out[1] = s_np[0];
        out[2] = s_nf[0];
        out[3] = s_np[0] < count ? flags[s_np[0]] >> kFlagIterShift : 0;
        out[4] = s_nf[0] < count ? flags[s_nf[0]] >> kFlagIterShift : 0;
    }
}

__global__ void nan_rows_kernel(double* __restrict__ base, int64_t row_stride, int rows, int64_t b_stride, int len,
                                const int* __restrict__ list, int count) {
    const int64_t per = (int64_t)rows * len;
    const int64_t total = per * count;
    const double nan = __longlong_as_double(-1LL);   // all-ones bits
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(i / per);
        const int64_t rem = i - (int64_t)k * per;
        const int r = (int)(rem / len), e = (int)(rem - (int64_t)r * len);
        base[(int64_t)r * row_stride + (int64_t)list[k] * b_stride + e] = nan;
    }
}

hipError_t launch_nan_rows(double* base, int64_t row_stride, int rows, int64_t b_stride, int len, const int* list,
                           int count, hipStream_t s) {
    if (count <= 0 || rows <= 0 || len <= 0) return hipSuccess;
    nan_rows_kernel<<<grid_for((int64_t)count * rows * len, 256), 256, 0, s>>>(base, row_stride, rows, b_stride, len,
                                                                               list, count);
    return hipGetLastError();
}

hipError_t launch_flag_summary(const int* flags, int count, int* out, hipStream_t s) {
    flag_summary_kernel<<<1, kFlagThreads, 0, s>>>(flags, count, out);
    return hipGetLastError();
}

// ============================================================== plain start of v
// fsum[f] = sum_n ||y(n,f)||^2 / M (FP64, fixed order: per-thread strided sums,
// then a tree over the workgroup).
template <typename T2>
__global__ void power_sums_kernel(const T2* __restrict__ y, int M, int N, int npad, double* __restrict__ fsum) {
    __shared__ double red[256];
    const int f = blockIdx.x;
    double s = 0.0;
    for (int n = threadIdx.x; n < N; n += 256) {
        double p = 0.0;
        for (int m = 0; m < M; ++m) {
            const T2 val = y[((int64_t)f * M + m) * npad + n];
            p += (double)val.x * (double)val.x + (double)val.y * (double)val.y;
        }
        s += p / M;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) fsum[f] = red[0];
}

hipError_t launch_power_sums(bool fp64, const void* y, int M, int F, int N, int npad, double* fsum,
                             hipStream_t s) {
    if (fp64)
        power_sums_kernel<double2><<<F, 256, 0, s>>>(static_cast<const double2*>(y), M, N, npad, fsum);
    else
        power_sums_kernel<float2><<<F, 256, 0, s>>>(static_cast<const float2*>(y), M, N, npad, fsum);
    return hipGetLastError();
}

// floor = 1e-12 * mean over bins of ||y||^2 / M (1 if that mean is zero),
// from the per-frequency sums in a fixed order; stored at fsum[F].
__global__ void power_floor_kernel(double* __restrict__ fsum, int F, int N) {
    __shared__ double red[256];
    double s = 0.0;
    for (int g = threadIdx.x; g < F; g += 256) s += fsum[g];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mean = red[0] / ((double)F * (double)N);
        fsum[F] = mean > 0.0 ? 1e-12 * mean : 1.0;
    }
}

// v_j(n,f) = max(||y(n,f)||^2 / M, floor) for both sources; padding frames get 1.
template <typename T, typename T2>
__global__ void default_v_kernel(const T2* __restrict__ y, const double* __restrict__ fsum, int M, int F,
                                 int N, int npad, T* __restrict__ v) {
    const int f = blockIdx.y;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= npad) return;
    const double vfloor = fsum[F];
    double val = 1.0;
    if (n < N) {
        double p = 0.0;
        for (int m = 0; m < M; ++m) {
            const T2 yy = y[((int64_t)f * M + m) * npad + n];
            p += (double)yy.x * (double)yy.x + (double)yy.y * (double)yy.y;
        }
        val = p / M;
        if (!(val >= vfloor)) val = vfloor;
    }
    v[(int64_t)f * npad + n] = (T)val;
    v[((int64_t)F + f) * npad + n] = (T)val;
}

hipError_t launch_default_v(bool fp64, const void* y, double* fsum, int M, int F, int N, int npad,
                            void* v, hipStream_t s) {
    power_floor_kernel<<<1, 256, 0, s>>>(fsum, F, N);
    const dim3 grid((npad + 255) / 256, F);
    if (fp64)
        default_v_kernel<double, double2><<<grid, 256, 0, s>>>(static_cast<const double2*>(y), fsum, M, F, N, npad, static_cast<double*>(v));
    else
        default_v_kernel<float, float2><<<grid, 256, 0, s>>>(static_cast<const float2*>(y), fsum, M, F, N, npad, static_cast<float*>(v));
    return hipGetLastError();
}

template <typename T>
__global__ void copy_v_in_kernel(const T* __restrict__ v0, int F, int N, int npad, T* __restrict__ v) {
    const int64_t total = 2LL * F * npad;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int n = (int)(i % npad);
        const int64_t row = i / npad;
        v[i] = (n < N) ? v0[row * N + n] : T(1);
    }
}

hipError_t launch_copy_v_in(bool fp64, const void* v0, int F, int N, int npad, void* v, hipStream_t s) {
    const unsigned g = grid_for(2LL * F * npad, 256);
    if (fp64)
        copy_v_in_kernel<double><<<g, 256, 0, s>>>(static_cast<const double*>(v0), F, N, npad, static_cast<double*>(v));
    else
        copy_v_in_kernel<float><<<g, 256, 0, s>>>(static_cast<const float*>(v0), F, N, npad, static_cast<float*>(v));
    return hipGetLastError();
}

// ============================================================== batched GEVD
// One wavefront per pencil (A, B) at A + i*stride_a, B + i*stride_b, starting
// from the identity basis: P + i*stride_p receives Q (M x M), lam +
// i*stride_l the eigenvalues, logdet[i] = log|det Q|^2 = -log det B (if
// logdet is not null) and flags[i] the FCA flag bits. On failure P = I and
// lam = 1.
template <int M>
__global__ __launch_bounds__(64) void gevd_kernel(const double2* __restrict__ A, const double2* __restrict__ B,
                                                  int64_t stride_a, int64_t stride_b, int per, int64_t outer,
                                                  double2* __restrict__ P, int64_t stride_p,
                                                  double* __restrict__ lam, int64_t stride_l,
                                                  double* __restrict__ logdet, int* __restrict__ flags) {
    constexpr int MM = M * M;
    __shared__ double2 sA[MM], sB[MM], sId[MM], sPn[MM];
    __shared__ double sLam[M];
    __shared__ GevdScratch sWs;
    const int64_t i = blockIdx.x;
    const int tid = threadIdx.x;
    // pencil i of run i / per: its inputs at (i / per) outer + (i % per) stride
    const int64_t ia = (i / per) * outer + (i % per) * stride_a, ib = (i / per) * outer + (i % per) * stride_b;
    if (tid < MM) {
        const int r = tid / M, c = tid % M;
        // Hermitian inputs: build the full matrices from the upper triangles
        const double2 a = (r <= c) ? A[ia + r * M + c] : cconj(A[ia + c * M + r]);
        const double2 b = (r <= c) ? B[ib + r * M + c] : cconj(B[ib + c * M + r]);
        sA[tid] = (r == c) ? make_double2(a.x, 0.0) : a;
        sB[tid] = (r == c) ? make_double2(b.x, 0.0) : b;
        sId[tid] = make_double2(r == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    double dld = 0.0;
    const int flag = gevd_wave<M>(sA, sB, sId, sWs, sPn, sLam, &dld, 1e-30);
    wave_lds_sync();
    const bool ok = !(flag & kFreezeMask);
    if (tid < MM) P[i * stride_p + tid] = ok ? sPn[tid] : sId[tid];
    if (tid < M) lam[i * stride_l + tid] = ok ? sLam[tid] : 1.0;
    if (tid == 0) {
        if (logdet) logdet[i] = ok ? dld : 0.0;
        flags[i] = flag;
    }
}

hipError_t launch_gevd_runs(int M, int count, int per, int64_t outer, const double2* A, const double2* B,
                            int64_t stride_a, int64_t stride_b, double2* P, int64_t stride_p, double* lam,
                            int64_t stride_l, double* logdet, int* flags, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (per < 1) return hipErrorInvalidValue;
    switch (M) {
#define FCA_GEVD_CASE(MM_)                                                                                 \
    case MM_:                                                                                              \
        gevd_kernel<MM_><<<count, 64, 0, s>>>(A, B, stride_a, stride_b, per, outer, P, stride_p, lam,     \
                                              stride_l, logdet, flags);                                    \
        break;
        FCA_GEVD_CASE(1) FCA_GEVD_CASE(2) FCA_GEVD_CASE(3) FCA_GEVD_CASE(4)
        FCA_GEVD_CASE(5) FCA_GEVD_CASE(6) FCA_GEVD_CASE(7) FCA_GEVD_CASE(8)
#undef FCA_GEVD_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gevd(int M, int count, const double2* A, const double2* B, int64_t stride_a,
                       int64_t stride_b, double2* P, int64_t stride_p, double* lam, int64_t stride_l,
                       double* logdet, int* flags, hipStream_t s) {
    return launch_gevd_runs(M, count, count > 0 ? count : 1, 0, A, B, stride_a, stride_b, P, stride_p, lam,
                            stride_l, logdet, flags, s);
}

// R1 = I, R2 = I + 0.5 e1 e1^H at every frequency: R[2][F][M][M].
__global__ void default_R_kernel(int M, int F, double2* __restrict__ R) {
    const int64_t total = 2LL * F * M * M;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int ent = (int)(i % (M * M));
        const int j = (int)(i / ((int64_t)F * M * M));
        const int a = ent / M, b = ent % M;
        double re = (a == b) ? 1.0 : 0.0;
        if (j == 1 && a == 0 && b == 0) re += 0.5;
        R[i] = make_double2(re, 0.0);
    }
}

hipError_t launch_default_R(int M, int F, double2* R, hipStream_t s) {
    default_R_kernel<<<grid_for(2LL * F * M * M, 256), 256, 0, s>>>(M, F, R);
    return hipGetLastError();
}

// ============================================================== mask-weighted covariances
// Initial spatial covariances from time-frequency masks (the kind of start the
// experiments of Section 4 use): with r = v1 / (v1 + v2) of the stored
// powers (1/2 where both vanish), sharpened to r^p / (r^p + (1 - r)^p), the
// masks are w_1 = r and w_2 = 1 - r, A_j = sum_n w_j y y^H, and
// R_j = M A_j / tr(A_j) + load I (trace M before the loading; (1 + load) I
// where tr(A_j) = 0). One wave per (mixture, frequency): blockIdx.x = f,
// blockIdx.y = entry of `mix` (a wave-sized workgroup keeps the fixed cost
// of the reduction to one wave per problem). The upper triangles of A_j are
// FP64 register sums (both sources in one pass over the frames for M <= 4,
// one source per pass above), reduced by a butterfly in a fixed order. An
// integer p is applied by repeated multiplication.
__device__ __forceinline__ double mask_power(double r, double p, int ip) {
    if (ip > 0) {
        double x = r;
        for (int k = 1; k < ip; ++k) x *= r;
        return x;
    }
    return pow(r, p);
}

constexpr int kMaskThreads = 64;

template <int M, typename T>
__global__ __launch_bounds__(kMaskThreads) void mask_cov_kernel(const MaskCovMix* __restrict__ mix, int F,
                                                       const typename Vec2<T>::type* __restrict__ y,
                                                       const T* __restrict__ v, double2* __restrict__ R, double p,
                                                       double load) {
    constexpr int NU = M * (M + 1) / 2;  // upper-triangle entries
    constexpr int NS = M <= 4 ? 2 : 1;   // sources per pass
    __shared__ double red[NS][2 * NU];
    const MaskCovMix mx = mix[blockIdx.y];
    const int f = blockIdx.x, tid = threadIdx.x;
    const int ip = (p == floor(p) && p <= 64.0) ? (int)p : 0;  // integer exponent, or 0
    const auto* yf = y + mx.y_base + (int64_t)f * M * mx.npad;
    const T* v1 = v + mx.v_base + (int64_t)f * mx.npad;
    const T* v2 = v1 + (int64_t)F * mx.npad;
    for (int j0 = 0; j0 < 2; j0 += NS) {
        double are[NS][NU], aim[NS][NU];
#pragma unroll
        for (int q = 0; q < NS; ++q)
#pragma unroll
            for (int u = 0; u < NU; ++u) are[q][u] = aim[q][u] = 0.0;
        for (int n = tid; n < mx.N; n += kMaskThreads) {
            const double a = (double)v1[n], b = (double)v2[n];
            double r = (a + b > 0.0) ? a / (a + b) : 0.5;
            if (p != 1.0) {
                const double rp = mask_power(r, p, ip), sp = mask_power(1.0 - r, p, ip);
                r = rp / (rp + sp);
            }
            double yr[M], yi[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const auto ym = yf[(int64_t)m * mx.npad + n];
                yr[m] = (double)ym.x;
                yi[m] = (double)ym.y;
            }
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const double wt = (j0 + q) == 0 ? r : 1.0 - r;
                int u = 0;
#pragma unroll
                for (int i = 0; i < M; ++i) {
                    const double wr = wt * yr[i], wi = wt * yi[i];
#pragma unroll
                    for (int k = i; k < M; ++k, ++u) {  // w y_i conj(y_k)
                        are[q][u] = fma(wr, yr[k], fma(wi, yi[k], are[q][u]));
                        aim[q][u] = fma(wi, yr[k], fma(-wr, yi[k], aim[q][u]));
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NS; ++q)
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                double x = are[q][u], z = aim[q][u];
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    x += __shfl_xor(x, off, 64);
                    z += __shfl_xor(z, off, 64);
                }
                if (tid == 0) {
                    red[q][u] = x;
                    red[q][NU + u] = z;
                }
            }
        __syncthreads();
        if (tid < NS * M * M) {
            const int q = tid / (M * M), e = tid % (M * M);
            const int i = e / M, k = e % M;
            const int a = i < k ? i : k, c = i < k ? k : i;  // upper entry (a, c)
            const int u = a * M - a * (a - 1) / 2 + (c - a);
            double tr = 0.0;
            for (int d = 0; d < M; ++d) tr += red[q][d * M - d * (d - 1) / 2];
            const double xr = red[q][u];
            double xi = red[q][NU + u];
            if (i > k) xi = -xi;  // lower entry: conjugate
            double2 out;
            if (tr > 0.0) {
                out.x = (double)M * xr / tr;
                out.y = (double)M * xi / tr;
            } else {
                out.x = i == k ? 1.0 : 0.0;
                out.y = 0.0;
            }
            if (i == k) {
                out.x += load;
                out.y = 0.0;
            }
            R[mx.R_base + (int64_t)(j0 + q) * F * M * M + (int64_t)f * M * M + e] = out;
        }
        __syncthreads();  // red is reused by the next pass
    }
}

template <typename T>
static hipError_t launch_mask_cov_t(int M, const MaskCovMix* mix, int count, int F, const void* y, const void* v,
                                    double2* R, double p, double load, hipStream_t s) {
    const dim3 grid((unsigned)F, (unsigned)count);
    using T2 = typename Vec2<T>::type;
    const T2* yy = static_cast<const T2*>(y);
    const T* vv = static_cast<const T*>(v);
    switch (M) {
        case 2: mask_cov_kernel<2, T><<<grid, kMaskThreads, 0, s>>>(mix, F, yy, vv, R, p, load); break;
        case 3: mask_cov_kernel<3, T><<<grid, kMaskThreads, 0, s>>>(mix, F, yy, vv, R, p, load); break;
        case 4: mask_cov_kernel<4, T><<<grid, kMaskThreads, 0, s>>>(mix, F, yy, vv, R, p, load); break;
        case 5: mask_cov_kernel<5, T><<<grid, kMaskThreads, 0, s>>>(mix, F, yy, vv, R, p, load); break;
        case 6: mask_cov_kernel<6, T><<<grid, kMaskThreads, 0, s>>>(mix, F, yy, vv, R, p, load); break;
        case 7: mask_cov_kernel<7, T><<<grid, kMaskThreads, 0, s>>>(mix, F, yy, vv, R, p, load); break;
        case 8: mask_cov_kernel<8, T><<<grid, kMaskThreads, 0, s>>>(mix, F, yy, vv, R, p, load); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mask_cov(bool fp64, int M, const MaskCovMix* mix, int count, int F, const void* y, const void* v,
                           double2* R, double p, double load, hipStream_t s) {
    if (count < 1 || count > 65535 || F < 1) return hipErrorInvalidValue;
    return fp64 ? launch_mask_cov_t<double>(M, mix, count, F, y, v, R, p, load, s)
                : launch_mask_cov_t<float>(M, mix, count, F, y, v, R, p, load, s);
}

// ============================================================== log-likelihood totals
// out[b*iters + it] = sum_f ll[it*ll_stride + b*F + f], FP64, fixed order.
__global__ void ll_reduce_kernel(const double* __restrict__ ll, int64_t ll_stride, int iters, int F,
                                 double* __restrict__ out) {
    __shared__ double red[256];
    const int it = blockIdx.x, b = blockIdx.y;
    double s = 0.0;
    for (int f = threadIdx.x; f < F; f += 256) s += ll[(int64_t)it * ll_stride + (int64_t)b * F + f];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)b * iters + it] = red[0];
}

hipError_t launch_ll_reduce(const double* ll, int64_t ll_stride, int iters, int B, int F, double* out,
                            hipStream_t s) {
    if (iters <= 0 || B <= 0) return hipSuccess;
    ll_reduce_kernel<<<dim3(iters, B), 256, 0, s>>>(ll, ll_stride, iters, F, out);
    return hipGetLastError();
}

// P^-1 of M x M complex matrices by Gauss-Jordan elimination with partial
// pivoting, one wavefront per matrix (four per workgroup): lane (r, c) =
// (lane / 8, lane % 8) holds entry (r, c) of the working matrix A (initially
// P) and of X (initially I); each step exchanges them through LDS. The pivot
// choice is made identically by every lane from the same LDS values, so the
// control flow stays uniform. Optional outputs: Pinv (stride kMaxM^2 per
// problem, like P) and R2 = (P P^H)^-1 = X^H X, R1 = P^-H Lambda P^-1 =
// X^H Lambda X (eq. recoverS with S~1 = Lambda, S~2 = I in the current
// eigenbasis), [count][M][M].
template <int M>
__global__ __launch_bounds__(256) void pinv_kernel(int count, const double2* __restrict__ P,
                                                   const double* __restrict__ lam, double2* __restrict__ Pinv,
                                                   double2* __restrict__ R1, double2* __restrict__ R2) {
    __shared__ double2 sA[4][64], sX[4][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + w;  // problem of this wave (wave-uniform)
    if (i >= count) return;
    const int r = lane >> 3, c = lane & 7;
    const bool in = r < M && c < M;
    double2* A = sA[w];
    double2* X = sX[w];
    const int64_t base = (int64_t)i * kMaxM * kMaxM;
    double2 a = in ? P[base + r * M + c] : make_double2(0.0, 0.0);
    double2 x = make_double2((in && r == c) ? 1.0 : 0.0, 0.0);
#pragma unroll 1
    for (int j = 0; j < M; ++j) {
        A[lane] = a;
        X[lane] = x;
        wave_lds_sync();
        int p = j;
        double best = cabs2(A[j * 8 + j]);
        for (int q = j + 1; q < M; ++q) {
            const double mag = cabs2(A[q * 8 + j]);
            if (mag > best) {
                best = mag;
                p = q;
            }
        }
        const int rr = (r == j) ? p : (r == p ? j : r);  // this lane's row after swapping rows j and p
        const double2 piv = A[p * 8 + j];
        const double inv = 1.0 / cabs2(piv);
        const double2 pinv = make_double2(piv.x * inv, -piv.y * inv);
        const double2 prA = cmul(A[p * 8 + c], pinv), prX = cmul(X[p * 8 + c], pinv);  // new row j
        if (r == j) {
            a = prA;
            x = prX;
        } else {
            const double2 f = A[rr * 8 + j];
            a = csub(A[rr * 8 + c], cmul(f, prA));
            x = csub(X[rr * 8 + c], cmul(f, prX));
        }
        wave_lds_sync();  // every lane has read this step's matrix before the next step writes
    }
    if (Pinv && in) Pinv[base + r * M + c] = x;
    if (R1) {
        X[lane] = x;
        wave_lds_sync();
        if (in) {
            const double* l = lam + (int64_t)i * kMaxM;
            double2 s1 = make_double2(0.0, 0.0), s2 = make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const double2 t = cmulc(X[k * 8 + c], X[k * 8 + r]);  // conj(X_kr) X_kc
                s2 = cadd(s2, t);
                s1 = cadd(s1, cscale(l[k], t));
            }
            if (r == c) {
                s1.y = 0.0;
                s2.y = 0.0;
            }
            R1[(int64_t)i * M * M + r * M + c] = s1;
            R2[(int64_t)i * M * M + r * M + c] = s2;
        }
    }
}

hipError_t launch_pinv(int M, int count, const double2* P, const double* lam, double2* Pinv, double2* R1,
                       double2* R2, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const unsigned g = (count + 3) / 4;
    switch (M) {
#define FCA_PINV_CASE(MM_) \
    case MM_: pinv_kernel<MM_><<<g, 256, 0, s>>>(count, P, lam, Pinv, R1, R2); break;
        FCA_PINV_CASE(1) FCA_PINV_CASE(2) FCA_PINV_CASE(3) FCA_PINV_CASE(4)
        FCA_PINV_CASE(5) FCA_PINV_CASE(6) FCA_PINV_CASE(7) FCA_PINV_CASE(8)
#undef FCA_PINV_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_recover_R(int M, int count, const double2* P, const double* lam, double2* R1,
                            double2* R2, hipStream_t s) {
    return launch_pinv(M, count, P, lam, nullptr, R1, R2, s);
}

// ============================================================== MMSE separation
// x1 = P^-H mu~1 with mu~1_i = v1 lam_i y~_i / d_i (eq. MMSEtilde and
// Algorithm 1, step 11), x2 = y - x1 (eq. MMSE: mu1 + mu2 = y). Grid
// (frame blocks, problems); P^-1 comes precomputed (pinv_kernel).
template <int M, typename T>
__global__ __launch_bounds__(256) void separate_kernel(const EmProblem* __restrict__ probs,
                                                       const typename Vec2<T>::type* __restrict__ y,
                                                       const T* __restrict__ v, const double2* __restrict__ Pg,
                                                       const double* __restrict__ lamg,
                                                       const double2* __restrict__ Pinv,
                                                       typename Vec2<T>::type* __restrict__ x,
                                                       const int64_t* __restrict__ x_off) {
    using T2 = typename Vec2<T>::type;
    using MT = Math<T>;
    __shared__ T2 sP[M * M];  // P and P^-H in the bulk precision
    __shared__ T2 sQ[M * M];
    __shared__ T sLam[M];
    const EmProblem pr = probs[blockIdx.y];
    if ((int)blockIdx.x * 256 >= pr.n) return;
    const int tid = threadIdx.x;
    const int64_t pbase = (int64_t)pr.pid * kMaxM * kMaxM;
    if (tid < M * M) {
        const double2 p = Pg[pbase + tid];
        const int a = tid / M, b = tid % M;
        const double2 q = cconj(Pinv[pbase + b * M + a]);
        sP[tid] = make_vec2<T>((T)p.x, (T)p.y);
        sQ[tid] = make_vec2<T>((T)q.x, (T)q.y);
    }
    if (tid < M) sLam[tid] = (T)lamg[(int64_t)pr.pid * kMaxM + tid];
    __syncthreads();
    const int n = blockIdx.x * 256 + tid;
    if (n >= pr.n) return;
    T yr[M], yi[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const T2 val = y[pr.y_off + (int64_t)m * pr.npad + n];
        yr[m] = val.x;
        yi[m] = val.y;
    }
    const T a1 = v[pr.v_off + n], a2 = v[pr.v_off + pr.v2_off + n];
    T mr[M], mi[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        T sr = T(0), si = T(0);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const T2 p = sP[m * M + i];
            sr = fma(p.x, yr[m], fma(p.y, yi[m], sr));
            si = fma(p.x, yi[m], fma(-p.y, yr[m], si));
        }
        const T g = a1 * sLam[i] * MT::rcp(fma(a1, sLam[i], a2));
        mr[i] = g * sr;
        mi[i] = g * si;
    }
    T2* x1 = x + x_off[2 * blockIdx.y] + (int64_t)n * M;
    T2* x2 = x + x_off[2 * blockIdx.y + 1] + (int64_t)n * M;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        T sr = T(0), si = T(0);
#pragma unroll
        for (int b = 0; b < M; ++b) {
            const T2 q = sQ[a * M + b];
            sr = fma(q.x, mr[b], fma(-q.y, mi[b], sr));
            si = fma(q.x, mi[b], fma(q.y, mr[b], si));
        }
        T2 o1, o2;
        o1.x = sr; o1.y = si;
        o2.x = yr[a] - sr; o2.y = yi[a] - si;
        x1[a] = o1;
        x2[a] = o2;
    }
}

hipError_t launch_separate(int M, bool fp64, const EmProblem* probs, int count, int max_n, const void* y,
                           const void* v, const double2* P, const double* lam, const double2* Pinv, void* x,
                           const int64_t* x_off, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const dim3 grid((max_n + 255) / 256, count);
    switch (M) {
#define FCA_SEP_CASE(MM_)                                                                                        \
    case MM_:                                                                                                    \
        if (fp64)                                                                                                \
            separate_kernel<MM_, double><<<grid, 256, 0, s>>>(probs, static_cast<const double2*>(y),              \
                static_cast<const double*>(v), P, lam, Pinv, static_cast<double2*>(x), x_off);                         \
        else                                                                                                     \
            separate_kernel<MM_, float><<<grid, 256, 0, s>>>(probs, static_cast<const float2*>(y),                \
                static_cast<const float*>(v), P, lam, Pinv, static_cast<float2*>(x), x_off);                           \
        break;
        FCA_SEP_CASE(1) FCA_SEP_CASE(2) FCA_SEP_CASE(3) FCA_SEP_CASE(4)
        FCA_SEP_CASE(5) FCA_SEP_CASE(6) FCA_SEP_CASE(7) FCA_SEP_CASE(8)
#undef FCA_SEP_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fca
