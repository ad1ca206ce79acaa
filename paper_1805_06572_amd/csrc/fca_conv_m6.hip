// fca_conv_m6.hip -- conventional-EM kernels for M = 6 (float bulk and FP64).
#include "fca_conv.h"

namespace fca {
template hipError_t launch_conv_fpt<6, float>(int fpt, const EmProblem* probs, int count, const void* y, void* v, int64_t v_alt, double2* P, double* lam, double* logdet, int* flags, double* ll, int64_t ll_stride, int iters, int it_base, hipStream_t s);
template hipError_t launch_conv_fpt<6, double>(int fpt, const EmProblem* probs, int count, const void* y, void* v, int64_t v_alt, double2* P, double* lam, double* logdet, int* flags, double* ll, int64_t ll_stride, int iters, int it_base, hipStream_t s);
}  // namespace fca
