// fca_em_nt128.hip -- EM-iteration kernels with 128 threads: resident problems of up to 1024 frames (an autotuning candidate).
#include "fca_em.h"

namespace fca {
template hipError_t launch_em_nt<128>(int M, bool fp64, int fpt, const EmProblem* probs, int count, const void* y,
                                      void* v, int64_t v_alt, double2* P, double* lam, double* logdet, int* flags,
                                      double* ll, int64_t ll_stride, int iters, int it_base, hipStream_t s);
}  // namespace fca
