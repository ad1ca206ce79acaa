// fca_em_nt256.hip -- EM-iteration kernels with kEmThreads threads: every frame count, resident (up to 2048 frames) and streamed.
#include "fca_em.h"

namespace fca {
template hipError_t launch_em_nt<256>(int M, bool fp64, int fpt, const EmProblem* probs, int count, const void* y,
                                      void* v, int64_t v_alt, double2* P, double* lam, double* logdet, int* flags,
                                      double* ll, int64_t ll_stride, int iters, int it_base, hipStream_t s);
}  // namespace fca
