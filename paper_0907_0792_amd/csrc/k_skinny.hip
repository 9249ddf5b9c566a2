// Inner product with few result rows (M <= 8): the paper's row form as an
// HBM stream (kernel in skinny.hpp). This unit holds the one-run-per-thread
// instances and the dispatch; k_skinny_wide.hip holds the four-run ones, so
// the two large sets of (dtype, op1, op2, M) instances compile in parallel.
#include "skinny.hpp"

namespace moa {

template hipError_t skinny_launch_r<1>(moa_dtype, moa_op, moa_op, const void *, const void *, void *, int64_t,
                                       int64_t, int64_t, hipStream_t);
extern template hipError_t skinny_launch_r<4>(moa_dtype, moa_op, moa_op, const void *, const void *, void *, int64_t,
                                              int64_t, int64_t, hipStream_t);

// Four runs per thread when that still gives at least 512 workgroups
// (measured ~20% faster on 4 x 128 . 128 x 2^22 FP64), else one.
hipError_t launch_skinny_inner(moa_dtype dt, moa_op op1, moa_op op2, const void *A, const void *B, void *D, int64_t M,
                               int64_t K, int64_t N, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  if (M > kSkinnyMaxRows) return hipErrorInvalidValue;
  const int64_t vec = dt == MOA_F64 ? 2 : 4;
  if (N >= (int64_t)512 * 256 * vec * 4) return skinny_launch_r<4>(dt, op1, op2, A, B, D, M, K, N, s);
  return skinny_launch_r<1>(dt, op1, op2, A, B, D, M, K, N, s);
}

}  // namespace moa
