// SIMT inner-product kernels, int32 bitwise folds (and, or, xor).
#include "simt.hpp"

namespace moa {

template hipError_t simt_fold<int32_t, MOA_AND>(moa_op, const int32_t *, const int32_t *, int32_t *, int64_t,
                                                int64_t, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t simt_fold<int32_t, MOA_OR>(moa_op, const int32_t *, const int32_t *, int32_t *, int64_t,
                                               int64_t, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t simt_fold<int32_t, MOA_XOR>(moa_op, const int32_t *, const int32_t *, int32_t *, int64_t,
                                                int64_t, int64_t, int, int64_t, int64_t, hipStream_t);

}  // namespace moa
