// SIMT inner-product kernels, int32 arithmetic folds (+, *, max, min).
#include "simt.hpp"

namespace moa {

template hipError_t simt_fold<int32_t, MOA_ADD>(moa_op, const int32_t *, const int32_t *, int32_t *, int64_t,
                                                int64_t, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t simt_fold<int32_t, MOA_MUL>(moa_op, const int32_t *, const int32_t *, int32_t *, int64_t,
                                                int64_t, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t simt_fold<int32_t, MOA_MAX>(moa_op, const int32_t *, const int32_t *, int32_t *, int64_t,
                                                int64_t, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t simt_fold<int32_t, MOA_MIN>(moa_op, const int32_t *, const int32_t *, int32_t *, int64_t,
                                                int64_t, int64_t, int, int64_t, int64_t, hipStream_t);

}  // namespace moa
