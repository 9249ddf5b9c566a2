// SIMT inner-product kernels, FP32 folds (+, *, max, min).
#include "simt.hpp"

namespace moa {

template hipError_t simt_fold<float, MOA_ADD>(moa_op, const float *, const float *, float *, int64_t,
                                              int64_t, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t simt_fold<float, MOA_MUL>(moa_op, const float *, const float *, float *, int64_t,
                                              int64_t, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t simt_fold<float, MOA_MAX>(moa_op, const float *, const float *, float *, int64_t,
                                              int64_t, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t simt_fold<float, MOA_MIN>(moa_op, const float *, const float *, float *, int64_t,
                                              int64_t, int64_t, int, int64_t, int64_t, hipStream_t);

}  // namespace moa
