// SIMT inner-product kernels, FP64 folds (+, *, max, min).
#include "simt.hpp"

namespace moa {

template hipError_t simt_fold<double, MOA_ADD>(moa_op, const double *, const double *, double *, int64_t,
                                               int64_t, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t simt_fold<double, MOA_MUL>(moa_op, const double *, const double *, double *, int64_t,
                                               int64_t, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t simt_fold<double, MOA_MAX>(moa_op, const double *, const double *, double *, int64_t,
                                               int64_t, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t simt_fold<double, MOA_MIN>(moa_op, const double *, const double *, double *, int64_t,
                                               int64_t, int64_t, int, int64_t, int64_t, hipStream_t);

}  // namespace moa
