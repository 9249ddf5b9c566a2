// Four-runs-per-thread instances of the few-row stream (kernel in
// skinny.hpp; dispatch in k_skinny.hip). The per-dtype instance sets are
// compiled in k_skinny_wide_{f64,f32,i32}.hip, in parallel.
#include "skinny.hpp"

namespace moa {

extern template hipError_t skinny_dispatch<double, 4>(moa_op, moa_op, const double *, const double *, double *,
                                                      int64_t, int64_t, int64_t, hipStream_t);
extern template hipError_t skinny_dispatch<float, 4>(moa_op, moa_op, const float *, const float *, float *, int64_t,
                                                     int64_t, int64_t, hipStream_t);
extern template hipError_t skinny_dispatch<int32_t, 4>(moa_op, moa_op, const int32_t *, const int32_t *, int32_t *,
                                                       int64_t, int64_t, int64_t, hipStream_t);
template hipError_t skinny_launch_r<4>(moa_dtype, moa_op, moa_op, const void *, const void *, void *, int64_t,
                                       int64_t, int64_t, hipStream_t);

}  // namespace moa
