// Four-runs-per-thread instances of the few-row stream (kernel in
// skinny.hpp; dispatch in k_skinny.hip).
#include "skinny.hpp"

namespace moa {

template hipError_t skinny_launch_r<4>(moa_dtype, moa_op, moa_op, const void *, const void *, void *, int64_t,
                                       int64_t, int64_t, hipStream_t);

}  // namespace moa
