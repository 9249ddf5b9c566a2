// Four-runs-per-thread few-row stream instances for F32, every op pair
// (kernel in skinny.hpp).
#include "skinny.hpp"

namespace moa {

template hipError_t skinny_dispatch<float, 4>(moa_op, moa_op, const float *, const float *, float *, int64_t,
                                           int64_t, int64_t, hipStream_t);

}  // namespace moa
