// Four-runs-per-thread few-row stream instances for I32, every op pair
// (kernel in skinny.hpp).
#include "skinny.hpp"

namespace moa {

template hipError_t skinny_dispatch<int32_t, 4>(moa_op, moa_op, const int32_t *, const int32_t *, int32_t *, int64_t,
                                           int64_t, int64_t, hipStream_t);

}  // namespace moa
