// Four-runs-per-thread few-row stream instances for F64, every op pair
// (kernel in skinny.hpp).
#include "skinny.hpp"

namespace moa {

template hipError_t skinny_dispatch<double, 4>(moa_op, moa_op, const double *, const double *, double *, int64_t,
                                           int64_t, int64_t, hipStream_t);

}  // namespace moa
