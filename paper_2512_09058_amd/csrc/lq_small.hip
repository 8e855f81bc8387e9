// Size-specialised kernels for uniform batches (placeholder: no variant yet).
#include "lq_internal.hpp"

namespace lq {
bool small_variant_available(lq_mode, int, int) { return false; }
hipError_t launch_factor_small(lq_mode, int, int, int, int, const lq_data&, void*, double*, int32_t*,
                               hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_solve_small(lq_mode, int, int, int, const SolveArgs&, hipStream_t) {
  return hipErrorInvalidValue;
}
}  // namespace lq
