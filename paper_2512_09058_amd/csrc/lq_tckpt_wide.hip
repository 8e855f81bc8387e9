// Checkpointed solve kernels of tile plans at padded nx 128 (nu up to 32, at most ten tile
// columns), in a translation unit of their own so that they compile beside the others.
#include "lq_tckpt.hpp"

namespace lq {

const void* tc_kernel_wide(int NUP, lq_mode mode) {
  if (NUP == 16) return tc_kernel<128, 16>(mode);
  if (NUP == 32) return tc_kernel<128, 32>(mode);
  return nullptr;
}

}  // namespace lq
