// Size-specialised kernels (lq_small.hpp) for one shape of every nx + nu = 16 that lq_small.hip
// does not compile.  With them every shape with nx + nu <= 16 has a compiled shape that covers it
// (NX >= nx, NU >= nu); a plan for an uncompiled shape pads its data to that envelope.
#include "lq_small.hpp"

namespace lq {

#define LQ_SMALL_ENV_SHAPES(X) \
  X(15, 1) X(14, 2) X(13, 3) X(11, 5) X(9, 7) X(8, 8) X(7, 9) X(6, 10) X(5, 11) X(4, 12) X(3, 13) X(2, 14) X(1, 15)

int small_env_count() {
  int n = 0;
#define X(a, b) ++n;
  LQ_SMALL_ENV_SHAPES(X)
#undef X
  return n;
}

void small_env_shape(int i, int* nx, int* nu) {
  int k = 0;
#define X(a, b)   \
  if (k++ == i) { \
    *nx = a;      \
    *nu = b;      \
    return;       \
  }
  LQ_SMALL_ENV_SHAPES(X)
#undef X
  *nx = *nu = 0;
}

hipError_t launch_factor_small_env(lq_mode mode, int batch, int N, int nx, int nu, const lq_data& d, void* F,
                                   double* V, int32_t* info, hipStream_t st) {
#define X(a, b) \
  if (nx == a && nu == b) return factor_shape<a, b>(mode, batch, N, d, F, V, info, st);
  LQ_SMALL_ENV_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_solve_small_env(lq_mode mode, int N, int nx, int nu, const SolveArgs& a, hipStream_t st) {
#define X(a_, b_) \
  if (nx == a_ && nu == b_) return solve_shape<a_, b_>(mode, N, a, st);
  LQ_SMALL_ENV_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace lq
