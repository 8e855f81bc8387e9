// Dispatch of the size-specialised kernels (lq_small.hpp) over the compiled shapes: the shapes of
// the workloads here, and in lq_small_env.hip one shape for every nx + nu = 16 not listed here, so
// that every shape with nx + nu <= 16 has a compiled shape that covers it (the envelope a plan pads
// an uncompiled shape to).
#include "lq_small.hpp"

namespace lq {
namespace {

#define LQ_SMALL_SHAPES(X) X(12, 4) X(4, 2) X(8, 4) X(10, 6) X(6, 2)

bool compiled_here(int nx, int nu) {
#define X(a, b) \
  if (nx == a && nu == b) return true;
  LQ_SMALL_SHAPES(X)
#undef X
  return false;
}

bool compiled_env(int nx, int nu) {
  for (int i = 0; i < small_env_count(); ++i) {
    int a, b;
    small_env_shape(i, &a, &b);
    if (a == nx && b == nu) return true;
  }
  return false;
}

}  // namespace

bool small_variant_available(lq_mode mode, int nx, int nu) {
  if (mode == LQ_MIXED_BF16) return false;
  return compiled_here(nx, nu) || compiled_env(nx, nu);
}

// Smallest compiled shape (nx + nu, then nx) with NX >= nx and NU >= nu; false if none.
bool small_envelope(lq_mode mode, int nx, int nu, int* NX, int* NU) {
  if (mode == LQ_MIXED_BF16 || nx < 1 || nu < 1 || nx + nu > 16) return false;
  int bx = 0, bu = 0;
  auto consider = [&](int a, int b) {
    if (a < nx || b < nu) return;
    if (bx == 0 || a + b < bx + bu || (a + b == bx + bu && a < bx)) {
      bx = a;
      bu = b;
    }
  };
#define X(a, b) consider(a, b);
  LQ_SMALL_SHAPES(X)
#undef X
  for (int i = 0; i < small_env_count(); ++i) {
    int a, b;
    small_env_shape(i, &a, &b);
    consider(a, b);
  }
  if (bx == 0) return false;
  *NX = bx;
  *NU = bu;
  return true;
}

// The staged loads move 16-byte chunks: every array of the problem, the workspace and the
// outputs must be 16-byte aligned.
bool small_aligned(const lq_data& d, const void* ws) {
  const void* p[] = {d.A, d.B, d.Q, d.R, d.S, d.q, d.r, d.f, d.x0, ws};
  for (const void* q : p)
    if (q && ((uintptr_t)q & 15)) return false;
  return true;
}

hipError_t launch_factor_small(lq_mode mode, int batch, int N, int nx, int nu, const lq_data& d, void* F,
                               double* V, int32_t* info, hipStream_t st) {
#define X(a, b) \
  if (nx == a && nu == b) return factor_shape<a, b>(mode, batch, N, d, F, V, info, st);
  LQ_SMALL_SHAPES(X)
#undef X
  return launch_factor_small_env(mode, batch, N, nx, nu, d, F, V, info, st);
}

hipError_t launch_solve_small(lq_mode mode, int N, int nx, int nu, const SolveArgs& a, hipStream_t st) {
  if (a.rhs != RHS_PRIMAL) return hipErrorInvalidValue;
#define X(a_, b_) \
  if (nx == a_ && nu == b_) return solve_shape<a_, b_>(mode, N, a, st);
  LQ_SMALL_SHAPES(X)
#undef X
  return launch_solve_small_env(mode, N, nx, nu, a, st);
}

}  // namespace lq
