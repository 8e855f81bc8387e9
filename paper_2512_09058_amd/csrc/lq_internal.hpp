// Internal definitions shared by the host runtime and the kernels of liblqkkt.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lqkkt.h"

namespace lq {

// Per-instance descriptor: sizes and element offsets into the packed input, output and
// workspace arrays.  Built on the host by the plan, read once per instance by the kernels.
struct Desc {
  int32_t N, nx, nu, pad;
  int64_t oA, oB, oQ, oR, oS, oq, or_, of, ox0;  // inputs
  int64_t ox, ou, olam;                           // outputs (x_1..x_N, u_0..u_{N-1}, lam)
  int64_t oF;   // factor region (elements of the factor type)
  int64_t oV;   // rbar (N nu) then p ((N+1) nx), float64: sweep of lq_factor's right-hand side
  int64_t oV2;  // refinement / adjoint state, float64 (layout: v2_* below)
  int64_t oZB;  // adjoint solution: xbar (N nx), ubar (N nu), lambar (N nx), float64
  int64_t oK;   // stages (N + 1) of the instances before this one (per-stage arrays of updates)
};

// Factor block of one stage (elements): [LR packed lower, nu(nu+1)/2][1/diag LR, nu]
// [LS, nx*nu row-major][LQ packed lower, nx(nx+1)/2][1/diag LQ, nx].  Stage N holds only
// the LQ part (chol Q_N); stage 0 leaves the LQ part unused.
// One copy: `blocks` row-major blocks of r x c elements (the source of a pad, the destination of
// an unpad) and R x C elements (the other side); padding entries of a pad get `diag` on the
// diagonal and 0 elsewhere.
struct PadOp {
  const double* src;
  double* dst;
  int64_t blocks;
  int32_t r, c, R, C;
  double diag;
  int32_t unpad;
};
constexpr int kPadOps = 12;

__host__ __device__ inline int64_t stage_factor_elems(int nx, int nu) {
  return (int64_t)nu * (nu + 1) / 2 + nu + (int64_t)nx * nu + (int64_t)nx * (nx + 1) / 2 + nx;
}
__host__ __device__ inline int off_dR(int nx, int nu) { return nu * (nu + 1) / 2; }
__host__ __device__ inline int off_LS(int nx, int nu) { return nu * (nu + 1) / 2 + nu; }
__host__ __device__ inline int off_LQ(int nx, int nu) { return nu * (nu + 1) / 2 + nu + nx * nu; }
__host__ __device__ inline int off_dQ(int nx, int nu) {
  return nu * (nu + 1) / 2 + nu + nx * nu + nx * (nx + 1) / 2;
}

// Refinement state of one instance (float64): rbar2 [N nu] | p2 [(N+1) nx] | flam [N nx]
// (= -rho_l, the dynamics residual) | rho_u [N nu] | rho_x [(N+1) nx] (k = 1..N used).
__host__ __device__ inline int64_t v2_elems(int64_t N, int64_t nx, int64_t nu) {
  return 2 * N * nu + 2 * (N + 1) * nx + N * nx;
}
__host__ __device__ inline int64_t v2_p2(int64_t N, int64_t nx, int64_t nu) { return N * nu; }
__host__ __device__ inline int64_t v2_flam(int64_t N, int64_t nx, int64_t nu) { return N * nu + (N + 1) * nx; }
__host__ __device__ inline int64_t v2_rhou(int64_t N, int64_t nx, int64_t nu) { return N * nu + (N + 1) * nx + N * nx; }
__host__ __device__ inline int64_t v2_rhox(int64_t N, int64_t nx, int64_t nu) {
  return 2 * N * nu + (N + 1) * nx + N * nx;
}

// Factor region of a checkpointed instance (stride s): one slot per stage 0, s, 2s, ... and N,
// then a segment buffer of s stage blocks.  ckpt_slot(k) is the slot of such a stage k.
__host__ __device__ inline int64_t ckpt_slots(int64_t N, int64_t s) { return N / s + 1 + (N % s ? 1 : 0); }
__host__ __device__ inline int64_t ckpt_slot(int64_t k, int64_t N, int64_t s) {
  return k == N ? ckpt_slots(N, s) - 1 : k / s;
}

// LDS layout of the tile factor kernel (byte offsets) for TU input and TX state tiles of 16:
// U^Q tiles of the state block (TX(TX+1)/2, factor type), input-pivot panels (TU x T float64
// tiles), state-pivot panels (mixed: 2 x T float64 tiles; float64 mode keeps them in the U^Q
// tiles), W slabs (2 x T product-type tiles, aliased with a panel region that is dead while they
// live), the inverse of the current diagonal tile, the scratch tile of the diagonal step, vectors.
struct TileLds {
  int oLQB, oUP, oXP, oWS, oDI, oSC, oVec, total;
};
__host__ __device__ inline TileLds tile_lds(int TU, int TX, bool f64) {
  const int T = TU + TX, tileD = 16 * 17 * 8, tileF = 16 * 20 * 4;
  const int tileQ = f64 ? tileD : tileF, tileW = f64 ? tileD : tileF;
  TileLds L;
  int o = 0;
  L.oLQB = o;
  o += TX * (TX + 1) / 2 * tileQ;
  if (f64) {
    L.oUP = L.oWS = L.oXP = o;
    const int up = TU * T * tileD, ws = 2 * T * tileW;
    o += up > ws ? up : ws;
  } else {
    L.oUP = o;
    o += TU * T * tileD;
    L.oXP = L.oWS = o;
    const int xp = 2 * T * tileD, ws = 2 * T * tileW;
    o += xp > ws ? xp : ws;
  }
  L.oDI = o;
  o += tileD;
  L.oSC = o;  // scratch tile of the diagonal step (one wavefront at a time)
  o += tileD;
  L.oVec = o;
  o += 8 * (48 * TX + 32 * T + 16 * TU);
  L.total = o;
  return L;
}

// c ? v : 0 without control flow.  Written as a select, the compiler sinks a load feeding it into
// a load under a divergent branch, and the end of that branch waits for every load in flight,
// which serialises loads meant to overlap.  The mask here is opaque to the optimiser, so the load
// (from a clamped, always valid address) stays unconditional and its wait moves to the first use.
// By default the asm is not volatile, so the loads around it may be reordered freely; with ORD
// it is volatile and also keeps the loads around it in program order (a masking step then waits
// for its load before the next load is issued, but the compiler holds fewer loads in flight, which
// measured faster where registers are short: the checkpointed solve and the nx = 128 solve).
template <bool ORD = false>
__device__ __forceinline__ double keep_if(bool c, double v) {
  int m = c ? -1 : 0;
  if constexpr (ORD) asm volatile("" : "+v"(m));
  else asm("" : "+v"(m));
  return __longlong_as_double(__double_as_longlong(v) & (long long)m);
}

// Maximum that propagates NaN (fmax would drop it and hide a non-finite residual), and the
// relative residual max|rho| / max|b| from the two maxima (NaN if either is).
__device__ __forceinline__ double nan_max(double m, double v) { return (v > m || v != v) ? v : m; }
__device__ __forceinline__ double rel_of(double mr, double mb) {
  return mb != mb ? mb : (mb > 0.0 ? mr / mb : mr);
}

// Right-hand side selector of the solve kernels.
enum RhsKind : int32_t { RHS_PRIMAL = 0, RHS_ADJOINT = 1 };

struct SolveArgs {
  const Desc* desc;
  int32_t batch;
  lq_data d;
  const void* F;       // factors (double or float)
  const double* V;     // factor-time right-hand-side sweep (rbar, p)
  double* V2;          // correction sweeps
  double* x;           // solution being refined (primal x/u/lam or adjoint xbar/ubar/lambar)
  double* u;
  double* lam;
  const double* gx;    // adjoint right-hand side (RHS_ADJOINT)
  const double* gu;
  double tol;
  int32_t max_it;
  int32_t check;
  int32_t rhs;         // RhsKind
  int32_t out_is_zb;   // 1: x/u/lam point into the workspace adjoint region (per-instance oZB)
  double* rel_res;
  int32_t* iters;
  int32_t* info;
  int32_t ckpt;                // checkpoint stride of the factors (0: every stage stored)
  int32_t lds_factor_doubles;  // with checkpoints: LDS doubles of the factor scratch
  int32_t stage_doubles;       // LDS doubles of the stage-matrix staging buffer
};

// Launch shape of the generic kernels: threads per workgroup (64, 128 or 256); without a
// counter one workgroup per instance in the given order, with a counter a persistent grid of
// `grid` workgroups pulling instances from it.
struct GenericLaunch {
  int32_t threads;
  int32_t grid;
  const int32_t* order;  // device, [batch], instance indices longest first (may be NULL)
  int32_t* counter;      // device work counter (NULL: one workgroup per instance)
  int32_t ckpt;          // checkpoint stride (factor kernel)
};

// Gradient outer products of the adjoint.
struct GradArgs {
  const Desc* desc;
  int32_t batch;
  lq_data d;
  const double *x, *u, *lam;  // primal solution
  const double* ZB;           // adjoint solution region (workspace)
  double *gA, *gB, *gQ, *gR, *gS, *gq, *gr, *gf, *gx0;
};

// Error message of the calling thread (lq_last_error): set_error records it and returns code.
int set_error(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
// Raise (never lower) a kernel's dynamic-LDS limit.
hipError_t raise_lds_limit(const void* kernel, size_t lds);

}  // namespace lq
