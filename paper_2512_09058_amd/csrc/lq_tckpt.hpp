// Checkpointed solve kernel template of tile plans (shared by lq_tckpt.hip, padded nx 32 / 64, and
// lq_tckpt_wide.hip, padded nx 128, which compile in parallel): the register-streaming solve
// (primal and adjoint, refinement included) with the factor blocks of each checkpoint segment
// recomputed on demand by the tile factor sweep, in the same workgroup (factor scratch overlaid on
// the solve's per-stage LDS staging area).  The workgroup has one wavefront per tile column of the
// padded sizes, the count the factor kernel of a checkpointed tile plan also uses, so the
// recomputed blocks are those of the factor kernel bit for bit.
#pragma once
#include "lq_tsolve.hpp"

namespace lq {
namespace {

// Wavefronts per workgroup for padded sizes NXP, NUP (tile columns NXP/16 + NUP/16).
constexpr int tc_waves(int NXP, int NUP) {
  return NXP / 16 + NUP / 16 <= 3 ? 3 : NXP / 16 + NUP / 16 <= 5 ? 5 : 10;
}

template <int NXP, int NUP, typename TF, typename TP>
__global__ void __launch_bounds__(64 * tc_waves(NXP, NUP)) __attribute__((amdgpu_waves_per_eu(3)))
k_solve_tile_ckpt(SolveArgs a, const int32_t* __restrict__ order, int32_t* counter) {
  constexpr int W = tc_waves(NXP, NUP);
  extern __shared__ __align__(16) double sm_tc[];
  each_instance(a.batch, order, counter, [&](int b) { tsolve_one<W, NXP, NUP, TF, W, TP>(a, b, sm_tc); });
}

// The kernel of one padded shape for a mode (float64, float32 factors, bf16 products).
template <int NXP, int NUP>
const void* tc_kernel(lq_mode mode) {
  if (mode == LQ_F64) return (const void*)k_solve_tile_ckpt<NXP, NUP, double, double>;
  if (mode == LQ_MIXED_F32) return (const void*)k_solve_tile_ckpt<NXP, NUP, float, float>;
  if (mode == LQ_MIXED_BF16) return (const void*)k_solve_tile_ckpt<NXP, NUP, float, BF16>;
  return nullptr;
}

}  // namespace

// Kernels of padded nx 128 (lq_tckpt_wide.hip); nullptr for another nu.
const void* tc_kernel_wide(int NUP, lq_mode mode);

}  // namespace lq
