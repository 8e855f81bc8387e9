// Checkpointed solve kernels of tile plans: the register-streaming solve (primal and adjoint,
// refinement included) with the factor blocks of each checkpoint segment recomputed on demand by
// the tile factor sweep, in the same workgroup (factor scratch overlaid on the solve's per-stage
// LDS staging area).  The workgroup has one wavefront per tile column of the padded sizes, the
// count the factor kernel of a checkpointed tile plan also uses, so the recomputed blocks are those
// of the factor kernel bit for bit.
#include "lq_tsolve.hpp"

namespace lq {
hipError_t raise_lds_limit(const void* kernel, size_t lds);  // lq_api.hip
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

__global__ void k_reset_counter_tc(int32_t* c) {
  if (threadIdx.x == 0) c[0] = 0;
}

template <int NXP, int NUP>
const void* tc_kernel(lq_mode mode) {
  if (mode == LQ_F64) return (const void*)k_solve_tile_ckpt<NXP, NUP, double, double>;
  if (mode == LQ_MIXED_F32) return (const void*)k_solve_tile_ckpt<NXP, NUP, float, float>;
  return nullptr;
}

const void* tc_kernel(int NXP, int NUP, lq_mode mode) {
#define TCK(X, U) \
  if (NXP == X && NUP == U) return tc_kernel<X, U>(mode);
  TCK(32, 16) TCK(32, 32) TCK(32, 64) TCK(64, 16) TCK(64, 32) TCK(64, 64)
#undef TCK
  return nullptr;
}

}  // namespace

// Padded sizes of the checkpointed tile solve for a batch's largest nx, nu (false: none).
bool tckpt_sizes(int maxnx, int maxnu, int* NXP, int* NUP) {
  if (maxnx > 64 || maxnu > 64) return false;
  *NXP = maxnx <= 32 ? 32 : 64;
  *NUP = maxnu <= 16 ? 16 : maxnu <= 32 ? 32 : 64;
  return true;
}
bool tckpt_mode_supported(lq_mode mode) { return mode == LQ_F64 || mode == LQ_MIXED_F32; }
int tckpt_waves(int NXP, int NUP) { return tc_waves(NXP, NUP); }

// Dynamic LDS: the solve's vectors, then the larger of its staging area and the factor scratch
// (tile_lds bytes, the largest over the batch).
size_t tckpt_lds_bytes(int NXP, int NUP, size_t tile_lds) {
  const size_t st = sizeof(double) * (size_t)tsolve_stage_doubles(tc_waves(NXP, NUP), NXP, NUP);
  return sizeof(double) * (size_t)tsolve_vec_doubles(NXP, NUP) + (st > tile_lds ? st : tile_lds);
}

hipError_t prepare_tckpt(int NXP, int NUP, lq_mode mode, size_t lds) {
  const void* k = tc_kernel(NXP, NUP, mode);
  if (!k) return hipErrorInvalidValue;
  return raise_lds_limit(k, lds);
}

int tckpt_blocks_per_cu(int NXP, int NUP, lq_mode mode, size_t lds) {
  int n = 0;
  const void* k = tc_kernel(NXP, NUP, mode);
  if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 64 * tc_waves(NXP, NUP), lds) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n > 0 ? n : 1;
}

hipError_t launch_solve_tckpt(int NXP, int NUP, lq_mode mode, const SolveArgs& a, size_t lds, const GenericLaunch& c,
                              hipStream_t st) {
  const void* k = tc_kernel(NXP, NUP, mode);
  if (!k) return hipErrorInvalidValue;
  if (c.counter) hipLaunchKernelGGL(k_reset_counter_tc, dim3(1), dim3(64), 0, st, c.counter);
  const dim3 grid(c.counter ? c.grid : a.batch), block(64 * tc_waves(NXP, NUP));
  void* args[] = {(void*)&a, (void*)&c.order, (void*)&c.counter};
  return hipLaunchKernel(k, grid, block, args, lds, st);
}

}  // namespace lq
