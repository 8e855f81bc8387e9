// Checkpointed solve kernels of tile plans (padded nx 32 / 64 with nu up to 64 here, padded nx 128
// with nu up to 32 in lq_tckpt_wide.hip; float64, float32 and bf16-product factors; the kernel is
// described in lq_tckpt.hpp), with their launch and sizing helpers.
#include "lq_tckpt.hpp"

namespace lq {
hipError_t raise_lds_limit(const void* kernel, size_t lds);  // lq_api.hip
namespace {

__global__ void k_reset_counter_tc(int32_t* c) {
  if (threadIdx.x == 0) c[0] = 0;
}

const void* tc_kernel(int NXP, int NUP, lq_mode mode) {
#define TCK(X, U) \
  if (NXP == X && NUP == U) return tc_kernel<X, U>(mode);
  TCK(32, 16) TCK(32, 32) TCK(32, 64) TCK(64, 16) TCK(64, 32) TCK(64, 64)
#undef TCK
  if (NXP == 128) return tc_kernel_wide(NUP, mode);
  return nullptr;
}

}  // namespace

// Padded sizes of the checkpointed tile solve for a batch's largest nx, nu (false: none): nx up to
// 64 with nu up to 64, or nx up to 128 with nu up to 32 (at most ten tile columns, the factor
// sweep's widest workgroup).
bool tckpt_sizes(int maxnx, int maxnu, int* NXP, int* NUP) {
  if (maxnx > 128 || maxnu > 64 || (maxnx > 64 && maxnu > 32)) return false;
  *NXP = maxnx <= 32 ? 32 : maxnx <= 64 ? 64 : 128;
  *NUP = maxnu <= 16 ? 16 : maxnu <= 32 ? 32 : 64;
  return true;
}
bool tckpt_mode_supported(lq_mode mode) { return mode == LQ_F64 || mode == LQ_MIXED_F32 || mode == LQ_MIXED_BF16; }
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
