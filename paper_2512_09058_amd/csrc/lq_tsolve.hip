// Register-streaming solve kernels (device code in lq_tsolve.hpp) and their host side.
#include "lq_tsolve.hpp"

namespace lq {
hipError_t raise_lds_limit(const void* kernel, size_t lds);  // lq_api.hip
namespace {

// Register target: two wavefronts per SIMD (several instances per CU hide each other's latency).
template <int W, int NXP, int NUP, typename TF>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(2)))
k_solve_tile(SolveArgs a, const int32_t* __restrict__ order, int32_t* counter) {
  extern __shared__ double sm_ts[];
  each_instance(a.batch, order, counter, [&](int b) { tsolve_one<W, NXP, NUP, TF>(a, b, sm_ts); });
}

__global__ void k_reset_counter_ts(int32_t* c) {
  if (threadIdx.x == 0) c[0] = 0;
}

// Wavefronts per workgroup for the padded state size.
constexpr int ts_waves(int NXP) { return NXP <= 32 ? 2 : 8; }

template <int NXP, int NUP, typename TF>
const void* ts_kernel() {
  return (const void*)k_solve_tile<ts_waves(NXP), NXP, NUP, TF>;
}

const void* ts_kernel(int NXP, int NUP, bool f64) {
#define TSK(X, U)                                                                         \
  if (NXP == X && NUP == U) return f64 ? ts_kernel<X, U, double>() : ts_kernel<X, U, float>();
  TSK(32, 16) TSK(32, 32) TSK(32, 64) TSK(64, 16) TSK(64, 32) TSK(64, 64) TSK(128, 16) TSK(128, 32) TSK(128, 64)
#undef TSK
  return nullptr;
}

}  // namespace

// Padded sizes of the register-streaming solve for a batch's largest nx, nu (false: none).
bool tsolve_sizes(int maxnx, int maxnu, int* NXP, int* NUP) {
  if (maxnx > 128 || maxnu > 64) return false;
  *NXP = maxnx <= 32 ? 32 : maxnx <= 64 ? 64 : 128;
  *NUP = maxnu <= 16 ? 16 : maxnu <= 32 ? 32 : 64;
  return true;
}
int tsolve_threads(int NXP) { return 64 * ts_waves(NXP); }
size_t tsolve_lds_bytes(int NXP, int NUP) {
  return sizeof(double) * (size_t)tsolve_lds_doubles(ts_waves(NXP), NXP, NUP);
}

hipError_t prepare_tsolve(int NXP, int NUP, lq_mode mode) {
  return raise_lds_limit(ts_kernel(NXP, NUP, mode == LQ_F64), tsolve_lds_bytes(NXP, NUP));
}

int tsolve_blocks_per_cu(int NXP, int NUP, lq_mode mode) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ts_kernel(NXP, NUP, mode == LQ_F64), tsolve_threads(NXP),
                                                   tsolve_lds_bytes(NXP, NUP)) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n > 0 ? n : 1;
}

hipError_t launch_solve_tsolve(int NXP, int NUP, lq_mode mode, const SolveArgs& a, const GenericLaunch& c,
                               hipStream_t st) {
  if (c.counter) hipLaunchKernelGGL(k_reset_counter_ts, dim3(1), dim3(64), 0, st, c.counter);
  const dim3 grid(c.counter ? c.grid : a.batch), block(tsolve_threads(NXP));
  const size_t lds = tsolve_lds_bytes(NXP, NUP);
  const void* k = ts_kernel(NXP, NUP, mode == LQ_F64);
  if (!k) return hipErrorInvalidValue;
  void* args[] = {(void*)&a, (void*)&c.order, (void*)&c.counter};
  return hipLaunchKernel(k, grid, block, args, lds, st);
}

}  // namespace lq
