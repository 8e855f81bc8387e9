// Matrix-core tile factor kernel (the sweep itself is in lq_tile_factor.hpp) and its host side.
#include "lq_tile_factor.hpp"

namespace lq {
hipError_t raise_lds_limit(const void* kernel, size_t lds);  // lq_api.hip
namespace {

// Instances of this workgroup: without a counter the one at position blockIdx.x, with a counter
// positions pulled from it until the batch is exhausted (every workgroup exits once the counter
// has passed batch).  One call site, so the body is inlined once.
template <typename F>
__device__ __forceinline__ void for_each_instance(int batch, const int32_t* order, int32_t* counter, F&& body) {
  __shared__ int s_next;
  for (int it = 0;; ++it) {
    int t;
    if (counter) {
      if (threadIdx.x == 0) s_next = atomicAdd(counter, 1);
      __syncthreads();
      t = s_next;
      __syncthreads();
    } else {
      t = it == 0 ? (int)blockIdx.x : batch;
    }
    if (t >= batch) break;
    body(order ? order[t] : t);
  }
}

// Wavefronts per SIMD the register allocation targets: enough resident workgroups that several
// instances share a CU (their latency chains overlap).
template <int TMAX>
struct TileOcc {
  static constexpr int v = 3;
};

template <int TMAX, typename TF, typename TP>
__global__ void __launch_bounds__(64 * TMAX) __attribute__((amdgpu_waves_per_eu(TileOcc<TMAX>::v)))
k_factor_tile(const Desc* __restrict__ desc, int batch, lq_data d,
                                                          TF* __restrict__ F, double* __restrict__ Vws,
                                                          int32_t* __restrict__ info, const int32_t* __restrict__ order,
                                                          int32_t* counter, int ckpt) {
  extern __shared__ __align__(16) unsigned char lds_tile[];
  __shared__ int s_info;
  for_each_instance(batch, order, counter, [&](int b) {
    const Desc D = desc[b];
    // every stage block stored, or with a checkpoint stride only those of stages 0, s, 2s, ..., N
    TF* Fi = F + D.oF;
    const int64_t fs = stage_factor_elems(D.nx, D.nu);
    auto dst = [&](int k) -> TF* {
      if (ckpt == 0) return Fi + (int64_t)k * fs;
      return (k % ckpt == 0 || k == D.N) ? Fi + ckpt_slot(k, D.N, ckpt) * fs : nullptr;
    };
    factor_tile_range<TMAX, TF, TP>(D, d, 0, D.N, dst, (const TF*)nullptr, Vws + D.oV, lds_tile, s_info);
    if (threadIdx.x == 0) info[b] = s_info;
    __syncthreads();
  });
}

__global__ void k_reset_counter_tile(int32_t* c) {
  if (threadIdx.x == 0) c[0] = 0;
}

template <int TMAX>
const void* tile_kernel(lq_mode mode) {
  if (mode == LQ_F64) return (const void*)k_factor_tile<TMAX, double, double>;
  if (mode == LQ_MIXED_BF16) return (const void*)k_factor_tile<TMAX, float, BF16>;
  return (const void*)k_factor_tile<TMAX, float, float>;
}

template <int TMAX>
hipError_t launch_tile(lq_mode mode, dim3 grid, dim3 block, size_t lds, hipStream_t st, const Desc* desc, int batch,
                       const lq_data& d, void* F, double* V, int32_t* info, const GenericLaunch& c) {
  if (mode == LQ_F64)
    hipLaunchKernelGGL((k_factor_tile<TMAX, double, double>), grid, block, lds, st, desc, batch, d, (double*)F, V,
                       info, c.order, c.counter, c.ckpt);
  else if (mode == LQ_MIXED_BF16)
    hipLaunchKernelGGL((k_factor_tile<TMAX, float, BF16>), grid, block, lds, st, desc, batch, d, (float*)F, V, info,
                       c.order, c.counter, c.ckpt);
  else
    hipLaunchKernelGGL((k_factor_tile<TMAX, float, float>), grid, block, lds, st, desc, batch, d, (float*)F, V,
                       info, c.order, c.counter, c.ckpt);
  return hipGetLastError();
}

}  // namespace

// Largest tile count the tile kernels take (one wavefront per tile column).
int tile_max_columns() { return 10; }

// Wavefronts per workgroup (= instantiated column count) for an instance set of at most T columns.
int tile_waves(int T) { return T <= 3 ? 3 : T <= 5 ? 5 : 10; }

bool tile_mode_supported(lq_mode mode) { return mode == LQ_F64 || mode == LQ_MIXED_F32 || mode == LQ_MIXED_BF16; }

size_t tile_lds_bytes(int nx, int nu, lq_mode mode) {
  const TileLds L = tile_lds((nu + 15) / 16, (nx + 15) / 16, mode == LQ_F64);
  return (size_t)L.total;
}

hipError_t prepare_tile(int waves, lq_mode mode, size_t lds) {
  const void* k = waves == 3 ? tile_kernel<3>(mode) : waves == 5 ? tile_kernel<5>(mode) : tile_kernel<10>(mode);
  return raise_lds_limit(k, lds);
}

int tile_blocks_per_cu(int waves, lq_mode mode, size_t lds) {
  int n = 0;
  const void* k = waves == 3 ? tile_kernel<3>(mode) : waves == 5 ? tile_kernel<5>(mode) : tile_kernel<10>(mode);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 64 * waves, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n > 0 ? n : 1;
}

hipError_t launch_factor_tile(lq_mode mode, int waves, const Desc* desc, int batch, const lq_data& d, void* F,
                              double* V, int32_t* info, size_t lds, const GenericLaunch& c, hipStream_t st) {
  if (c.counter) hipLaunchKernelGGL(k_reset_counter_tile, dim3(1), dim3(64), 0, st, c.counter);
  const dim3 grid(c.counter ? c.grid : batch), block(64 * waves);
  if (waves == 3) return launch_tile<3>(mode, grid, block, lds, st, desc, batch, d, F, V, info, c);
  if (waves == 5) return launch_tile<5>(mode, grid, block, lds, st, desc, batch, d, F, V, info, c);
  return launch_tile<10>(mode, grid, block, lds, st, desc, batch, d, F, V, info, c);
}

}  // namespace lq
