// Copies between a problem of shape (nx, nu) and its padding to a compiled size-specialised shape
// (NX, NU) >= (nx, nu), for plans whose shape has no size-specialised kernel of its own.  The padded
// problem adds states with identity cost and no coupling (zero rows and columns of A, B, S, zero
// q, f, x_init) and inputs with identity cost and no coupling (zero columns of B, zero rows of S,
// zero r): its KKT system is block diagonal with the original one and an identity block whose
// right-hand side is zero, so its solution restricted to the original unknowns is the original
// solution, its extra unknowns are zero, and its residual rows are the original ones plus zeros.
// Its Riccati factors are those of the original problem in the leading rows and columns (the
// padded rows of every stage matrix are identity rows), which extract_small_factors copies out.
#include <algorithm>

#include "lq_internal.hpp"

namespace lq {

namespace {

struct PadOps {
  PadOp op[kPadOps];
};

// Grid: x strides over the destination rows of the largest copy (16 lanes per row: C, c <= 16),
// y = the copy.  Coalesced destination writes; the source rows are read where they overlap.
// 32-bit row indices (the plan keeps every padded array below 2^31 rows): a 64-bit division per
// element would cost more than the element's memory traffic.
__global__ void __launch_bounds__(256) k_pad(PadOps ops) {
  const PadOp o = ops.op[blockIdx.y];
  const uint32_t dr = o.unpad ? o.r : o.R, dc = o.unpad ? o.c : o.C;  // destination block shape
  const uint32_t sc = o.unpad ? o.C : o.c;                             // source row length
  const uint32_t srows = o.unpad ? o.R : o.r;
  const uint32_t rows = (uint32_t)(o.blocks * dr);
  const uint32_t j = threadIdx.x & 15;
  for (uint32_t row = (blockIdx.x * blockDim.x + threadIdx.x) >> 4; row < rows; row += (gridDim.x * blockDim.x) >> 4) {
    if (j >= dc) continue;
    const uint32_t blk = row / dr, i = row - blk * dr;
    double v;
    if (o.unpad || (i < (uint32_t)o.r && j < (uint32_t)o.c))
      v = o.src[((uint64_t)blk * srows + i) * sc + j];
    else
      v = i == j ? o.diag : 0.0;
    o.dst[(uint64_t)row * dc + j] = v;
  }
}

// Real factor blocks (shape nx, nu) from the padded ones (NX, NU), both in the packed stage
// layout [L^R packed][1/diag L^R][L^S nx x nu][L^Q packed][1/diag L^Q]: the triangles and the
// diagonals of the real shape are prefixes of the padded ones, L^S is the leading nx x nu block.
template <typename TF>
__global__ void __launch_bounds__(256) k_extract_factors(const TF* __restrict__ src, TF* __restrict__ dst,
                                                         uint32_t blocks, int nx, int nu, int NX, int NU) {
  const uint32_t fr = (uint32_t)stage_factor_elems(nx, nu), fp = (uint32_t)stage_factor_elems(NX, NU);
  const uint32_t odr = nu * (nu + 1) / 2, ols = odr + nu, olq = ols + nx * nu, odq = olq + nx * (nx + 1) / 2;
  const uint32_t Podr = NU * (NU + 1) / 2, Pols = Podr + NU, Polq = Pols + NX * NU, Podq = Polq + NX * (NX + 1) / 2;
  const uint32_t total = blocks * fr;  // below 2^31 (the plan checks)
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const uint32_t blk = e / fr, w = e - blk * fr;
    uint32_t s;
    if (w < odr) s = w;
    else if (w < ols) s = Podr + (w - odr);
    else if (w < olq) {
      const uint32_t t = w - ols, i = t / nu, jj = t - i * nu;
      s = Pols + i * NU + jj;
    } else if (w < odq) s = Polq + (w - olq);
    else s = Podq + (w - odq);
    dst[e] = src[(uint64_t)blk * fp + s];
  }
}

}  // namespace

hipError_t launch_pad(const PadOp* ops, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n > kPadOps) return hipErrorInvalidValue;
  PadOps all;
  int64_t most = 0;
  for (int i = 0; i < n; ++i) {
    all.op[i] = ops[i];
    most = std::max(most, ops[i].blocks * (ops[i].unpad ? ops[i].r : ops[i].R));
  }
  if (most * 16 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;  // 32-bit row indices
  const int64_t want = (most * 16 + 255) / 256;
  const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(want, 4096)), (unsigned)n);
  hipLaunchKernelGGL(k_pad, grid, dim3(256), 0, st, all);
  return hipGetLastError();
}

hipError_t launch_extract_small_factors(bool f64, const void* src, void* dst, int64_t blocks, int nx, int nu, int NX,
                                        int NU, hipStream_t st) {
  const int64_t total = blocks * stage_factor_elems(nx, nu);
  const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 8192)));
  if (total >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  if (f64)
    hipLaunchKernelGGL(k_extract_factors<double>, grid, dim3(256), 0, st, (const double*)src, (double*)dst,
                       (uint32_t)blocks, nx, nu, NX, NU);
  else
    hipLaunchKernelGGL(k_extract_factors<float>, grid, dim3(256), 0, st, (const float*)src, (float*)dst,
                       (uint32_t)blocks, nx, nu, NX, NU);
  return hipGetLastError();
}

}  // namespace lq
