// Batched symmetric positive definite block-tridiagonal systems (paper, Sec. "Cyclic reduction of
// block-tridiagonal linear systems", eq. block-tri, and the appendix "Cyclic reduction and parallel
// cyclic reduction"): cyclic reduction (factorisation and solution), parallel cyclic reduction and
// preconditioned conjugate gradients, on the workgroup-level float64 routines of lq_wgblas.hpp.
//
// A system has Nb diagonal blocks M_k (n x n, SPD) and Nb - 1 subdiagonal blocks K_k (block row
// k + 1, block column k); arrays are row-major [batch][Nb][n][n], [batch][Nb-1][n][n] and
// [batch][Nb][n].  Nb need not be a power of two: a neighbour outside 0..Nb-1 is absent.
//
// Cyclic reduction eliminates at level l (s = 2^l) the block rows k = s (2i + 1) < Nb from their
// neighbours k - s and k + s, in parallel: L_k = chol(M_k), U_k = C(k - s, k) L_k^{-T},
// Y_k = C(k + s, k) L_k^{-T} (C(r, c) the coupling block of the reduced system at row r, column c),
// then every remaining row j = 2 s i gets M_j -= Y_{j-s} Y_{j-s}^T + U_{j+s} U_{j+s}^T and the
// fill-in C(j, j - 2s) = -Y_{j-s} U_{j-s}^T; block 0 is factored last.  These L, U, Y are the
// blocks of the Cholesky factor of the matrix with its block rows ordered by 2-adic valuation
// (Sec. "Cyclic reduction as block Cholesky factorization").  Each level is two launches over
// (block, system): the eliminations, then the updates of the rows that remain.
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "lq_internal.hpp"
#include "lq_wgblas.hpp"
#include "lqblocktri.h"

namespace lq {
namespace {

using wg::NT;

struct BT {
  int32_t batch, Nb, n;
  int64_t nn;  // n * n
};

__host__ __device__ inline int64_t blk(const BT& t, int b, int k) { return ((int64_t)b * t.Nb + k) * t.nn; }

// Copy M into the working diagonal blocks and K into the coupling slots: Kw[k] = C(k, k - 1) = K_{k-1}.
__global__ void __launch_bounds__(NT, 2) k_cr_init(BT t, const double* __restrict__ M, const double* __restrict__ K,
                                                double* Lw, double* Kw) {
  const int k = blockIdx.x, b = blockIdx.y;
  const double* src = M + blk(t, b, k);
  double* dst = Lw + blk(t, b, k);
  for (int64_t e = threadIdx.x; e < t.nn; e += NT) dst[e] = src[e];
  if (k >= 1) {
    const double* ks = K + ((int64_t)b * (t.Nb - 1) + (k - 1)) * t.nn;
    double* kd = Kw + blk(t, b, k);
    for (int64_t e = threadIdx.x; e < t.nn; e += NT) kd[e] = ks[e];
  }
}

__device__ inline void report(int32_t* info, int b, int code) {
  if (threadIdx.x == 0 && code) atomicCAS(info + b, 0, code);
}

// Level l eliminations: block k = s (2 i + 1) for i = blockIdx.x.
__global__ void __launch_bounds__(NT, 2) k_cr_elim(BT t, int s, double* Lw, const double* Kw, double* U, double* Y,
                                                int32_t* info) {
  extern __shared__ __align__(16) unsigned char smraw[];
  wg::Smem& sm = *reinterpret_cast<wg::Smem*>(smraw);
  const int k = s * (2 * blockIdx.x + 1), b = blockIdx.y, n = t.n;
  double* L = Lw + blk(t, b, k);
  const int f = wg::potrf(n, L, n, sm);
  report(info, b, f ? k + 1 : 0);
  // U_k = C(k - s, k) L^{-T} = Kw[k]^T L^{-T}
  wg::transpose(n, n, Kw + blk(t, b, k), n, U + blk(t, b, k), n);
  wg::trsm_rlt(n, n, L, n, U + blk(t, b, k), n, sm);
  if (k + s < t.Nb) {  // Y_k = C(k + s, k) L^{-T} = Kw[k + s] L^{-T}
    wg::copy(n, n, Kw + blk(t, b, k + s), n, Y + blk(t, b, k), n);
    wg::trsm_rlt(n, n, L, n, Y + blk(t, b, k), n, sm);
  }
}

// Level l updates of the rows that remain: j = 2 s i for i = blockIdx.x.
__global__ void __launch_bounds__(NT, 2) k_cr_update(BT t, int s, double* Lw, double* Kw, const double* U, const double* Y) {
  extern __shared__ __align__(16) unsigned char smraw[];
  wg::Smem& sm = *reinterpret_cast<wg::Smem*>(smraw);
  const int j = 2 * s * blockIdx.x, b = blockIdx.y, n = t.n;
  double* Mj = Lw + blk(t, b, j);
  if (j >= s) wg::gemm<false, true, 1>(n, n, n, -1.0, Y + blk(t, b, j - s), n, Y + blk(t, b, j - s), n, 1.0, Mj, n, sm);
  if (j + s < t.Nb) wg::gemm<false, true, 1>(n, n, n, -1.0, U + blk(t, b, j + s), n, U + blk(t, b, j + s), n, 1.0, Mj, n, sm);
  if (j >= 2 * s)  // fill-in C(j, j - 2s) = -Y_{j-s} U_{j-s}^T
    wg::gemm<false, true, 0>(n, n, n, -1.0, Y + blk(t, b, j - s), n, U + blk(t, b, j - s), n, 0.0, Kw + blk(t, b, j), n, sm);
}

__global__ void __launch_bounds__(NT, 2) k_cr_last(BT t, double* Lw, int32_t* info) {
  extern __shared__ __align__(16) unsigned char smraw[];
  wg::Smem& sm = *reinterpret_cast<wg::Smem*>(smraw);
  const int b = blockIdx.x;
  const int f = wg::potrf(t.n, Lw + blk(t, b, 0), t.n, sm);
  report(info, b, f ? 1 : 0);
}

// Solution with the CR factors, one workgroup per system: forward substitution level by level,
// then recovery of the eliminated unknowns (eq. cr-odd) from the last level back.
__global__ void __launch_bounds__(NT, 2) k_cr_solve(BT t, const double* Lw, const double* U, const double* Y,
                                                 const double* __restrict__ rhs, double* x) {
  extern __shared__ __align__(16) unsigned char smraw[];
  wg::Smem& sm = *reinterpret_cast<wg::Smem*>(smraw);
  const int b = blockIdx.x, n = t.n, Nb = t.Nb;
  const int64_t vo = (int64_t)b * Nb * n;
  double* xb = x + vo;
  wg::copy(1, Nb * n, rhs + vo, Nb * n, xb, Nb * n);
  int top = 0;
  while ((1 << top) < Nb) ++top;
  for (int l = 0; l < top; ++l) {
    const int s = 1 << l;
    for (int k = s; k < Nb; k += 2 * s) wg::trsv<false>(n, Lw + blk(t, b, k), n, xb + (int64_t)k * n, sm);
    for (int j = 0; j < Nb; j += 2 * s) {  // b_j -= Y_{j-s} bt_{j-s} + U_{j+s} bt_{j+s}
      if (j >= s) wg::gemv<false>(n, n, -1.0, Y + blk(t, b, j - s), n, xb + (int64_t)(j - s) * n, 1.0, xb + (int64_t)j * n, sm);
      if (j + s < Nb) wg::gemv<false>(n, n, -1.0, U + blk(t, b, j + s), n, xb + (int64_t)(j + s) * n, 1.0, xb + (int64_t)j * n, sm);
    }
  }
  wg::trsv<false>(n, Lw + blk(t, b, 0), n, xb, sm);
  wg::trsv<true>(n, Lw + blk(t, b, 0), n, xb, sm);
  for (int l = top - 1; l >= 0; --l) {
    const int s = 1 << l;
    for (int k = s; k < Nb; k += 2 * s) {  // x_k = L^{-T} (bt_k - U_k^T x_{k-s} - Y_k^T x_{k+s})
      double* xk = xb + (int64_t)k * n;
      wg::gemv<true>(n, n, -1.0, U + blk(t, b, k), n, xb + (int64_t)(k - s) * n, 1.0, xk, sm);
      if (k + s < Nb) wg::gemv<true>(n, n, -1.0, Y + blk(t, b, k), n, xb + (int64_t)(k + s) * n, 1.0, xk, sm);
      wg::trsv<true>(n, Lw + blk(t, b, k), n, xk, sm);
    }
  }
}

// ---- parallel cyclic reduction (Alg. "pcr"), non-periodic: neighbours outside 0..Nb-1 absent --
// Working arrays: Mw, Kw (Kw[k] = C(k + s, k), the coupling to the row s below), bw; per level
// the factors L, Y, U and bt = L^{-1} b, then the next level's M2, K2, b2.

__global__ void __launch_bounds__(NT, 2) k_pcr_init(BT t, const double* __restrict__ M, const double* __restrict__ K,
                                                 const double* __restrict__ rhs, double* Mw, double* Kw, double* bw) {
  const int k = blockIdx.x, b = blockIdx.y, n = t.n;
  for (int64_t e = threadIdx.x; e < t.nn; e += NT) Mw[blk(t, b, k) + e] = M[blk(t, b, k) + e];
  if (k + 1 < t.Nb) {
    const double* ks = K + ((int64_t)b * (t.Nb - 1) + k) * t.nn;
    for (int64_t e = threadIdx.x; e < t.nn; e += NT) Kw[blk(t, b, k) + e] = ks[e];
  } else {
    for (int64_t e = threadIdx.x; e < t.nn; e += NT) Kw[blk(t, b, k) + e] = 0.0;
  }
  const int64_t vo = ((int64_t)b * t.Nb + k) * n;
  for (int e = threadIdx.x; e < n; e += NT) bw[vo + e] = rhs[vo + e];
}

__global__ void __launch_bounds__(NT, 2) k_pcr_elim(BT t, int s, const double* Mw, const double* Kw, const double* bw,
                                                 double* L, double* U, double* Y, double* bt, int32_t* info) {
  extern __shared__ __align__(16) unsigned char smraw[];
  wg::Smem& sm = *reinterpret_cast<wg::Smem*>(smraw);
  const int k = blockIdx.x, b = blockIdx.y, n = t.n;
  double* Lk = L + blk(t, b, k);
  wg::copy(n, n, Mw + blk(t, b, k), n, Lk, n);
  const int f = wg::potrf(n, Lk, n, sm);
  report(info, b, f ? k + 1 : 0);
  if (k + s < t.Nb) {  // Y_k = C(k + s, k) L^{-T}
    wg::copy(n, n, Kw + blk(t, b, k), n, Y + blk(t, b, k), n);
    wg::trsm_rlt(n, n, Lk, n, Y + blk(t, b, k), n, sm);
  }
  if (k - s >= 0) {  // U_k = C(k - s, k) L^{-T} = C(k, k - s)^T L^{-T}
    wg::transpose(n, n, Kw + blk(t, b, k - s), n, U + blk(t, b, k), n);
    wg::trsm_rlt(n, n, Lk, n, U + blk(t, b, k), n, sm);
  }
  const int64_t vo = ((int64_t)b * t.Nb + k) * n;
  wg::copy(1, n, bw + vo, n, bt + vo, n);
  wg::trsv<false>(n, Lk, n, bt + vo, sm);
}

__global__ void __launch_bounds__(NT, 2) k_pcr_update(BT t, int s, const double* Mw, const double* bw, const double* U,
                                                   const double* Y, const double* bt, double* M2, double* K2,
                                                   double* b2) {
  extern __shared__ __align__(16) unsigned char smraw[];
  wg::Smem& sm = *reinterpret_cast<wg::Smem*>(smraw);
  const int k = blockIdx.x, b = blockIdx.y, n = t.n;
  double* Mk = M2 + blk(t, b, k);
  wg::copy(n, n, Mw + blk(t, b, k), n, Mk, n);
  const int64_t vo = ((int64_t)b * t.Nb + k) * n;
  wg::copy(1, n, bw + vo, n, b2 + vo, n);
  if (k - s >= 0) {
    wg::gemm<false, true, 1>(n, n, n, -1.0, Y + blk(t, b, k - s), n, Y + blk(t, b, k - s), n, 1.0, Mk, n, sm);
    wg::gemv<false>(n, n, -1.0, Y + blk(t, b, k - s), n, bt + vo - (int64_t)s * n, 1.0, b2 + vo, sm);
  }
  if (k + s < t.Nb) {
    wg::gemm<false, true, 1>(n, n, n, -1.0, U + blk(t, b, k + s), n, U + blk(t, b, k + s), n, 1.0, Mk, n, sm);
    wg::gemv<false>(n, n, -1.0, U + blk(t, b, k + s), n, bt + vo + (int64_t)s * n, 1.0, b2 + vo, sm);
  }
  if (k + 2 * s < t.Nb)  // C(k + 2s, k) = -Y_{k+s} U_{k+s}^T
    wg::gemm<false, true, 0>(n, n, n, -1.0, Y + blk(t, b, k + s), n, U + blk(t, b, k + s), n, 0.0, K2 + blk(t, b, k), n, sm);
  else
    wg::fill(n, n, 0.0, K2 + blk(t, b, k), n);
}

__global__ void __launch_bounds__(NT, 2) k_pcr_last(BT t, const double* Mw, const double* bw, double* L, double* x,
                                                 int32_t* info) {
  extern __shared__ __align__(16) unsigned char smraw[];
  wg::Smem& sm = *reinterpret_cast<wg::Smem*>(smraw);
  const int k = blockIdx.x, b = blockIdx.y, n = t.n;
  double* Lk = L + blk(t, b, k);
  wg::copy(n, n, Mw + blk(t, b, k), n, Lk, n);
  const int f = wg::potrf(n, Lk, n, sm);
  report(info, b, f ? k + 1 : 0);
  const int64_t vo = ((int64_t)b * t.Nb + k) * n;
  wg::copy(1, n, bw + vo, n, x + vo, n);
  wg::trsv<false>(n, Lk, n, x + vo, sm);
  wg::trsv<true>(n, Lk, n, x + vo, sm);
}

// ---- preconditioned conjugate gradients ------------------------------------------------------
// Block-Jacobi (D^{-1}) and stair (D^{-1} (I - Koff D^{-1})) preconditioners from the explicit
// inverses D_k^{-1} = L_k^{-T} L_k^{-1} of the diagonal blocks, formed once.

__global__ void __launch_bounds__(NT, 2) k_pcg_inv(BT t, const double* __restrict__ M, double* L, double* Dinv,
                                                int32_t* info) {
  extern __shared__ __align__(16) unsigned char smraw[];
  wg::Smem& sm = *reinterpret_cast<wg::Smem*>(smraw);
  const int k = blockIdx.x, b = blockIdx.y, n = t.n;
  double* Lk = L + blk(t, b, k);
  wg::copy(n, n, M + blk(t, b, k), n, Lk, n);
  const int f = wg::potrf(n, Lk, n, sm);
  report(info, b, f ? k + 1 : 0);
  double* Di = Dinv + blk(t, b, k);
  // T = I L^{-T} = L^{-T} into Di, then D^{-1} = T T^T = L^{-T} L^{-1} (through Lk's slot)
  for (int64_t e = threadIdx.x; e < t.nn; e += NT) Di[e] = (e / n == e % n) ? 1.0 : 0.0;
  wg::trsm_rlt(n, n, Lk, n, Di, n, sm);
  wg::gemm<false, true, 0>(n, n, n, 1.0, Di, n, Di, n, 0.0, Lk, n, sm);  // Lk <- D^{-1}
  wg::copy(n, n, Lk, n, Di, n);
}

// y = Mat x for the whole system (one workgroup), rows (k, i) over the threads.
__device__ inline void bt_matvec(const BT& t, int b, const double* M, const double* K, const double* x, double* y) {
  const int n = t.n, Nb = t.Nb;
  wg::sync();
  for (int e = threadIdx.x; e < Nb * n; e += NT) {
    const int k = e / n, i = e % n;
    const double* Mr = M + blk(t, b, k) + (int64_t)i * n;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s = fma(Mr[j], x[(int64_t)k * n + j], s);
    if (k >= 1) {  // K_{k-1} x_{k-1}
      const double* Kr = K + ((int64_t)b * (Nb - 1) + (k - 1)) * t.nn + (int64_t)i * n;
      for (int j = 0; j < n; ++j) s = fma(Kr[j], x[(int64_t)(k - 1) * n + j], s);
    }
    if (k + 1 < Nb) {  // K_k^T x_{k+1}
      const double* Kc = K + ((int64_t)b * (Nb - 1) + k) * t.nn + i;
      for (int j = 0; j < n; ++j) s = fma(Kc[(int64_t)j * n], x[(int64_t)(k + 1) * n + j], s);
    }
    y[e] = s;
  }
  wg::sync();
}

// y = D^{-1} x blockwise.
__device__ inline void bt_dinv(const BT& t, int b, const double* Dinv, const double* x, double* y) {
  const int n = t.n;
  wg::sync();
  for (int e = threadIdx.x; e < t.Nb * n; e += NT) {
    const int k = e / n, i = e % n;
    const double* Dr = Dinv + blk(t, b, k) + (int64_t)i * n;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s = fma(Dr[j], x[(int64_t)k * n + j], s);
    y[e] = s;
  }
  wg::sync();
}

// w = Koff v (the off-diagonal part of the matrix only).
__device__ inline void bt_koff(const BT& t, int b, const double* K, const double* v, double* w) {
  const int n = t.n, Nb = t.Nb;
  wg::sync();
  for (int e = threadIdx.x; e < Nb * n; e += NT) {
    const int k = e / n, i = e % n;
    double s = 0.0;
    if (k >= 1) {
      const double* Kr = K + ((int64_t)b * (Nb - 1) + (k - 1)) * t.nn + (int64_t)i * n;
      for (int j = 0; j < n; ++j) s = fma(Kr[j], v[(int64_t)(k - 1) * n + j], s);
    }
    if (k + 1 < Nb) {
      const double* Kc = K + ((int64_t)b * (Nb - 1) + k) * t.nn + i;
      for (int j = 0; j < n; ++j) s = fma(Kc[(int64_t)j * n], v[(int64_t)(k + 1) * n + j], s);
    }
    w[e] = s;
  }
  wg::sync();
}

__global__ void __launch_bounds__(NT, 2) k_pcg(BT t, const double* __restrict__ M, const double* __restrict__ K,
                                            const double* __restrict__ rhs, const double* Dinv, int stair, double tol,
                                            int max_it, double* x, double* work, int32_t* iters, double* relres,
                                            int32_t* info) {
  extern __shared__ __align__(16) unsigned char smraw[];
  wg::Smem& sm = *reinterpret_cast<wg::Smem*>(smraw);
  const int b = blockIdx.x, N = t.Nb * t.n;
  const int64_t vo = (int64_t)b * N;
  const double* bb = rhs + vo;
  double* xb = x + vo;
  double* r = work + vo * 5;
  double* z = r + N;
  double* p = z + N;
  double* q = p + N;
  double* u = q + N;
  auto precond = [&](const double* src, double* dst) {
    if (!stair) {
      bt_dinv(t, b, Dinv, src, dst);
    } else {  // dst = D^{-1} (src - Koff D^{-1} src)
      bt_dinv(t, b, Dinv, src, u);
      bt_koff(t, b, K, u, q);
      for (int e = threadIdx.x; e < N; e += NT) q[e] = src[e] - q[e];
      bt_dinv(t, b, Dinv, q, dst);
    }
  };
  for (int e = threadIdx.x; e < N; e += NT) {
    xb[e] = 0.0;
    r[e] = bb[e];
  }
  const double nb = wg::absmax(N, bb, sm);
  int it = 0;
  double res = nb > 0.0 ? 1.0 : 0.0;
  if (nb > 0.0) {
    precond(r, z);
    for (int e = threadIdx.x; e < N; e += NT) p[e] = z[e];
    double rz = wg::dot(N, r, z, sm);
    double rn = wg::absmax(N, r, sm);
    while (rn > tol * nb && it < max_it) {
      bt_matvec(t, b, M, K, p, q);
      const double alpha = rz / wg::dot(N, p, q, sm);
      for (int e = threadIdx.x; e < N; e += NT) {
        xb[e] = fma(alpha, p[e], xb[e]);
        r[e] = fma(-alpha, q[e], r[e]);
      }
      ++it;
      precond(r, z);
      const double rz2 = wg::dot(N, r, z, sm);
      const double beta = rz2 / rz;
      for (int e = threadIdx.x; e < N; e += NT) p[e] = fma(beta, p[e], z[e]);
      rz = rz2;
      rn = wg::absmax(N, r, sm);
    }
    // true residual of the returned iterate
    bt_matvec(t, b, M, K, xb, q);
    for (int e = threadIdx.x; e < N; e += NT) q[e] = bb[e] - q[e];
    res = wg::absmax(N, q, sm) / nb;
  }
  if (threadIdx.x == 0) {
    if (iters) iters[b] = it;
    if (relres) relres[b] = res;
    if (info && info[b] == 0 && !(res <= tol)) info[b] = res == res ? -2 : -1;
  }
}

int bt_fail(int code, const char* msg) { return set_error(code, "%s", msg); }

hipError_t lds_ready(const void* k) { return raise_lds_limit(k, sizeof(wg::Smem)); }

int check_sizes(int32_t batch, int32_t Nb, int32_t n) {
  if (batch <= 0 || Nb <= 0 || n <= 0) return bt_fail(LQ_EINVAL, "batch, Nb and n must be positive");
  if (n > 256) return bt_fail(LQ_EUNSUPPORTED, "block size above 256");
  if (batch > 65535 || Nb > (1 << 20)) return bt_fail(LQ_EUNSUPPORTED, "batch above 65535 or Nb above 2^20");
  return LQ_OK;
}

int launch_rc(hipError_t e) {
  if (e != hipSuccess) return set_error(LQ_EHIP, "launch failed: %s", hipGetErrorString(e));
  return LQ_OK;
}

// info <- 0 with a kernel (no memset node in captured graphs).
__global__ void k_zero_i32(int32_t* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

hipError_t zero_info(int32_t* info, int batch, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_i32, dim3((batch + 255) / 256), dim3(256), 0, st, info, batch);
  return hipGetLastError();
}

}  // namespace
}  // namespace lq

using namespace lq;

extern "C" size_t lq_bt_workspace_bytes(int32_t batch, int32_t Nb, int32_t n, lq_bt_method method) {
  if (batch <= 0 || Nb <= 0 || n <= 0) return 0;
  const size_t blocks = (size_t)batch * Nb * n * n * sizeof(double), vec = (size_t)batch * Nb * n * sizeof(double);
  switch (method) {
    case LQ_BT_CR: return 4 * blocks;               // L (in place of M), coupling, U, Y
    case LQ_BT_PCR: return 9 * blocks + 4 * vec;    // M, K (two levels each), L, U, Y; b (two), bt
    case LQ_BT_PCG: return 2 * blocks + 5 * vec;    // L, D^{-1}; r, z, p, q, u
  }
  return 0;
}

extern "C" int lq_bt_cr_factor(int32_t batch, int32_t Nb, int32_t n, const double* M, const double* K, void* ws,
                               int32_t* info, hipStream_t st) {
  clear_error();
  int rc = check_sizes(batch, Nb, n);
  if (rc) return rc;
  if (!M || (Nb > 1 && !K) || !ws || !info) return bt_fail(LQ_EINVAL, "lq_bt_cr_factor: M, K, ws, info are required");
  const BT t{batch, Nb, n, (int64_t)n * n};
  const size_t blocks = (size_t)batch * Nb * n * n;
  double* Lw = (double*)ws;
  double* Kw = Lw + blocks;
  double* U = Kw + blocks;
  double* Y = U + blocks;
  const size_t lds = sizeof(wg::Smem);
  hipError_t e = zero_info(info, batch, st);
  if (e == hipSuccess) e = lds_ready((const void*)k_cr_elim);
  if (e == hipSuccess) e = lds_ready((const void*)k_cr_update);
  if (e == hipSuccess) e = lds_ready((const void*)k_cr_last);
  if (e != hipSuccess) return launch_rc(e);
  hipLaunchKernelGGL(k_cr_init, dim3(Nb, batch), dim3(NT), 0, st, t, M, K, Lw, Kw);
  for (int s = 1; s < Nb; s *= 2) {
    const int elim = (Nb - s + 2 * s - 1) / (2 * s);  // k = s (2i + 1) < Nb
    const int keep = (Nb + 2 * s - 1) / (2 * s);      // j = 2 s i < Nb
    hipLaunchKernelGGL(k_cr_elim, dim3(elim, batch), dim3(NT), lds, st, t, s, Lw, Kw, U, Y, info);
    hipLaunchKernelGGL(k_cr_update, dim3(keep, batch), dim3(NT), lds, st, t, s, Lw, Kw, U, Y);
  }
  hipLaunchKernelGGL(k_cr_last, dim3(batch), dim3(NT), lds, st, t, Lw, info);
  return launch_rc(hipGetLastError());
}

extern "C" int lq_bt_cr_solve(int32_t batch, int32_t Nb, int32_t n, const void* ws, const double* b, double* x,
                              hipStream_t st) {
  clear_error();
  int rc = check_sizes(batch, Nb, n);
  if (rc) return rc;
  if (!ws || !b || !x) return bt_fail(LQ_EINVAL, "lq_bt_cr_solve: ws, b, x are required");
  if (b == x) return bt_fail(LQ_EINVAL, "lq_bt_cr_solve: b and x must not be the same array");
  const BT t{batch, Nb, n, (int64_t)n * n};
  const size_t blocks = (size_t)batch * Nb * n * n;
  const double* Lw = (const double*)ws;
  const double* U = Lw + 2 * blocks;
  const double* Y = Lw + 3 * blocks;
  hipError_t e = lds_ready((const void*)k_cr_solve);
  if (e != hipSuccess) return launch_rc(e);
  hipLaunchKernelGGL(k_cr_solve, dim3(batch), dim3(NT), sizeof(wg::Smem), st, t, Lw, U, Y, b, x);
  return launch_rc(hipGetLastError());
}

extern "C" int lq_bt_pcr_solve(int32_t batch, int32_t Nb, int32_t n, const double* M, const double* K,
                               const double* b, double* x, void* ws, int32_t* info, hipStream_t st) {
  clear_error();
  int rc = check_sizes(batch, Nb, n);
  if (rc) return rc;
  if (!M || (Nb > 1 && !K) || !b || !x || !ws || !info) return bt_fail(LQ_EINVAL, "lq_bt_pcr_solve: M, K, b, x, ws, info are required");
  const BT t{batch, Nb, n, (int64_t)n * n};
  const size_t blocks = (size_t)batch * Nb * n * n, vec = (size_t)batch * Nb * n;
  double* w = (double*)ws;
  double* Mw[2] = {w, w + blocks};
  double* Kw[2] = {w + 2 * blocks, w + 3 * blocks};
  double* L = w + 4 * blocks;
  double* U = w + 5 * blocks;
  double* Y = w + 6 * blocks;
  double* bw[2] = {w + 9 * blocks, w + 9 * blocks + vec};
  double* bt = w + 9 * blocks + 2 * vec;
  const size_t lds = sizeof(wg::Smem);
  hipError_t e = zero_info(info, batch, st);
  if (e == hipSuccess) e = lds_ready((const void*)k_pcr_elim);
  if (e == hipSuccess) e = lds_ready((const void*)k_pcr_update);
  if (e == hipSuccess) e = lds_ready((const void*)k_pcr_last);
  if (e != hipSuccess) return launch_rc(e);
  const double* Kin = Nb > 1 ? K : M;  // (not read when Nb == 1)
  hipLaunchKernelGGL(k_pcr_init, dim3(Nb, batch), dim3(NT), 0, st, t, M, Kin, b, Mw[0], Kw[0], bw[0]);
  int cur = 0;
  for (int s = 1; s < Nb; s *= 2) {
    hipLaunchKernelGGL(k_pcr_elim, dim3(Nb, batch), dim3(NT), lds, st, t, s, Mw[cur], Kw[cur], bw[cur], L, U, Y, bt, info);
    hipLaunchKernelGGL(k_pcr_update, dim3(Nb, batch), dim3(NT), lds, st, t, s, Mw[cur], bw[cur], U, Y, bt,
                       Mw[1 - cur], Kw[1 - cur], bw[1 - cur]);
    cur = 1 - cur;
  }
  hipLaunchKernelGGL(k_pcr_last, dim3(Nb, batch), dim3(NT), lds, st, t, Mw[cur], bw[cur], L, x, info);
  return launch_rc(hipGetLastError());
}

extern "C" int lq_bt_pcg(int32_t batch, int32_t Nb, int32_t n, const double* M, const double* K, const double* b,
                         double* x, int32_t precond, double tol, int32_t max_it, void* ws, int32_t* iters,
                         double* rel_res, int32_t* info, hipStream_t st) {
  clear_error();
  int rc = check_sizes(batch, Nb, n);
  if (rc) return rc;
  if (!M || (Nb > 1 && !K) || !b || !x || !ws || !info) return bt_fail(LQ_EINVAL, "lq_bt_pcg: M, K, b, x, ws, info are required");
  if (precond != LQ_BT_PRECOND_JACOBI && precond != LQ_BT_PRECOND_STAIR) return bt_fail(LQ_EINVAL, "lq_bt_pcg: unknown preconditioner");
  if (!(tol >= 0.0) || max_it < 0) return bt_fail(LQ_EINVAL, "lq_bt_pcg: tol >= 0 and max_it >= 0 are required");
  const BT t{batch, Nb, n, (int64_t)n * n};
  const size_t blocks = (size_t)batch * Nb * n * n;
  double* L = (double*)ws;
  double* Dinv = L + blocks;
  double* work = Dinv + blocks;
  const size_t lds = sizeof(wg::Smem);
  hipError_t e = zero_info(info, batch, st);
  if (e == hipSuccess) e = lds_ready((const void*)k_pcg_inv);
  if (e == hipSuccess) e = lds_ready((const void*)k_pcg);
  if (e != hipSuccess) return launch_rc(e);
  hipLaunchKernelGGL(k_pcg_inv, dim3(Nb, batch), dim3(NT), lds, st, t, M, L, Dinv, info);
  hipLaunchKernelGGL(k_pcg, dim3(batch), dim3(NT), lds, st, t, M, Nb > 1 ? K : M, b, Dinv,
                     precond == LQ_BT_PRECOND_STAIR ? 1 : 0, tol, max_it, x, work, iters, rel_res, info);
  return launch_rc(hipGetLastError());
}
