// Workgroup-level float64 dense linear algebra on row-major matrices in global memory, for the
// kernels whose operands are whole n x n blocks (block-tridiagonal cyclic reduction, the
// parallel-in-time interval recursion and its Schur complement).  Every routine is called by all
// NT threads of a workgroup with uniform arguments; it synchronises the workgroup on entry and
// before it returns, so consecutive calls may read what the previous one wrote.
//
// Layout: element (i, j) of a matrix X with leading dimension ldx is X[i * ldx + j].
// Lower-triangular factors are stored in full n x n storage; their upper parts are not read.
//
// gemm: 64 x 64 output tiles, k in steps of 16 staged in LDS (k-major, so that each thread's four
// rows and four columns are contiguous), 4 x 4 accumulators per thread.  potrf: right-looking,
// 64-column panels: the diagonal block is factored in LDS, the panel below it solved row by row
// (rows in parallel), the trailing lower triangle updated by gemm.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace lq {
namespace wg {

constexpr int NT = 256;  // threads per workgroup of every kernel that uses these routines
constexpr int TB = 64;   // gemm output tile
constexpr int KB = 16;   // gemm k step
constexpr int DB = 64;   // potrf panel width

// LDS of the routines; kernels place one in dynamic shared memory.
struct Smem {
  double a[KB][TB + 2];
  double b[KB][TB + 2];
  double d[DB][DB + 1];
  double red[NT];
  int flag;
};

__device__ __forceinline__ void sync() { __syncthreads(); }

// C = alpha op(A) op(B) + beta C for the m x n matrix C (UPLO = 1: only entries i >= j are
// written, and tiles entirely above the diagonal are skipped).  op(A) is m x k (A stored k x m
// when TA), op(B) is k x n (B stored n x k when TBT).  beta == 0 does not read C.
template <bool TA, bool TBT, int UPLO>
__device__ void gemm(int m, int n, int k, double alpha, const double* __restrict__ A, int lda,
                     const double* __restrict__ B, int ldb, double beta, double* C, int ldc, Smem& sm) {
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  sync();
  for (int i0 = 0; i0 < m; i0 += TB)
    for (int j0 = 0; j0 < n; j0 += TB) {
      if (UPLO == 1 && j0 > i0 + TB - 1) continue;
      double acc[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
      for (int k0 = 0; k0 < k; k0 += KB) {
        for (int e = tid; e < TB * KB; e += NT) {
          int r, kk;
          if (TA) { r = e % TB; kk = e / TB; } else { kk = e % KB; r = e / KB; }
          const int gi = i0 + r, gk = k0 + kk;
          double v = 0.0;
          if (gi < m && gk < k) v = TA ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk];
          sm.a[kk][r] = v;
        }
        for (int e = tid; e < TB * KB; e += NT) {
          int c, kk;
          if (TBT) { kk = e % KB; c = e / KB; } else { c = e % TB; kk = e / TB; }
          const int gj = j0 + c, gk = k0 + kk;
          double v = 0.0;
          if (gj < n && gk < k) v = TBT ? B[(int64_t)gj * ldb + gk] : B[(int64_t)gk * ldb + gj];
          sm.b[kk][c] = v;
        }
        sync();
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
          double av[4], bv[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) av[r] = sm.a[kk][ty * 4 + r];
#pragma unroll
          for (int c = 0; c < 4; ++c) bv[c] = sm.b[kk][tx * 4 + c];
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = fma(av[r], bv[c], acc[r][c]);
        }
        sync();
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int gi = i0 + ty * 4 + r, gj = j0 + tx * 4 + c;
          if (gi < m && gj < n && (UPLO == 0 || gi >= gj)) {
            double* p = C + (int64_t)gi * ldc + gj;
            *p = beta == 0.0 ? alpha * acc[r][c] : fma(alpha, acc[r][c], beta * *p);
          }
        }
    }
  sync();
}

// Y = X for an m x n block (Y and X may have different leading dimensions).
__device__ inline void copy(int m, int n, const double* X, int ldx, double* Y, int ldy) {
  sync();
  for (int e = threadIdx.x; e < m * n; e += NT) {
    const int i = e / n, j = e % n;
    Y[(int64_t)i * ldy + j] = X[(int64_t)i * ldx + j];
  }
  sync();
}

// Y = X^T (X is m x n, Y is n x m).
__device__ inline void transpose(int m, int n, const double* X, int ldx, double* Y, int ldy) {
  sync();
  for (int e = threadIdx.x; e < m * n; e += NT) {
    const int j = e / m, i = e % m;
    Y[(int64_t)j * ldy + i] = X[(int64_t)i * ldx + j];
  }
  sync();
}

__device__ inline void fill(int m, int n, double v, double* Y, int ldy) {
  sync();
  for (int e = threadIdx.x; e < m * n; e += NT) Y[(int64_t)(e / n) * ldy + e % n] = v;
  sync();
}

// Zero the strictly upper part of the n x n matrix L (so that it can be used as a full operand).
__device__ inline void zero_upper(int n, double* L, int ldl) {
  sync();
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int i = e / n, j = e % n;
    if (j > i) L[(int64_t)i * ldl + j] = 0.0;
  }
  sync();
}

// X <- X L^{-T} for the m x nb block X and the nb x nb lower-triangular L held in sm.d (nb <= DB):
// rows in parallel, 16 columns at a time in registers.
__device__ inline void trsm_rlt_lds(int m, int nb, double* X, int ldx, Smem& sm) {
  for (int r = threadIdx.x; r < m; r += NT) {
    double* x = X + (int64_t)r * ldx;
    for (int c0 = 0; c0 < nb; c0 += 16) {
      double y[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) y[c] = c0 + c < nb ? x[c0 + c] : 0.0;
      for (int t = 0; t < c0; ++t) {
        const double xt = x[t];
#pragma unroll
        for (int c = 0; c < 16; ++c)
          if (c0 + c < nb) y[c] = fma(-xt, sm.d[c0 + c][t], y[c]);
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        if (c0 + c < nb) {
#pragma unroll
          for (int t = 0; t < c; ++t) y[c] = fma(-y[t], sm.d[c0 + c][c0 + t], y[c]);
          y[c] = y[c] / sm.d[c0 + c][c0 + c];
        }
      }
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c0 + c < nb) x[c0 + c] = y[c];
    }
  }
}

// In-place Cholesky of the n x n symmetric matrix A (lower part read and written: A = L L^T).
// Returns (uniformly) 0, or 1 + the index of the first pivot that is not positive (1 + n + j if
// it is not finite); failed pivots are replaced by 1 so that the factor stays finite.
__device__ inline int potrf(int n, double* A, int lda, Smem& sm) {
  const int tid = threadIdx.x;
  sync();
  if (tid == 0) sm.flag = 0;
  for (int j0 = 0; j0 < n; j0 += DB) {
    const int nb = n - j0 < DB ? n - j0 : DB;
    sync();
    for (int e = tid; e < DB * DB; e += NT) {
      const int r = e / DB, c = e % DB;
      sm.d[r][c] = (r < nb && c <= r) ? A[(int64_t)(j0 + r) * lda + j0 + c] : 0.0;
    }
    sync();
    for (int j = 0; j < nb; ++j) {
      if (tid == 0) {
        double d = sm.d[j][j];
        const bool good = d > 0.0 && d <= 1.7976931348623157e308;
        if (!good && sm.flag == 0) sm.flag = 1 + j0 + j + (isfinite(d) ? 0 : n);
        sm.d[j][j] = sqrt(good ? d : 1.0);
      }
      sync();
      const double inv = 1.0 / sm.d[j][j];
      for (int r = j + 1 + tid; r < nb; r += NT) sm.d[r][j] *= inv;
      sync();
      const int w = nb - j - 1;
      for (int e = tid; e < w * w; e += NT) {
        const int r = j + 1 + e / w, c = j + 1 + e % w;
        if (c <= r) sm.d[r][c] = fma(-sm.d[r][j], sm.d[c][j], sm.d[r][c]);
      }
      sync();
    }
    for (int e = tid; e < nb * nb; e += NT) {
      const int r = e / nb, c = e % nb;
      if (c <= r) A[(int64_t)(j0 + r) * lda + j0 + c] = sm.d[r][c];
    }
    const int m = n - j0 - nb;
    if (m > 0) {
      // panel below the diagonal block: X <- X L_jj^{-T}
      trsm_rlt_lds(m, nb, A + (int64_t)(j0 + nb) * lda + j0, lda, sm);
      sync();
      // trailing lower triangle: A22 -= X X^T
      gemm<false, true, 1>(m, m, nb, -1.0, A + (int64_t)(j0 + nb) * lda + j0, lda,
                           A + (int64_t)(j0 + nb) * lda + j0, lda, 1.0,
                           A + (int64_t)(j0 + nb) * lda + j0 + nb, lda, sm);
    }
  }
  sync();
  const int f = sm.flag;
  sync();
  return f;
}

// X <- X L^{-T} for the m x n matrix X and the n x n lower-triangular L in global memory:
// 64-column panels of L staged in LDS, the columns to the right updated by gemm.
__device__ inline void trsm_rlt(int m, int n, const double* L, int ldl, double* X, int ldx, Smem& sm) {
  const int tid = threadIdx.x;
  for (int j0 = 0; j0 < n; j0 += DB) {
    const int nb = n - j0 < DB ? n - j0 : DB;
    sync();
    for (int e = tid; e < DB * DB; e += NT) {
      const int r = e / DB, c = e % DB;
      sm.d[r][c] = (r < nb && c <= r) ? L[(int64_t)(j0 + r) * ldl + j0 + c] : 0.0;
    }
    sync();
    trsm_rlt_lds(m, nb, X + j0, ldx, sm);
    sync();
    const int rest = n - j0 - nb;
    if (rest > 0)  // X[:, j0+nb:] -= X[:, j0:j0+nb] L[j0+nb:, j0:j0+nb]^T
      gemm<false, true, 0>(m, rest, nb, -1.0, X + j0, ldx, L + (int64_t)(j0 + nb) * ldl + j0, ldl, 1.0,
                           X + j0 + nb, ldx, sm);
  }
  sync();
}

// ---- vectors (one workgroup; the vector lives in global memory) -----------------------------

// y = alpha op(A) x + beta y for the m x n matrix A (op(A) = A^T when T: then y has n entries).
// beta == 0 does not read y.  x and y must not overlap.
template <bool T>
__device__ inline void gemv(int m, int n, double alpha, const double* A, int lda, const double* x, double beta,
                            double* y) {
  sync();
  if (!T) {
    // a wavefront per row, lanes over the columns, reduced by shuffles
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int r = w; r < m; r += NT / 64) {
      double s = 0.0;
      for (int c = lane; c < n; c += 64) s = fma(A[(int64_t)r * lda + c], x[c], s);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
      if (lane == 0) y[r] = beta == 0.0 ? alpha * s : fma(alpha, s, beta * y[r]);
    }
  } else {
    // a thread per column (rows read coalesced across threads)
    for (int c = threadIdx.x; c < n; c += NT) {
      double s = 0.0;
      for (int r = 0; r < m; ++r) s = fma(A[(int64_t)r * lda + c], x[r], s);
      y[c] = beta == 0.0 ? alpha * s : fma(alpha, s, beta * y[c]);
    }
  }
  sync();
}

// In place x <- L^{-1} x (TR = false) or x <- L^{-T} x (TR = true) for the n x n lower-triangular
// L (n <= NT): the vector is held in LDS, one column (or row) of L per step.
template <bool TR>
__device__ inline void trsv(int n, const double* L, int ldl, double* x, Smem& sm) {
  const int i = threadIdx.x;
  sync();
  if (i < n) sm.red[i] = x[i];
  for (int s = 0; s < n; ++s) {
    const int t = TR ? n - 1 - s : s;
    sync();
    const double xt = sm.red[t] / L[(int64_t)t * ldl + t];
    sync();
    if (i == t) sm.red[i] = xt;
    else if (!TR && i > t && i < n) sm.red[i] = fma(-L[(int64_t)i * ldl + t], xt, sm.red[i]);
    else if (TR && i < t) sm.red[i] = fma(-L[(int64_t)t * ldl + i], xt, sm.red[i]);
  }
  sync();
  if (i < n) x[i] = sm.red[i];
  sync();
}

// max |v_i| over a vector, reduced over the workgroup (NaN propagates).
__device__ inline double absmax(int n, const double* v, Smem& sm) {
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) {
    const double a = fabs(v[i]);
    m = (a > m || a != a) ? a : m;
  }
  sync();
  sm.red[threadIdx.x] = m;
  sync();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double o = sm.red[threadIdx.x + s];
      const double c = sm.red[threadIdx.x];
      sm.red[threadIdx.x] = (o > c || o != o) ? o : c;
    }
    sync();
  }
  const double r = sm.red[0];
  sync();
  return r;
}

// sum of x_i y_i over the workgroup.
__device__ inline double dot(int n, const double* x, const double* y, Smem& sm) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) s = fma(x[i], y[i], s);
  sync();
  sm.red[threadIdx.x] = s;
  sync();
  for (int st = NT / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sm.red[threadIdx.x] += sm.red[threadIdx.x + st];
    sync();
  }
  const double r = sm.red[0];
  sync();
  return r;
}

}  // namespace wg
}  // namespace lq
