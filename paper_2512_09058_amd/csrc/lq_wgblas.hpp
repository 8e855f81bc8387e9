// Workgroup-level float64 dense linear algebra on row-major matrices in global memory, for the
// kernels whose operands are whole n x n blocks (block-tridiagonal cyclic reduction, the
// parallel-in-time interval recursion and its Schur complement).  Every routine is called by all
// NT threads of a workgroup with uniform arguments; it synchronises the workgroup on entry and
// before it returns, so consecutive calls may read what the previous one wrote.
//
// Layout: element (i, j) of a matrix X with leading dimension ldx is X[i * ldx + j].
// Lower-triangular factors are stored in full n x n storage; their upper parts are not read.
//
// gemm: 64 x 64 output tiles, k in steps of 16 staged in LDS (k-major), each wavefront a 32 x 32
// quadrant of 2 x 2 float64 16x16x4 matrix-core fragments; the next k step's operands are loaded
// into registers (from clamped, always valid addresses, masked when stored to LDS) while the
// current one is multiplied.  potrf: right-looking,
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
static_assert(NT == 256 && TB == 64, "gemm: four wavefronts, one 32 x 32 quadrant of the 64 x 64 tile each");

typedef double d4 __attribute__((ext_vector_type(4)));

// LDS of the routines; kernels place one in dynamic shared memory.
struct Smem {
  double a[KB][TB + 2];
  double b[KB][TB + 2];
  double d[DB][DB + 1];
  double red[NT];
  int flag;
};

__device__ __forceinline__ void sync() { __syncthreads(); }

// Lane k (a constant after unrolling) of each 16-lane row, broadcast to the whole row: one 64-bit
// DPP row_newbcast, no scalar register round trip.
__device__ __forceinline__ double row_bcast(double v, int k) {
  long x = __double_as_longlong(v);
  switch (k) {
#define LQ_RB(K) \
  case K:        \
    x = __builtin_amdgcn_update_dpp((long)0, x, 0x150 + K, 0xF, 0xF, true); \
    break;
    LQ_RB(0) LQ_RB(1) LQ_RB(2) LQ_RB(3) LQ_RB(4) LQ_RB(5) LQ_RB(6) LQ_RB(7) LQ_RB(8) LQ_RB(9) LQ_RB(10)
    LQ_RB(11) LQ_RB(12) LQ_RB(13) LQ_RB(14) LQ_RB(15)
#undef LQ_RB
  }
  return __longlong_as_double(x);
}

// Value of lane l (uniform l) of a wavefront for every lane.
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __hiloint2double(hi, lo);
}


// C = alpha op(A) op(B) + beta C for the m x n matrix C (UPLO = 1: only entries i >= j are
// written, and tiles entirely above the diagonal are skipped).  op(A) is m x k (A stored k x m
// when TA), op(B) is k x n (B stored n x k when TBT).  AUP: op(A) is upper triangular (entries
// with column < row are zero and are not read), so each row tile starts its k loop at its first
// row.  beta == 0 does not read C.
template <bool TA, bool TBT, int UPLO, bool AUP = false>
__device__ void gemm(int m, int n, int k, double alpha, const double* __restrict__ A, int lda,
                     const double* __restrict__ B, int ldb, double beta, double* C, int ldc, Smem& sm) {
  constexpr int PER = TB * KB / NT;  // operand elements per thread and k step
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lg = lane >> 4, lc = lane & 15, wy = w >> 1, wx = w & 1;  // wavefront w: 32 x 32 quadrant (wy, wx)
  const int nti = (m + TB - 1) / TB, ntj = (n + TB - 1) / TB;
  sync();
  if (k <= 0 || m <= 0 || n <= 0) return;
  // The (tile, k step) sequence is walked as one pipeline: while one step is multiplied, the
  // operands of the next step -- the next k step of this tile or the first of the next tile --
  // are loaded, so no tile boundary exposes a full load latency.
  auto kbeg = [&](int ti) { return AUP ? ((ti * TB) / KB) * KB : 0; };
  auto next_tile = [&](int& ti, int& tj) {  // advance to the next tile to compute (ti = nti: done)
    do {
      if (++tj >= ntj) { tj = 0; ++ti; }
    } while (ti < nti && (UPLO == 1 && tj * TB > ti * TB + TB - 1));
  };
  auto skip_empty = [&](int& ti, int& tj) {  // tiles whose k range is empty are written directly
    while (ti < nti && kbeg(ti) >= k) {
      for (int fi = 0; fi < 2; ++fi)
        for (int fj = 0; fj < 2; ++fj)
          for (int t = 0; t < 4; ++t) {
            const int gi = ti * TB + 32 * wy + 16 * fi + 4 * t + lg, gj = tj * TB + 32 * wx + 16 * fj + lc;
            if (gi < m && gj < n && (UPLO == 0 || gi >= gj)) {
              double* p = C + (int64_t)gi * ldc + gj;
              *p = beta == 0.0 ? 0.0 : beta * *p;
            }
          }
      next_tile(ti, tj);
    }
  };
  double ra[PER], rb[PER];
  unsigned va = 0, vb = 0;
  auto load = [&](int i0, int j0, int k0) {
    va = vb = 0;
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + t * NT;
      int r, kk;
      if (TA) { r = e % TB; kk = e / TB; } else { kk = e % KB; r = e / KB; }
      const int gi = i0 + r, gk = k0 + kk;
      va |= (gi < m && gk < k) ? (1u << t) : 0u;
      const int ci = gi < m ? gi : m - 1, ck = gk < k ? gk : k - 1;
      ra[t] = TA ? A[(int64_t)ck * lda + ci] : A[(int64_t)ci * lda + ck];
    }
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + t * NT;
      int c, kk;
      if (TBT) { kk = e % KB; c = e / KB; } else { c = e % TB; kk = e / TB; }
      const int gj = j0 + c, gk = k0 + kk;
      vb |= (gj < n && gk < k) ? (1u << t) : 0u;
      const int cj = gj < n ? gj : n - 1, ck = gk < k ? gk : k - 1;
      rb[t] = TBT ? B[(int64_t)cj * ldb + ck] : B[(int64_t)ck * ldb + cj];
    }
  };
  int ti = 0, tj = 0;
  skip_empty(ti, tj);
  if (ti >= nti) { sync(); return; }
  int k0 = kbeg(ti);
  load(ti * TB, tj * TB, k0);
  d4 acc[2][2];
#pragma unroll
  for (int fi = 0; fi < 2; ++fi)
#pragma unroll
    for (int fj = 0; fj < 2; ++fj) acc[fi][fj] = d4{0.0, 0.0, 0.0, 0.0};
  while (ti < nti) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + t * NT;
      if (TA) sm.a[e / TB][e % TB] = (va >> t) & 1u ? ra[t] : 0.0;
      else sm.a[e % KB][e / KB] = (va >> t) & 1u ? ra[t] : 0.0;
      if (TBT) sm.b[e % KB][e / KB] = (vb >> t) & 1u ? rb[t] : 0.0;
      else sm.b[e / TB][e % TB] = (vb >> t) & 1u ? rb[t] : 0.0;
    }
    sync();
    // next step of the pipeline
    int nti_ = ti, ntj_ = tj, nk0 = k0 + KB;
    const bool last = nk0 >= k;
    if (last) {
      next_tile(nti_, ntj_);
      skip_empty(nti_, ntj_);
      nk0 = nti_ < nti ? kbeg(nti_) : 0;
    }
    if (nti_ < nti) load(nti_ * TB, ntj_ * TB, nk0);
    // the finishing tile's C entries (when beta != 0) load while its last step is multiplied
    double cv[16];
    if (last && beta != 0.0) {
#pragma unroll
      for (int fi = 0; fi < 2; ++fi)
#pragma unroll
        for (int fj = 0; fj < 2; ++fj)
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int gi = ti * TB + 32 * wy + 16 * fi + 4 * t + lg, gj = tj * TB + 32 * wx + 16 * fj + lc;
            cv[(fi * 2 + fj) * 4 + t] = C[(int64_t)(gi < m ? gi : m - 1) * ldc + (gj < n ? gj : n - 1)];
          }
    }
    // 16x16x4 float64 matrix-core steps: lane 16 g + c supplies A(row c, k = 4q + g) and
    // B(k = 4q + g, column c) and accumulates D(row 4t + g, column c) in slot t
#pragma unroll
    for (int q = 0; q < KB / 4; ++q) {
      const double a0 = sm.a[4 * q + lg][32 * wy + lc], a1 = sm.a[4 * q + lg][32 * wy + 16 + lc];
      const double b0 = sm.b[4 * q + lg][32 * wx + lc], b1 = sm.b[4 * q + lg][32 * wx + 16 + lc];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    sync();
    if (last) {
#pragma unroll
      for (int fi = 0; fi < 2; ++fi)
#pragma unroll
        for (int fj = 0; fj < 2; ++fj) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int gi = ti * TB + 32 * wy + 16 * fi + 4 * t + lg, gj = tj * TB + 32 * wx + 16 * fj + lc;
            if (gi < m && gj < n && (UPLO == 0 || gi >= gj)) {
              const double v = acc[fi][fj][t];
              C[(int64_t)gi * ldc + gj] = beta == 0.0 ? alpha * v : fma(alpha, v, beta * cv[(fi * 2 + fj) * 4 + t]);
            }
          }
          acc[fi][fj] = d4{0.0, 0.0, 0.0, 0.0};
        }
    }
    ti = nti_;
    tj = ntj_;
    k0 = nk0;
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
// rows in parallel, TC columns at a time in registers.
__device__ inline void trsm_rlt_lds(int m, int nb, double* X, int ldx, Smem& sm) {
  constexpr int TC = 8;
  for (int r = threadIdx.x; r < m; r += NT) {
    double* x = X + (int64_t)r * ldx;
    for (int c0 = 0; c0 < nb; c0 += TC) {
      double y[TC];
#pragma unroll
      for (int c = 0; c < TC; ++c) y[c] = c0 + c < nb ? x[c0 + c] : 0.0;
      for (int t = 0; t < c0; ++t) {
        const double xt = x[t];
#pragma unroll
        for (int c = 0; c < TC; ++c) y[c] = fma(-xt, sm.d[c0 + c < nb ? c0 + c : 0][t], y[c]);
      }
#pragma unroll
      for (int c = 0; c < TC; ++c) {
        if (c0 + c < nb) {
#pragma unroll
          for (int t = 0; t < c; ++t) y[c] = fma(-y[t], sm.d[c0 + c][c0 + t], y[c]);
          y[c] = y[c] / sm.d[c0 + c][c0 + c];
        }
      }
#pragma unroll
      for (int c = 0; c < TC; ++c)
        if (c0 + c < nb) x[c0 + c] = y[c];
    }
  }
}

// In-place Cholesky of the n x n symmetric matrix A (lower part read and written: A = L L^T).
// Returns (uniformly) 0, or 1 + the index of the first pivot that is not positive (1 + n + j if
// it is not finite); failed pivots are replaced by 1 so that the factor stays finite.
// Right-looking with 16-column panels: wavefront 0 factors the 16 x 16 diagonal block in registers
// (lane r holds row r; pivots and column entries move by DPP row broadcasts, no barrier), the rows below it
// are solved against it in parallel, and the trailing lower triangle is updated by gemm.
__device__ inline int potrf(int n, double* A, int lda, Smem& sm) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  sync();
  if (tid == 0) sm.flag = 0;
  for (int j0 = 0; j0 < n; j0 += 16) {
    const int nb = n - j0 < 16 ? n - j0 : 16;
    if (w == 0) {
      const bool on = lane < nb;
      double h[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) h[c] = (on && c <= lane && c < nb) ? A[(int64_t)(j0 + lane) * lda + j0 + c] : 0.0;
      int kind = 0;
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        if (c < nb) {
          double d = row_bcast(h[c], c);
          const bool good = d > 0.0 && d <= 1.7976931348623157e308;
          if (!good && kind == 0) kind = 1 + j0 + c + (isfinite(d) ? 0 : n);
          d = good ? d : 1.0;
          const double sq = sqrt(d), inv = 1.0 / sq;
          h[c] = lane == c ? sq : (lane > c ? h[c] * inv : h[c]);
#pragma unroll
          for (int cc = c + 1; cc < 16; ++cc) {
            if (cc < nb) {
              const double lcc = row_bcast(h[c], cc);  // L(cc, c)
              if (lane >= cc) h[cc] = fma(-h[c], lcc, h[cc]);
            }
          }
        }
      }
      if (on) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const double v = c <= lane ? h[c] : 0.0;
          if (c < nb) {
            sm.d[lane][c] = v;
            if (c <= lane) A[(int64_t)(j0 + lane) * lda + j0 + c] = v;
          }
        }
      }
      if (lane == 0 && kind && sm.flag == 0) sm.flag = kind;
    }
    sync();
    const int m = n - j0 - nb;
    if (m > 0) {
      trsm_rlt_lds(m, nb, A + (int64_t)(j0 + nb) * lda + j0, lda, sm);  // panel: X <- X L_jj^{-T}
      sync();
      gemm<false, true, 1>(m, m, nb, -1.0, A + (int64_t)(j0 + nb) * lda + j0, lda,
                           A + (int64_t)(j0 + nb) * lda + j0, lda, 1.0,
                           A + (int64_t)(j0 + nb) * lda + j0 + nb, lda, sm);  // A22 -= X X^T
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
// beta == 0 does not read y.  x and y must not overlap.  Both forms read A coalesced: A x with a
// wavefront per row (lanes over the columns, shuffle reduction); A^T x with the rows dealt over
// the wavefronts (lanes over the columns) and the per-wavefront sums added through LDS.
template <bool T>
__device__ inline void gemv(int m, int n, double alpha, const double* A, int lda, const double* x, double beta,
                            double* y, Smem& sm) {
  sync();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int NW = NT / 64;
  if (!T) {
    for (int r = w; r < m; r += NW) {
      double s = 0.0;
      for (int c = lane; c < n; c += 64) s = fma(A[(int64_t)r * lda + c], x[c], s);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
      if (lane == 0) y[r] = beta == 0.0 ? alpha * s : fma(alpha, s, beta * y[r]);
    }
    sync();
  } else {
    double* part = &sm.d[0][0];  // NW x n partial sums (n <= 1040)
    for (int c0 = 0; c0 < n; c0 += 64) {
      const int c = c0 + lane;
      double s = 0.0;
      if (c < n) {
#pragma unroll 4
        for (int r = w; r < m; r += NW) s = fma(A[(int64_t)r * lda + c], x[r], s);
        part[w * n + c] = s;
      }
    }
    sync();
    for (int c = threadIdx.x; c < n; c += NT) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) s += part[q * n + c];
      y[c] = beta == 0.0 ? alpha * s : fma(alpha, s, beta * y[c]);
    }
    sync();
  }
}

// In place x <- L^{-1} x (TR = false) or x <- L^{-T} x (TR = true) for an n x n lower-triangular L
// (n <= NT) given by accessors Lat(i, j) (j <= i) and dinv_at(i) = 1 / L(i, i).  Blocked by 16:
// wavefront 0 solves each 16 x 16 diagonal block in registers (readlane broadcasts, no barrier),
// then all threads update the remaining entries, one row (or column) of the block per thread.
// The vector lives in LDS during the solve; x is read from and written back to global memory.
template <bool TR, class LAT, class DAT>
__device__ inline void trsv_blocked(int n, LAT Lat, DAT dinv_at, double* x, Smem& sm) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  sync();
  if (tid < n) sm.red[tid] = x[tid];
  sync();
  const int nblk = (n + 15) / 16;
  for (int bi = 0; bi < nblk; ++bi) {
    const int c0 = TR ? (nblk - 1 - bi) * 16 : bi * 16;
    const int nb = n - c0 < 16 ? n - c0 : 16;
    if (w == 0) {
      const bool on = lane < nb;
      double xi = on ? sm.red[c0 + lane] : 0.0;
      const double d = on ? dinv_at(c0 + lane) : 0.0;
      double Lv[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        if (!TR) Lv[t] = (on && t < lane) ? Lat(c0 + lane, c0 + t) : 0.0;      // row of the block
        else Lv[t] = (on && t < nb && t > lane) ? Lat(c0 + t, c0 + lane) : 0.0;  // column of the block
      }
      if (!TR) {
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          if (t < nb) {
            if (lane == t) xi *= d;
            const double xt = lane_value(xi, t);
            if (lane > t) xi = fma(-Lv[t], xt, xi);
          }
        }
      } else {
#pragma unroll
        for (int t = 15; t >= 0; --t) {
          if (t < nb) {
            if (lane == t) xi *= d;
            const double xt = lane_value(xi, t);
            if (lane < t) xi = fma(-Lv[t], xt, xi);
          }
        }
      }
      if (on) sm.red[c0 + lane] = xi;
    }
    sync();
    if (!TR) {
      for (int i = c0 + nb + tid; i < n; i += NT) {
        double v = sm.red[i];
        for (int t = 0; t < nb; ++t) v = fma(-Lat(i, c0 + t), sm.red[c0 + t], v);
        sm.red[i] = v;
      }
    } else {
      for (int i = tid; i < c0; i += NT) {
        double v = sm.red[i];
        for (int t = 0; t < nb; ++t) v = fma(-Lat(c0 + t, i), sm.red[c0 + t], v);
        sm.red[i] = v;
      }
    }
    sync();
  }
  if (tid < n) x[tid] = sm.red[tid];
  sync();
}

// Dense lower-triangular L (row-major, leading dimension ldl).
template <bool TR>
__device__ inline void trsv(int n, const double* L, int ldl, double* x, Smem& sm) {
  trsv_blocked<TR>(
      n, [&](int i, int j) { return L[(int64_t)i * ldl + j]; }, [&](int i) { return 1.0 / L[(int64_t)i * ldl + i]; },
      x, sm);
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
