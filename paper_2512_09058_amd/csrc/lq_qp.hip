// Box-constrained LQ QPs: proximal augmented Lagrangian with semismooth Newton inner steps (the
// paper's Sec. "Solving problems with inequality constraints") and the exact line search of Sec.
// "Parallel exact line search".  The Newton systems (eq. newton-sys-with-x0 with x_0 eliminated,
// eq. elim-x0) are written in the layout of the LQ data and solved by lq_factor / lq_solve; the
// kernels here form them, measure the direction, search the step and update the iterate and the
// outer variables.  Per instance and stage j the constraint rows are w_j = C_j x_j + D_j u_j with
// bounds [bl_j, bu_j]; the proximal Sigma-augmented Lagrangian (eq. ocp-al-funcs) at multipliers y
// and penalties Sigma has the generalised Hessian (eq. qpalm-ocp-hessians)
//   [[R, S], [S^T, Q]] + [D^T; C^T] Sigma^J [D C] + Gamma^{-1},   J: rows with w + y / Sigma outside
// [bl, bu], and the gradient [r; q] + H_cost [u; x] + [D^T; C^T] yhat + Gamma^{-1} (z - zbar), with
// yhat = y + Sigma (w - Pi(w + y / Sigma)).
#include <float.h>
#include <math.h>

#include <algorithm>

#include "lq_qp.hpp"

namespace lq {

constexpr int QT = 256;  // threads per workgroup
constexpr int QSG = 4;   // stages per workgroup in the stage-parallel kernels
constexpr int NP = 6;    // partial sums per (instance, stage): eta, beta, inner residual, |d|, scale, -

enum { FL_INNER = 0, FL_OUTER = 1, FL_FAIL = 2, FL_ITERS = 3, FL_EXACT = 4, FL_N = 8 };


__device__ __forceinline__ double projb(double v, double lo, double hi) { return fmin(fmax(v, lo), hi); }

__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < QT / 64; ++i) s += red[i];
  return s;
}

__device__ double block_max(double v, double* red) {
  const int tid = threadIdx.x;
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = red[0];
  for (int i = 1; i < QT / 64; ++i) s = fmax(s, red[i]);
  return s;
}

__device__ int block_sum_i(int v, int* redi) {
  const int tid = threadIdx.x;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((tid & 63) == 0) redi[tid >> 6] = v;
  __syncthreads();
  int s = 0;
  for (int i = 0; i < QT / 64; ++i) s += redi[i];
  return s;
}

// Exclusive prefix sum of v over the workgroup (thread order), and its total: a shuffle scan in
// each wavefront, then the wavefront totals through LDS.
__device__ int block_excl_scan(int v, int* redi, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) redi[w] = x;
  __syncthreads();
  int off = 0, tot = 0;
  for (int i = 0; i < QT / 64; ++i) {
    const int t = redi[i];
    off += i < w ? t : 0;
    tot += t;
  }
  *total = tot;
  return off + x - v;
}

constexpr int RPT = 4;  // staged rollout: elements per thread and stage (two LDS slots of RPT QT)

// Elements of one stage staged by rollout_staged: [A_k B_k] row-major (nx rows of nx + nu), u_k,
// and f_k when the problem has f.
__host__ __device__ inline int roll_elems(int nx, int nu, bool hf) { return nx * (nx + nu) + nu + (hf ? nx : 0); }

// rollout with every stage's [A_k B_k], u_k, f_k copied into LDS one stage ahead, in two slots:
// the loads of stage k + 1 are issued before stage k's products and stored into the other slot
// after them, so that a stage waits for what is left of one round trip at most, and the products
// read LDS only.  The same terms in the same order as the loop of rollout below.
__device__ void rollout_staged(const QPArgs& a, const Desc& D, double* xs, double* buf) {
  const int N = D.N, nx = D.nx, nu = D.nu, tid = threadIdx.x, w = nx + nu;
  const bool hf = a.d.f != nullptr;
  const int ne = roll_elems(nx, nu, hf), nab = nx * w;
  const double* A = a.d.A + D.oA;
  const double* B = a.d.B + D.oB;
  const double* U = a.u + D.ou;
  const double* F = hf ? a.d.f + D.of : A;  // (no f element is staged without f)
  // this thread's elements: array (0 A, 1 B, 2 u, 3 f) and offset within a stage; past the last
  // element the last one is loaded again and not stored
  int kind[RPT], off[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int e = min(tid + q * QT, ne - 1);
    if (e < nab) {
      const int r = e / w, c = e - r * w;
      kind[q] = c < nx ? 0 : 1;
      off[q] = c < nx ? r * nx + c : r * nu + (c - nx);
    } else if (e < nab + nu) {
      kind[q] = 2;
      off[q] = e - nab;
    } else {
      kind[q] = 3;
      off[q] = e - nab - nu;
    }
  }
  auto src = [&](int k, int q) -> const double* {
    const int64_t kk = min(k, N - 1);
    return kind[q] == 0 ? A + kk * nx * nx + off[q]
         : kind[q] == 1 ? B + kk * nx * nu + off[q]
         : kind[q] == 2 ? U + kk * nu + off[q]
                        : F + kk * nx + off[q];
  };
#pragma unroll
  for (int q = 0; q < RPT; ++q)
    if (tid + q * QT < ne) buf[tid + q * QT] = *src(0, q);
  const double* x0 = a.d.x0 + D.ox0;
  for (int i = tid; i < nx; i += QT) xs[i] = x0[i];
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    double v[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) v[q] = *src(k + 1, q);
    const double* M = buf + (k & 1) * ne;
    double s = 0.0;
    if (tid < nx) {
      s = hf ? M[nab + nu + tid] : 0.0;
      for (int c = 0; c < nx; ++c) s += M[tid * w + c] * xs[c];
      for (int c = 0; c < nu; ++c) s += M[tid * w + nx + c] * M[nab + c];
    }
    __syncthreads();
    if (tid < nx) {
      xs[tid] = s;
      a.x[D.ox + (int64_t)k * nx + tid] = s;
    }
    double* Mn = buf + ((k + 1) & 1) * ne;
#pragma unroll
    for (int q = 0; q < RPT; ++q)
      if (tid + q * QT < ne) Mn[tid + q * QT] = v[q];
    __syncthreads();
  }
}

// x_{k+1} = A_k x_k + B_k u_k + f_k from x_init, the whole workgroup on one instance (staged
// through LDS where the launch gave the slots and a stage fits them).
__device__ void rollout(const QPArgs& a, const Desc& D, double* xs) {
  if (a.orbuf > 0 && roll_elems(D.nx, D.nu, a.d.f != nullptr) <= RPT * QT) {
    rollout_staged(a, D, xs, xs + a.orbuf);
    return;
  }
  const int N = D.N, nx = D.nx, nu = D.nu, tid = threadIdx.x;
  const double* x0 = a.d.x0 + D.ox0;
  for (int i = tid; i < nx; i += QT) xs[i] = x0[i];
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    const double* Ak = a.d.A + D.oA + (int64_t)k * nx * nx;
    const double* Bk = a.d.B + D.oB + (int64_t)k * nx * nu;
    const double* uk = a.u + D.ou + (int64_t)k * nu;
    double v[1] = {0.0};
    const int i = tid;
    if (i < nx) {
      double s = a.d.f ? a.d.f[D.of + (int64_t)k * nx + i] : 0.0;
      for (int c = 0; c < nx; ++c) s += Ak[(int64_t)i * nx + c] * xs[c];
      for (int c = 0; c < nu; ++c) s += Bk[(int64_t)i * nu + c] * uk[c];
      v[0] = s;
    }
    __syncthreads();
    if (i < nx) {
      xs[i] = v[0];
      a.x[D.ox + (int64_t)k * nx + i] = v[0];
    }
    __syncthreads();
  }
}

// Start: u (0 unless warm), x simulated, y (0 unless warm), penalties, centre, flags, zero parts of
// the Newton systems.
__global__ __launch_bounds__(QT) void k_qp_init(QPArgs a) {
  extern __shared__ double sm[];
  const int b = blockIdx.x, tid = threadIdx.x;
  const Desc D = a.desc[b];
  const int N = D.N, nx = D.nx, nu = D.nu, m = a.m;
  const int64_t R = (int64_t)m * (N + 1), oR = (int64_t)m * D.oK;
  if (!a.warm) {
    for (int64_t e = tid; e < (int64_t)N * nu; e += QT) a.u[D.ou + e] = 0.0;
    for (int64_t e = tid; e < R; e += QT) a.y[oR + e] = 0.0;
  }
  for (int64_t e = tid; e < R; e += QT) {
    a.sig[oR + e] = a.sigma0;
    a.eprev[oR + e] = INFINITY;
  }
  for (int i = tid; i < nx; i += QT) a.x0n[D.ox0 + i] = 0.0;
  if (tid < FL_N) a.fl[(int64_t)b * FL_N + tid] = 0;
  if (tid == 0) a.tau[b] = 0.0;
  __syncthreads();
  rollout(a, D, sm);
  for (int64_t e = tid; e < (int64_t)N * nx; e += QT) a.xbar[D.ox + e] = a.x[D.ox + e];
  for (int64_t e = tid; e < (int64_t)N * nu; e += QT) a.ubar[D.ou + e] = a.u[D.ou + e];
}

// Stage products of the refinement kernel.  Rows: one wavefront per row (four rows at a time, so
// that their loads are in flight together), lanes over the columns, a wavefront reduction.
// Columns: lanes over the columns, the wavefronts over the rows, partial sums through LDS.  (The
// Newton and direction kernels keep one thread per output row: with several workgroups per CU
// their strided reads cost less than these reductions' shuffles and barriers, measured.)
constexpr int QW = QT / 64;  // wavefronts per workgroup

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// out(i, sum_q M[i][q] v1[q], sum_q M[i][q] v2[q]) for rows i < r of the row-major M (row length
// ld, c columns used; v1, v2 in LDS, v2 may be null), called on lane 0 of row i's wavefront (each
// row always on the same wavefront).
template <typename Out>
__device__ void rows_mv(const double* M, int r, int c, int ld, const double* v1, const double* v2, Out&& out) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i0 = 4 * w; i0 < r; i0 += 4 * QW) {
    double s1[4], s2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      s1[t] = s2[t] = 0.0;
      const int i = i0 + t;
      if (i < r)
        for (int q = lane; q < c; q += 64) {
          const double mv = M[(int64_t)i * ld + q];
          s1[t] = fma(mv, v1[q], s1[t]);
          if (v2) s2[t] = fma(mv, v2[q], s2[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double a1 = wave_sum(s1[t]), a2 = v2 ? wave_sum(s2[t]) : 0.0;
      if (lane == 0 && i0 + t < r) out(i0 + t, a1, a2);
    }
  }
}

// out(q, sum_i M[i][q] w1[i], sum_i M[i][q] w2[i]) for columns q < c (w1, w2 in LDS, w2 may be
// null), called on thread q after a barrier; part: LDS of 2 QW c doubles.  Ends with a barrier.
template <typename Out>
__device__ void cols_mv(const double* M, int r, int c, int ld, const double* w1, const double* w2, double* part,
                        Out&& out) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int q0 = 0; q0 < c; q0 += 64) {
    const int q = q0 + lane;
    if (q < c) {
      double s1 = 0.0, s2 = 0.0;
      for (int i = w; i < r; i += QW) {
        const double mv = M[(int64_t)i * ld + q];
        s1 = fma(mv, w1[i], s1);
        if (w2) s2 = fma(mv, w2[i], s2);
      }
      part[w * c + q] = s1;
      part[(QW + w) * c + q] = s2;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < c; q += QT) {
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < QW; ++k) {
      s1 += part[k * c + q];
      s2 += part[(QW + k) * c + q];
    }
    out(q, s1, s2);
  }
  __syncthreads();
}

// Newton system at the iterate, stage by stage (grid: stage groups x instances).
// Stage-parallel kernels: with STG the stage's matrices are first copied into LDS (one coalesced
// pass, every load in flight at once), so that the per-row loops below read LDS instead of
// waiting on one global load after another; the arithmetic, and its order, is the same either way.
// Copy n doubles from global memory into LDS with the whole workgroup.
__device__ __forceinline__ void stage_copy(double* dst, const double* __restrict__ src, int n) {
  for (int e = threadIdx.x; e < n; e += QT) dst[e] = src[e];
}

template <bool STG>
__global__ __launch_bounds__(QT) void k_qp_newton(QPArgs a) {
  extern __shared__ double sm[];
  __shared__ double red[QT / 64];
  const int b = blockIdx.y, tid = threadIdx.x;
  if (a.fl[(int64_t)b * FL_N + FL_OUTER]) return;
  const Desc D = a.desc[b];
  const int N = D.N, nx = D.nx, nu = D.nu, m = a.m;
  double* xs = sm;
  double* us = xs + nx;
  double* yh = us + nu;
  double* ss = yh + m;
  __shared__ int s_act[256];  // active rows of the stage (the only ones with Sigma^J and yhat nonzero)
  __shared__ int redi[QT / 64];
  for (int j = blockIdx.x * QSG; j < blockIdx.x * QSG + QSG && j <= N; ++j) {
    const double* xj = j == 0 ? a.d.x0 + D.ox0 : a.x + D.ox + (int64_t)(j - 1) * nx;
    for (int i = tid; i < nx; i += QT) xs[i] = xj[i];
    for (int c = tid; c < nu; c += QT) us[c] = j < N ? a.u[D.ou + (int64_t)j * nu + c] : 0.0;
    // stage matrices (Dj, Rj, Sj null where the stage has none; the staged copies are read only
    // where the global ones are not null)
    const double* Cj = a.C + (int64_t)m * D.oq + (int64_t)j * m * nx;
    const double* Dj = j < N ? a.D + (int64_t)m * D.or_ + (int64_t)j * m * nu : nullptr;
    const double* Qj = a.d.Q + D.oQ + (int64_t)j * nx * nx;
    const double* Rj = j < N ? a.d.R + D.oR + (int64_t)j * nu * nu : nullptr;
    const double* Sj = j < N && a.d.S ? a.d.S + D.oS + (int64_t)j * nu * nx : nullptr;
    const double *Cs = Cj, *Ds = Dj, *Qs = Qj, *Rs = Rj, *Ss = Sj;
    if constexpr (STG) {
      double* p = sm + a.omats;
      stage_copy(p, Cj, m * nx);
      Cs = p;
      p += m * nx;
      if (Dj) stage_copy(p, Dj, m * nu);
      Ds = p;
      p += m * nu;
      stage_copy(p, Qj, nx * nx);
      Qs = p;
      p += nx * nx;
      if (Rj) stage_copy(p, Rj, nu * nu);
      Rs = p;
      p += nu * nu;
      if (Sj) stage_copy(p, Sj, nu * nx);
      Ss = p;
    }
    __syncthreads();
    const int64_t rj = (int64_t)m * D.oK + (int64_t)j * m;
    double sc = 0.0;
    for (int i = tid; i < m; i += QT) {
      double wi = 0.0;
      for (int c = 0; c < nx; ++c) wi += Cs[(int64_t)i * nx + c] * xs[c];
      if (Dj)
        for (int c = 0; c < nu; ++c) wi += Ds[(int64_t)i * nu + c] * us[c];
      const double s = a.sig[rj + i], yi = a.y[rj + i];
      const double v = wi + yi / s;
      const double lo = a.bl[rj + i], hi = a.bu[rj + i];
      const bool act = v < lo || v > hi;
      const double h = yi + s * (wi - projb(v, lo, hi));
      yh[i] = h;
      ss[i] = act ? s : 0.0;
      a.w[rj + i] = wi;
      sc = fmax(sc, fabs(h));
    }
    for (int i = tid; i < nx; i += QT) sc = fmax(sc, fabs(xs[i]));
    for (int c = tid; c < nu; c += QT) sc = fmax(sc, fabs(us[c]));
    __syncthreads();
    sc = block_max(sc, red);
    if (tid == 0) a.part[(D.oK + j) * NP + 4] = sc;
    // active rows in increasing order (m <= QT: one row per thread), compacted by a prefix sum
    int na;
    {
      const bool on = tid < m && ss[tid] != 0.0;
      const int pos = block_excl_scan(on ? 1 : 0, redi, &na);
      if (on) s_act[pos] = tid;
    }
    __syncthreads();
    // Hessian blocks
    double* Qnj = a.Qn + D.oQ + (int64_t)j * nx * nx;
    for (int e = tid; e < nx * nx; e += QT) {
      const int p = e / nx, q = e % nx;
      double h = 0.5 * (Qs[p * nx + q] + Qs[q * nx + p]) + (p == q ? a.ginv : 0.0);
      for (int t = 0; t < na; ++t) {
        const int i = s_act[t];
        h += ss[i] * Cs[(int64_t)i * nx + p] * Cs[(int64_t)i * nx + q];
      }
      Qnj[e] = h;
    }
    if (j < N) {
      double* Rnj = a.Rn + D.oR + (int64_t)j * nu * nu;
      for (int e = tid; e < nu * nu; e += QT) {
        const int p = e / nu, q = e % nu;
        double h = 0.5 * (Rs[p * nu + q] + Rs[q * nu + p]) + (p == q ? a.ginv : 0.0);
        for (int t = 0; t < na; ++t) {
          const int i = s_act[t];
          h += ss[i] * Ds[(int64_t)i * nu + p] * Ds[(int64_t)i * nu + q];
        }
        Rnj[e] = h;
      }
      double* Snj = a.Sn + D.oS + (int64_t)j * nu * nx;
      for (int e = tid; e < nu * nx; e += QT) {
        const int p = e / nx, q = e % nx;
        double h = Sj ? Ss[e] : 0.0;
        for (int t = 0; t < na; ++t) {
          const int i = s_act[t];
          h += ss[i] * Ds[(int64_t)i * nu + p] * Cs[(int64_t)i * nx + q];
        }
        Snj[e] = h;
      }
      // r_j = R_sym u + S x + r + D^T yhat + (u - ubar) / gamma
      const double* ubj = a.ubar + D.ou + (int64_t)j * nu;
      for (int c = tid; c < nu; c += QT) {
        double g = a.d.r[D.or_ + (int64_t)j * nu + c] + a.ginv * (us[c] - ubj[c]);
        for (int q = 0; q < nu; ++q) g += 0.5 * (Rs[c * nu + q] + Rs[q * nu + c]) * us[q];
        if (Sj)
          for (int q = 0; q < nx; ++q) g += Ss[(int64_t)c * nx + q] * xs[q];
        for (int t = 0; t < na; ++t) g += Ds[(int64_t)s_act[t] * nu + c] * yh[s_act[t]];
        a.rn[D.or_ + (int64_t)j * nu + c] = g;
      }
    }
    // q_j = Q_sym x + q + C^T yhat + S^T u + (x - xbar) / gamma   (stage 0's is not used)
    const double* xbj = j >= 1 ? a.xbar + D.ox + (int64_t)(j - 1) * nx : nullptr;
    for (int p = tid; p < nx; p += QT) {
      double g = a.d.q[D.oq + (int64_t)j * nx + p] + (xbj ? a.ginv * (xs[p] - xbj[p]) : 0.0);
      for (int q = 0; q < nx; ++q) g += 0.5 * (Qs[p * nx + q] + Qs[q * nx + p]) * xs[q];
      if (Sj)
        for (int c = 0; c < nu; ++c) g += Ss[(int64_t)c * nx + p] * us[c];
      for (int t = 0; t < na; ++t) g += Cs[(int64_t)s_act[t] * nx + p] * yh[s_act[t]];
      a.qn[D.oq + (int64_t)j * nx + p] = g;
    }
    __syncthreads();
  }
}

// A factorisation that failed ends the instance.
__global__ void k_qp_check_info(QPArgs a, const int32_t* info) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.batch) return;
  int32_t* f = a.fl + (int64_t)b * FL_N;
  if (!f[FL_OUTER] && info[b] != 0) {
    f[FL_FAIL] = 1;
    f[FL_OUTER] = 1;
  }
}

// Direction measures, stage by stage: G d per row, the stage parts of eta and beta (eq. psi-prime:
// the cost's quadratic form and gradient along d, with the proximal term), the inner stationarity
// residual grad + M^T lam with the Newton multipliers, and |d|.
template <bool STG>
__global__ __launch_bounds__(QT) void k_qp_dir(QPArgs a) {
  extern __shared__ double sm[];
  __shared__ double red[QT / 64];
  const int b = blockIdx.y, tid = threadIdx.x;
  if (a.fl[(int64_t)b * FL_N + FL_OUTER] || a.fl[(int64_t)b * FL_N + FL_INNER]) return;
  const Desc D = a.desc[b];
  const int N = D.N, nx = D.nx, nu = D.nu, m = a.m;
  double* xs = sm;
  double* us = xs + nx;
  double* dxs = us + nu;
  double* dus = dxs + nx;
  for (int j = blockIdx.x * QSG; j < blockIdx.x * QSG + QSG && j <= N; ++j) {
    const double* xj = j == 0 ? a.d.x0 + D.ox0 : a.x + D.ox + (int64_t)(j - 1) * nx;
    for (int i = tid; i < nx; i += QT) {
      xs[i] = xj[i];
      dxs[i] = j == 0 ? 0.0 : a.dx[D.ox + (int64_t)(j - 1) * nx + i];
    }
    for (int c = tid; c < nu; c += QT) {
      us[c] = j < N ? a.u[D.ou + (int64_t)j * nu + c] : 0.0;
      dus[c] = j < N ? a.du[D.ou + (int64_t)j * nu + c] : 0.0;
    }
    // stage matrices (null where the stage has none; the staged copies are read only where the
    // global ones are not null)
    const double* Cj = a.C + (int64_t)m * D.oq + (int64_t)j * m * nx;
    const double* Dj = j < N ? a.D + (int64_t)m * D.or_ + (int64_t)j * m * nu : nullptr;
    const double* Qj = a.d.Q + D.oQ + (int64_t)j * nx * nx;
    const double* Sj = j < N && a.d.S ? a.d.S + D.oS + (int64_t)j * nu * nx : nullptr;
    const double* Rj = j < N ? a.d.R + D.oR + (int64_t)j * nu * nu : nullptr;
    const double* Aj = j < N ? a.d.A + D.oA + (int64_t)j * nx * nx : nullptr;
    const double* Bj = j < N ? a.d.B + D.oB + (int64_t)j * nx * nu : nullptr;
    const double *Cs = Cj, *Ds = Dj, *Qs = Qj, *Ss = Sj, *Rs = Rj, *As = Aj, *Bs = Bj;
    if constexpr (STG) {
      double* p = sm + a.omats;
      stage_copy(p, Cj, m * nx);
      Cs = p;
      p += m * nx;
      if (Dj) stage_copy(p, Dj, m * nu);
      Ds = p;
      p += m * nu;
      if (j >= 1) stage_copy(p, Qj, nx * nx);
      Qs = p;
      p += nx * nx;
      if (Sj) stage_copy(p, Sj, nu * nx);
      Ss = p;
      p += nu * nx;
      if (Rj) stage_copy(p, Rj, nu * nu);
      Rs = p;
      p += nu * nu;
      if (Aj && j >= 1) stage_copy(p, Aj, nx * nx);
      As = p;
      p += nx * nx;
      if (Bj) stage_copy(p, Bj, nx * nu);
      Bs = p;
    }
    __syncthreads();
    const int64_t rj = (int64_t)m * D.oK + (int64_t)j * m;
    double dm = 0.0;
    for (int i = tid; i < m; i += QT) {
      double g = 0.0;
      for (int c = 0; c < nx; ++c) g += Cs[(int64_t)i * nx + c] * dxs[c];
      if (Dj)
        for (int c = 0; c < nu; ++c) g += Ds[(int64_t)i * nu + c] * dus[c];
      a.gd[rj + i] = g;
    }
    const double* xbj = j >= 1 ? a.xbar + D.ox + (int64_t)(j - 1) * nx : nullptr;
    double eta = 0.0, beta = 0.0, rin = 0.0;
    if (j >= 1)
      for (int p = tid; p < nx; p += QT) {
        double hx = 0.0, gx = a.d.q[D.oq + (int64_t)j * nx + p];
        for (int q = 0; q < nx; ++q) {
          const double qs = 0.5 * (Qs[p * nx + q] + Qs[q * nx + p]);
          hx += qs * dxs[q];
          gx += qs * xs[q];
        }
        if (Sj)
          for (int c = 0; c < nu; ++c) {
            hx += Ss[(int64_t)c * nx + p] * dus[c];  // with the u part below: 2 du^T S dx in all
            gx += Ss[(int64_t)c * nx + p] * us[c];
          }
        eta += dxs[p] * hx + a.ginv * dxs[p] * dxs[p];
        beta += dxs[p] * (gx + a.ginv * (xs[p] - xbj[p]));
        dm = fmax(dm, fabs(dxs[p]));
        // inner residual of the x_j row: q_j + A_j^T lam_j - lam_{j-1}
        double r = a.qn[D.oq + (int64_t)j * nx + p] - a.dlam[D.olam + (int64_t)(j - 1) * nx + p];
        if (j < N)
          for (int q = 0; q < nx; ++q) r += As[(int64_t)q * nx + p] * a.dlam[D.olam + (int64_t)j * nx + q];
        rin = fmax(rin, fabs(r));
      }
    if (j < N) {
      const double* ubj = a.ubar + D.ou + (int64_t)j * nu;
      for (int c = tid; c < nu; c += QT) {
        double hu = 0.0, gu = a.d.r[D.or_ + (int64_t)j * nu + c];
        for (int q = 0; q < nu; ++q) {
          const double rs = 0.5 * (Rs[c * nu + q] + Rs[q * nu + c]);
          hu += rs * dus[q];
          gu += rs * us[q];
        }
        if (Sj)
          for (int q = 0; q < nx; ++q) {
            hu += Ss[(int64_t)c * nx + q] * dxs[q];
            gu += Ss[(int64_t)c * nx + q] * xs[q];
          }
        eta += dus[c] * hu + a.ginv * dus[c] * dus[c];
        beta += dus[c] * (gu + a.ginv * (us[c] - ubj[c]));
        dm = fmax(dm, fabs(dus[c]));
        double r = a.rn[D.or_ + (int64_t)j * nu + c];
        for (int q = 0; q < nx; ++q) r += Bs[(int64_t)q * nu + c] * a.dlam[D.olam + (int64_t)j * nx + q];
        rin = fmax(rin, fabs(r));
      }
    }
    eta = block_sum(eta, red);
    beta = block_sum(beta, red);
    rin = block_max(rin, red);
    dm = block_max(dm, red);
    if (tid == 0) {
      double* pj = a.part + (D.oK + j) * NP;
      pj[0] = eta;
      pj[1] = beta;
      pj[2] = rin;
      pj[3] = dm;
    }
    __syncthreads();
  }
}

// Refinement of a parallel-in-time Newton solve (whose Schur-complement solves lose accuracy at large
// penalties), stage by stage: the Newton system's KKT rows (eq. opt-cond-ocp-eq with the Newton
// Hessians, gradients qn, rn, f = 0, x_init = 0) at (dx, du, dlam), negated, as the right-hand side
// of the correction system: r' = rn + Rn du + Sn dx + B^T lam_j, q' = qn + Sn^T du + Qn dx + A^T lam_j
// - lam_{j-1}, f' = A dx + B du - dx_{j+1}.  Its solution added to (dx, du, dlam) cancels the residual.
__global__ __launch_bounds__(QT) void k_qp_newton_resid(QPArgs a) {
  extern __shared__ double sm[];
  const int b = blockIdx.y, tid = threadIdx.x;
  if (a.fl[(int64_t)b * FL_N + FL_OUTER]) return;
  const Desc D = a.desc[b];
  const int N = D.N, nx = D.nx, nu = D.nu;
  double* dxs = sm;        // dx_j    [nx]
  double* dus = dxs + nx;  // du_j    [nu]
  double* ls = dus + nu;   // lam_j   [nx]
  double* vx = ls + nx;    // q'_j    [nx]
  double* vu = vx + nx;    // r'_j    [nu]
  double* vf = vu + nu;    // f'_j    [nx]
  double* part = vf + nx;  // column partials [2 QW max(nx, nu)]
  for (int j = blockIdx.x * QSG; j < blockIdx.x * QSG + QSG && j <= N; ++j) {
    for (int i = tid; i < nx; i += QT) {
      dxs[i] = j == 0 ? 0.0 : a.dx[D.ox + (int64_t)(j - 1) * nx + i];
      ls[i] = j < N ? a.dlam[D.olam + (int64_t)j * nx + i] : 0.0;
      vx[i] = j >= 1 ? a.qn[D.oq + (int64_t)j * nx + i] - a.dlam[D.olam + (int64_t)(j - 1) * nx + i] : 0.0;
      vf[i] = j < N ? -a.dx[D.ox + (int64_t)j * nx + i] : 0.0;
    }
    for (int c = tid; c < nu; c += QT) {
      dus[c] = j < N ? a.du[D.ou + (int64_t)j * nu + c] : 0.0;
      vu[c] = j < N ? a.rn[D.or_ + (int64_t)j * nu + c] : 0.0;
    }
    __syncthreads();
    const double* Qn = a.Qn + D.oQ + (int64_t)j * nx * nx;
    const double* Rn = j < N ? a.Rn + D.oR + (int64_t)j * nu * nu : nullptr;
    const double* Sn = j < N ? a.Sn + D.oS + (int64_t)j * nu * nx : nullptr;
    const double* Aj = j < N ? a.d.A + D.oA + (int64_t)j * nx * nx : nullptr;
    const double* Bj = j < N ? a.d.B + D.oB + (int64_t)j * nx * nu : nullptr;
    if (j >= 1) rows_mv(Qn, nx, nx, nx, dxs, nullptr, [&](int p, double v, double) { vx[p] += v; });
    if (j < N) {
      rows_mv(Rn, nu, nu, nu, dus, nullptr, [&](int c, double v, double) { vu[c] += v; });
      rows_mv(Sn, nu, nx, nx, dxs, nullptr, [&](int c, double v, double) { vu[c] += v; });
      rows_mv(Aj, nx, nx, nx, dxs, nullptr, [&](int p, double v, double) { vf[p] += v; });
      rows_mv(Bj, nx, nu, nu, dus, nullptr, [&](int p, double v, double) { vf[p] += v; });
    }
    __syncthreads();
    if (j < N) {
      cols_mv(Bj, nx, nu, nu, ls, nullptr, part, [&](int c, double v, double) { vu[c] += v; });
      if (j >= 1) {
        cols_mv(Aj, nx, nx, nx, ls, nullptr, part, [&](int p, double v, double) { vx[p] += v; });
        cols_mv(Sn, nu, nx, nx, dus, nullptr, part, [&](int p, double v, double) { vx[p] += v; });
      }
    }
    for (int i = tid; i < nx; i += QT) {
      a.qc[D.oq + (int64_t)j * nx + i] = vx[i];
      if (j < N) a.fc[D.of + (int64_t)j * nx + i] = vf[i];
    }
    if (j < N)
      for (int c = tid; c < nu; c += QT) a.rc[D.or_ + (int64_t)j * nu + c] = vu[c];
    __syncthreads();
  }
}

__global__ void k_qp_add(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] += src[i];
}

// psi'(t) = eta t + beta + sum_i delta_i [delta_i t - alpha_i]_+ (eq. psi-prime) over the rows of
// one instance, each thread taking a contiguous chunk of rows (lower then upper bound of a row).
struct LineRows {
  const double *w, *gd, *y, *sig, *bl, *bu;
  int64_t R, chunk;
};

__device__ __forceinline__ void row_terms(const LineRows& L, int64_t r, double& d0, double& a0, double& d1,
                                          double& a1, bool& h0, bool& h1) {
  const double s = L.sig[r], rs = sqrt(s), g = L.gd[r], w = L.w[r], y = L.y[r];
  const double lo = L.bl[r], hi = L.bu[r];
  h0 = lo > -INFINITY;
  h1 = hi < INFINITY;
  d0 = -rs * g;
  a0 = h0 ? (y + s * (w - lo)) / rs : 0.0;
  d1 = rs * g;
  a1 = h1 ? -(y + s * (w - hi)) / rs : 0.0;
}

__device__ double slope_at(const LineRows& L, double eta, double beta, double t, double* red) {
  const int tid = threadIdx.x;
  double acc = 0.0;
  const int64_t r0 = tid * L.chunk, r1 = min(L.R, r0 + L.chunk);
  for (int64_t r = r0; r < r1; ++r) {
    double d0, a0, d1, a1;
    bool h0, h1;
    row_terms(L, r, d0, a0, d1, a1, h0, h1);
    if (h0) acc += d0 * fmax(d0 * t - a0, 0.0);
    if (h1) acc += d1 * fmax(d1 * t - a1, 0.0);
  }
  return eta * t + beta + block_sum(acc, red);
}

// Breakpoints t_i = alpha_i / delta_i strictly inside (lo, hi) owned by this thread (count, or the
// k-th of them in index order).
__device__ int local_breaks(const LineRows& L, double lo, double hi, int k, double* kth) {
  const int tid = threadIdx.x;
  int c = 0;
  const int64_t r0 = tid * L.chunk, r1 = min(L.R, r0 + L.chunk);
  for (int64_t r = r0; r < r1; ++r) {
    double d0, a0, d1, a1;
    bool h0, h1;
    row_terms(L, r, d0, a0, d1, a1, h0, h1);
    if (h0 && d0 != 0.0) {
      const double t = a0 / d0;
      if (t > lo && t < hi) {
        if (c == k) *kth = t;
        ++c;
      }
    }
    if (h1 && d1 != 0.0) {
      const double t = a1 / d1;
      if (t > lo && t < hi) {
        if (c == k) *kth = t;
        ++c;
      }
    }
  }
  return c;
}

// The row terms of one thread's chunk (at most RC rows), computed once per line search and kept
// in registers: slope and breakpoint passes then read no global memory.  Same terms, same order as
// slope_at / local_breaks (which the search uses for longer chunks).
constexpr int RC = 12;
struct RowCache {
  double d0[RC], a0[RC], d1[RC], a1[RC];
  bool h0[RC], h1[RC];
  int n;  // rows of this thread
};

__device__ __forceinline__ void row_cache_fill(const LineRows& L, RowCache& C) {
  const int64_t r0 = threadIdx.x * L.chunk, r1 = min(L.R, r0 + L.chunk);
  C.n = (int)max((int64_t)0, r1 - r0);
  // every slot is filled (rows past the chunk repeat a row of the instance and are never read),
  // so that the slots stay in registers
#pragma unroll
  for (int q = 0; q < RC; ++q) {
    const int64_t r = min(r0 + min(q, max(C.n - 1, 0)), L.R - 1);
    row_terms(L, r, C.d0[q], C.a0[q], C.d1[q], C.a1[q], C.h0[q], C.h1[q]);
  }
}

__device__ __forceinline__ double slope_cached(const RowCache& C, double eta, double beta, double t, double* red) {
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < RC; ++q) {
    if (q < C.n && C.h0[q]) acc += C.d0[q] * fmax(C.d0[q] * t - C.a0[q], 0.0);
    if (q < C.n && C.h1[q]) acc += C.d1[q] * fmax(C.d1[q] * t - C.a1[q], 0.0);
  }
  return eta * t + beta + block_sum(acc, red);
}

__device__ __forceinline__ int breaks_cached(const RowCache& C, double lo, double hi, int k, double* kth) {
  int c = 0;
#pragma unroll
  for (int q = 0; q < RC; ++q) {
    if (q < C.n && C.h0[q] && C.d0[q] != 0.0) {
      const double t = C.a0[q] / C.d0[q];
      if (t > lo && t < hi) {
        if (c == k) *kth = t;
        ++c;
      }
    }
    if (q < C.n && C.h1[q] && C.d1[q] != 0.0) {
      const double t = C.a1[q] / C.d1[q];
      if (t > lo && t < hi) {
        if (c == k) *kth = t;
        ++c;
      }
    }
  }
  return c;
}

// Exact line search, one workgroup per instance: the inner-loop test first (stationarity residual,
// a direction at rounding level), then the bisection over the breakpoints of psi' (a breakpoint in
// the current bracket chosen as pivot: the median in index order; psi' at it decides the side), the
// root on the last linear piece, and whether a full step crosses no breakpoint (the model is exact
// there: the inner minimiser).
__global__ __launch_bounds__(QT) void k_qp_search(QPArgs a) {
  __shared__ double red[QT / 64];
  __shared__ int redi[QT / 64];
  __shared__ double s_piv;
  const int b = blockIdx.x, tid = threadIdx.x;
  int32_t* f = a.fl + (int64_t)b * FL_N;
  if (f[FL_OUTER] || f[FL_INNER]) {
    if (tid == 0) a.tau[b] = 0.0;
    return;
  }
  const Desc D = a.desc[b];
  const int N = D.N;
  double eta = 0.0, beta = 0.0, rin = 0.0, dm = 0.0, sc = 1.0;
  for (int j = tid; j <= N; j += QT) {
    const double* pj = a.part + (D.oK + j) * NP;
    eta += pj[0];
    beta += pj[1];
    rin = fmax(rin, pj[2]);
    dm = fmax(dm, pj[3]);
    sc = fmax(sc, pj[4]);
  }
  eta = block_sum(eta, red);
  beta = block_sum(beta, red);
  rin = block_max(rin, red);
  dm = block_max(dm, red);
  sc = block_max(sc, red);
  if (rin <= a.inner_tol * sc || dm <= 1e-15 * sc) {
    if (tid == 0) {
      a.tau[b] = 0.0;
      f[FL_INNER] = 1;
    }
    return;
  }
  LineRows L;
  const int64_t o = (int64_t)a.m * D.oK;
  L.w = a.w + o; L.gd = a.gd + o; L.y = a.y + o; L.sig = a.sig + o; L.bl = a.bl + o; L.bu = a.bu + o;
  L.R = (int64_t)a.m * (N + 1);
  L.chunk = (L.R + QT - 1) / QT;
  const bool cached = L.chunk <= RC;  // (uniform)
  RowCache C;
  C.n = 0;
  if (cached) row_cache_fill(L, C);
  auto slope = [&](double t) { return cached ? slope_cached(C, eta, beta, t, red) : slope_at(L, eta, beta, t, red); };
  auto breaks = [&](double lo_, double hi_, int k, double* kth) {
    return cached ? breaks_cached(C, lo_, hi_, k, kth) : local_breaks(L, lo_, hi_, k, kth);
  };
  double tau;
  const double s0 = slope(0.0);
  if (!(s0 < 0.0)) {
    tau = 1.0;  // the decrease is below the rounding of psi': take the full Newton step
  } else {
    double lo = 0.0, hi = INFINITY;
    bool done = false;
    tau = 0.0;
    for (int it = 0; it < 200 && !done; ++it) {
      double dummy = 0.0;
      const int c = breaks(lo, hi, -1, &dummy);
      int total;
      const int pre = block_excl_scan(c, redi, &total);
      if (total == 0) break;
      const int rank = total / 2;
      if (rank >= pre && rank < pre + c) {
        double t = 0.0;
        breaks(lo, hi, rank - pre, &t);
        s_piv = t;
      }
      __syncthreads();
      const double tp = s_piv;
      const double sp = slope(tp);
      if (sp == 0.0) {
        tau = tp;
        done = true;
      } else if (sp < 0.0) {
        lo = tp;
      } else {
        hi = tp;
      }
    }
    if (!done) {
      // psi' is linear on (lo, hi): its root from two interior points
      const double t0 = hi < INFINITY ? lo + 0.25 * (hi - lo) : lo + 1.0;
      const double t1 = hi < INFINITY ? lo + 0.75 * (hi - lo) : lo + 2.0;
      const double f0 = slope(t0), f1 = slope(t1);
      tau = t0 - f0 * (t1 - t0) / (f1 - f0);
      tau = fmin(fmax(tau, lo), hi);
    }
  }
  // full step with no breakpoint crossed: the model is exact, the step ends the inner loop
  int exact = 0;
  if (fabs(tau - 1.0) <= 1e-8) {
    double dummy = 0.0;
    const int c = breaks(0.0, tau, -1, &dummy);
    exact = block_sum_i(c, redi) == 0;
  }
  if (tid == 0) {
    a.tau[b] = tau;
    f[FL_ITERS] += 1;
    f[FL_EXACT] = exact;
  }
}

// u <- u + tau du (grid: stage groups x instances); an exact full step ends the inner loop.
__global__ __launch_bounds__(QT) void k_qp_step(QPArgs a) {
  const int b = blockIdx.y, tid = threadIdx.x;
  const double t = a.tau[b];
  int32_t* f = a.fl + (int64_t)b * FL_N;
  if (t == 0.0) return;
  const Desc D = a.desc[b];
  const int N = D.N, nu = D.nu;
  for (int j = blockIdx.x * QSG; j < blockIdx.x * QSG + QSG && j < N; ++j)
    for (int c = tid; c < nu; c += QT) a.u[D.ou + (int64_t)j * nu + c] += t * a.du[D.ou + (int64_t)j * nu + c];
  if (blockIdx.x == 0 && tid == 0 && f[FL_EXACT]) f[FL_INNER] = 1;
}

// x simulated from the new u (x + tau dx in exact arithmetic): the iterate keeps the dynamics
// exactly, which the line search assumes, whatever the accuracy of the Newton solve.
__global__ __launch_bounds__(QT) void k_qp_rollout(QPArgs a) {
  extern __shared__ double sm[];
  const int b = blockIdx.x;
  if (a.tau[b] == 0.0) return;
  const Desc D = a.desc[b];
  rollout(a, D, sm);
}

// Number of instances still iterating: inner (outer and inner not done) or outer.
__global__ void k_qp_count(QPArgs a, int which, int32_t* out) {
  __shared__ int redi[QT / 64];
  int c = 0;
  for (int b = threadIdx.x; b < a.batch; b += QT) {
    const int32_t* f = a.fl + (int64_t)b * FL_N;
    c += which == 0 ? (!f[FL_OUTER] && !f[FL_INNER]) : !f[FL_OUTER];
  }
  c = block_sum_i(c, redi);
  if (threadIdx.x == 0) *out = c;
}

// Outer step, rows and stages: yhat, the violation e = (yhat - y) / Sigma, y <- yhat; partial maxima
// of |e| and |z - zbar| / gamma.
__global__ __launch_bounds__(QT) void k_qp_outer(QPArgs a) {
  extern __shared__ double sm[];
  __shared__ double red[QT / 64];
  const int b = blockIdx.y, tid = threadIdx.x;
  if (a.fl[(int64_t)b * FL_N + FL_OUTER]) return;
  const Desc D = a.desc[b];
  const int N = D.N, nx = D.nx, nu = D.nu, m = a.m;
  double* xs = sm;
  double* us = xs + nx;
  for (int j = blockIdx.x * QSG; j < blockIdx.x * QSG + QSG && j <= N; ++j) {
    const double* xj = j == 0 ? a.d.x0 + D.ox0 : a.x + D.ox + (int64_t)(j - 1) * nx;
    for (int i = tid; i < nx; i += QT) xs[i] = xj[i];
    for (int c = tid; c < nu; c += QT) us[c] = j < N ? a.u[D.ou + (int64_t)j * nu + c] : 0.0;
    __syncthreads();
    const double* Cj = a.C + (int64_t)m * D.oq + (int64_t)j * m * nx;
    const double* Dj = j < N ? a.D + (int64_t)m * D.or_ + (int64_t)j * m * nu : nullptr;
    const int64_t rj = (int64_t)m * D.oK + (int64_t)j * m;
    double em = 0.0, dz = 0.0;
    for (int i = tid; i < m; i += QT) {
      double wi = 0.0;
      for (int c = 0; c < nx; ++c) wi += Cj[(int64_t)i * nx + c] * xs[c];
      if (Dj)
        for (int c = 0; c < nu; ++c) wi += Dj[(int64_t)i * nu + c] * us[c];
      const double s = a.sig[rj + i], yi = a.y[rj + i];
      const double h = yi + s * (wi - projb(wi + yi / s, a.bl[rj + i], a.bu[rj + i]));
      const double ei = (h - yi) / s;
      a.e[rj + i] = ei;
      a.y[rj + i] = h;
      em = fmax(em, fabs(ei));
    }
    if (j >= 1)
      for (int i = tid; i < nx; i += QT) dz = fmax(dz, fabs(xs[i] - a.xbar[D.ox + (int64_t)(j - 1) * nx + i]));
    if (j < N)
      for (int c = tid; c < nu; c += QT) dz = fmax(dz, fabs(us[c] - a.ubar[D.ou + (int64_t)j * nu + c]));
    em = block_max(em, red);
    dz = block_max(dz, red);
    if (tid == 0) {
      a.part[(D.oK + j) * NP + 0] = em;
      a.part[(D.oK + j) * NP + 1] = dz * a.ginv;
    }
    __syncthreads();
  }
}

// Outer decision per instance; a continuing instance gets its states simulated again from u and a
// new inner loop.
__global__ __launch_bounds__(QT) void k_qp_outer_fin(QPArgs a) {
  extern __shared__ double sm[];
  __shared__ double red[QT / 64];
  const int b = blockIdx.x, tid = threadIdx.x;
  int32_t* f = a.fl + (int64_t)b * FL_N;
  if (f[FL_OUTER]) return;
  const Desc D = a.desc[b];
  double em = 0.0, dz = 0.0;
  for (int j = tid; j <= D.N; j += QT) {
    em = fmax(em, a.part[(D.oK + j) * NP + 0]);
    dz = fmax(dz, a.part[(D.oK + j) * NP + 1]);
  }
  em = block_max(em, red);
  dz = block_max(dz, red);
  if (em <= a.eps && dz <= a.eps) {
    if (tid == 0) f[FL_OUTER] = 1;
    return;
  }
  rollout(a, D, sm);
  if (tid == 0) f[FL_INNER] = 0;
}

// Penalties of rows whose violation did not shrink enough, the previous violation, the new centre.
__global__ __launch_bounds__(QT) void k_qp_outer_upd(QPArgs a) {
  const int b = blockIdx.y, tid = threadIdx.x;
  if (a.fl[(int64_t)b * FL_N + FL_OUTER]) return;
  const Desc D = a.desc[b];
  const int N = D.N, nx = D.nx, nu = D.nu, m = a.m;
  for (int j = blockIdx.x * QSG; j < blockIdx.x * QSG + QSG && j <= N; ++j) {
    const int64_t rj = (int64_t)m * D.oK + (int64_t)j * m;
    for (int i = tid; i < m; i += QT) {
      const double ae = fabs(a.e[rj + i]);
      if (ae > a.theta * a.eprev[rj + i]) a.sig[rj + i] = fmin(a.sigma_max, a.sigma_up * a.sig[rj + i]);
      a.eprev[rj + i] = ae;
    }
    if (j >= 1)
      for (int i = tid; i < nx; i += QT)
        a.xbar[D.ox + (int64_t)(j - 1) * nx + i] = a.x[D.ox + (int64_t)(j - 1) * nx + i];
    if (j < N)
      for (int c = tid; c < nu; c += QT) a.ubar[D.ou + (int64_t)j * nu + c] = a.u[D.ou + (int64_t)j * nu + c];
  }
}

// Status and step counts; the multipliers of the dynamics from the last Newton solve.
__global__ void k_qp_final(QPArgs a, double* lam, int32_t* status, int32_t* iters) {
  const int b = blockIdx.x, tid = threadIdx.x;
  const Desc D = a.desc[b];
  const int32_t* f = a.fl + (int64_t)b * FL_N;
  for (int64_t e = tid; e < (int64_t)D.N * D.nx; e += blockDim.x) lam[D.olam + e] = a.dlam[D.olam + e];
  if (tid == 0) {
    status[b] = f[FL_FAIL] ? 2 : (f[FL_OUTER] ? 0 : 1);
    iters[b] = f[FL_ITERS];
  }
}

// ---------------------------------------------------------------------------------------------
// Host side.

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

QPLayout qp_layout(const int64_t* totals, int64_t sumK, int batch, int m) {
  // totals: elements of Q, R, S, q, r, f, x0, x, u, lam (plan layout)
  QPLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = al256(o + bytes);
    return r;
  };
  L.oQn = take(8 * totals[0]);
  L.oRn = take(8 * totals[1]);
  L.oSn = take(8 * totals[2]);
  L.oqn = take(8 * totals[3]);
  L.orn = take(8 * totals[4]);
  L.ox0n = take(8 * totals[6]);
  L.odx = take(8 * totals[7]);
  L.odu = take(8 * totals[8]);
  L.odlam = take(8 * totals[9]);
  L.oqc = take(8 * totals[3]);
  L.orc = take(8 * totals[4]);
  L.ofc = take(8 * totals[5]);
  L.ocdx = take(8 * totals[7]);
  L.ocdu = take(8 * totals[8]);
  L.ocdlam = take(8 * totals[9]);
  L.oxb = take(8 * totals[7]);
  L.oub = take(8 * totals[8]);
  const size_t rows = 8 * (size_t)m * sumK;
  L.osig = take(rows);
  L.ow = take(rows);
  L.ogd = take(rows);
  L.oe = take(rows);
  L.oep = take(rows);
  L.opart = take(8 * (size_t)NP * sumK);
  L.otau = take(8 * (size_t)batch);
  L.ofl = take(4 * (size_t)FL_N * batch);
  L.orel = take(8 * (size_t)batch);
  L.oinfo = take(4 * (size_t)batch);
  L.ocnt = take(4 * 2);
  L.total = o;
  return L;
}

QPArgs qp_args(const Desc* desc, int batch, int m, const lq_data& d, const lq_qp_constraints& c, const lq_qp_opts& op,
               void* ws, const QPLayout& L, double* x, double* u, double* y) {
  char* w = (char*)ws;
  QPArgs a = {};
  a.desc = desc;
  a.batch = batch;
  a.m = m;
  a.d = d;
  a.C = c.C; a.D = c.D; a.bl = c.bl; a.bu = c.bu;
  a.Qn = (double*)(w + L.oQn); a.Rn = (double*)(w + L.oRn); a.Sn = (double*)(w + L.oSn);
  a.qn = (double*)(w + L.oqn); a.rn = (double*)(w + L.orn); a.x0n = (double*)(w + L.ox0n);
  a.x = x; a.u = u; a.y = y;
  a.dx = (double*)(w + L.odx); a.du = (double*)(w + L.odu); a.dlam = (double*)(w + L.odlam);
  a.qc = (double*)(w + L.oqc); a.rc = (double*)(w + L.orc); a.fc = (double*)(w + L.ofc);
  a.cdx = (double*)(w + L.ocdx); a.cdu = (double*)(w + L.ocdu); a.cdlam = (double*)(w + L.ocdlam);
  a.xbar = (double*)(w + L.oxb); a.ubar = (double*)(w + L.oub);
  a.sig = (double*)(w + L.osig); a.w = (double*)(w + L.ow); a.gd = (double*)(w + L.ogd);
  a.e = (double*)(w + L.oe); a.eprev = (double*)(w + L.oep);
  a.part = (double*)(w + L.opart); a.tau = (double*)(w + L.otau); a.fl = (int32_t*)(w + L.ofl);
  a.sigma0 = op.sigma0; a.ginv = 1.0 / op.gamma; a.eps = op.eps; a.theta = op.theta; a.sigma_up = op.sigma_up;
  a.sigma_max = op.sigma_max; a.inner_tol = op.inner_tol; a.warm = op.warm;
  return a;
}

// LDS of the QP kernels: the largest is the direction kernel's (vectors and row / column sums)
// or the Newton kernel's (with the rows' state), plus the column partials of cols_mv.
size_t qp_stage_lds(int nxmax, int numax, int m) {
  const size_t cm = std::max(std::max(nxmax, numax), m);
  return sizeof(double) * (6 * (size_t)nxmax + 5 * numax + 3 * m + 2 * QW * cm + 8);
}

hipError_t qp_refine(int which, const QPArgs& a, int maxN, int nxmax, int numax, const int64_t* tot, hipStream_t st) {
  if (which == 0) {
    const size_t lds = qp_stage_lds(nxmax, numax, a.m);
    const dim3 sgrid((maxN + 1 + QSG - 1) / QSG, a.batch);
    hipError_t e = raise_lds_limit((const void*)k_qp_newton_resid, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_qp_newton_resid, sgrid, dim3(QT), lds, st, a);
    return hipGetLastError();
  }
  double* dst[3] = {a.dx, a.du, a.dlam};
  const double* src[3] = {a.cdx, a.cdu, a.cdlam};
  const int64_t n[3] = {tot[7], tot[8], tot[9]};
  for (int k = 0; k < 3; ++k) {
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n[k] + 255) / 256, 4096));
    hipLaunchKernelGGL(k_qp_add, dim3(g), dim3(256), 0, st, dst[k], src[k], n[k]);
  }
  return hipGetLastError();
}

// Doubles of one stage's matrices staged by k_qp_newton / k_qp_dir: C, D, Q, S, R, A, B.
static size_t qp_mats_doubles(int nxmax, int numax, int m) {
  const size_t x = nxmax, u = numax;
  return (size_t)m * (x + u) + 2 * x * x + 2 * x * u + u * u;
}

hipError_t qp_launch(int which, const QPArgs& a0, int maxN, int nxmax, int numax, hipStream_t st, const int32_t* info,
                     int32_t* out) {
  const size_t base = qp_stage_lds(nxmax, numax, a0.m);
  const dim3 sgrid((maxN + 1 + QSG - 1) / QSG, a0.batch);
  // the stage-parallel kernels stage the stage matrices in LDS when the workgroup's LDS stays
  // within 64 KiB (two or more workgroups per CU); larger shapes read them from global memory
  const size_t staged = base + sizeof(double) * qp_mats_doubles(nxmax, numax, a0.m);
  const bool stg = staged <= 65536;
  QPArgs a = a0;
  a.omats = (int64_t)(base / sizeof(double));
  const size_t lds = base;
  // rollouts (k_qp_init, k_qp_rollout, k_qp_outer_fin): two LDS slots of RPT QT doubles after the
  // base region, where that stays within 64 KiB
  const size_t rslots = 2 * sizeof(double) * (size_t)RPT * QT;
  const bool rst = base + rslots <= 65536;
  a.orbuf = rst ? (int64_t)(base / sizeof(double)) : 0;
  const size_t lds_r = rst ? base + rslots : base;
  const void* kn = stg ? (const void*)k_qp_newton<true> : (const void*)k_qp_newton<false>;
  const void* kd = stg ? (const void*)k_qp_dir<true> : (const void*)k_qp_dir<false>;
  hipError_t e;
  switch (which) {
    case 0:
      if ((e = raise_lds_limit((const void*)k_qp_init, lds_r)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_qp_init, dim3(a.batch), dim3(QT), lds_r, st, a);
      break;
    case 1:
      if ((e = raise_lds_limit(kn, stg ? staged : lds)) != hipSuccess) return e;
      {
        void* args[] = {(void*)&a};
        if ((e = hipLaunchKernel(kn, sgrid, dim3(QT), args, stg ? staged : lds, st)) != hipSuccess) return e;
      }
      break;
    case 2:
      hipLaunchKernelGGL(k_qp_check_info, dim3((a.batch + 255) / 256), dim3(256), 0, st, a, info);
      if ((e = raise_lds_limit(kd, stg ? staged : lds)) != hipSuccess) return e;
      {
        void* args[] = {(void*)&a};
        if ((e = hipLaunchKernel(kd, sgrid, dim3(QT), args, stg ? staged : lds, st)) != hipSuccess) return e;
      }
      hipLaunchKernelGGL(k_qp_search, dim3(a.batch), dim3(QT), 0, st, a);
      hipLaunchKernelGGL(k_qp_step, sgrid, dim3(QT), 0, st, a);
      if ((e = raise_lds_limit((const void*)k_qp_rollout, lds_r)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_qp_rollout, dim3(a.batch), dim3(QT), lds_r, st, a);
      hipLaunchKernelGGL(k_qp_count, dim3(1), dim3(QT), 0, st, a, 0, out);
      break;
    case 3:
      if ((e = raise_lds_limit((const void*)k_qp_outer, lds)) != hipSuccess) return e;
      if ((e = raise_lds_limit((const void*)k_qp_outer_fin, lds_r)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_qp_outer, sgrid, dim3(QT), lds, st, a);
      hipLaunchKernelGGL(k_qp_outer_fin, dim3(a.batch), dim3(QT), lds_r, st, a);
      hipLaunchKernelGGL(k_qp_outer_upd, sgrid, dim3(QT), 0, st, a);
      hipLaunchKernelGGL(k_qp_count, dim3(1), dim3(QT), 0, st, a, 1, out);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t qp_finish(const QPArgs& a, double* lam, int32_t* status, int32_t* iters, hipStream_t st) {
  hipLaunchKernelGGL(k_qp_final, dim3(a.batch), dim3(QT), 0, st, a, lam, status, iters);
  return hipGetLastError();
}

}  // namespace lq
