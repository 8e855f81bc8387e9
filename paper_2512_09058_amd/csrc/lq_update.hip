// Factorisation updates of the stored float64 Riccati factors (paper, Sec. "Factorization updates",
// Alg. "fact-mod-riccati-update" with one interval) and the modification of the stage Hessians
// they stand for (eq. low-rank-update-Hj).
//
// A change dSigma_j of the penalty factors of the constraint rows (D_j u_j + C_j x_j) adds
// [D_j^T; C_j^T] dSigma_j [D_j C_j] to the stage Hessian.  With the columns of Upsilon scaled by
// sqrt|dSigma| and the signature S = sign(dSigma), the stored factors are updated stage by stage,
// backward in time (Upsilon of stage j in the order (u_j, x_j)):
//   stage N:   Phi_N = C_N^T columns;  L^Q_N <- hyh(L^Q_N, Phi_N)
//   stage j:   Upsilon_j = [B_j^T Phi_{j+1}, D_j^T; A_j^T Phi_{j+1}, C_j^T], S_j = diag(S_{j+1}, sign dSigma_j)
//              [L^R_j; L^S_j] and Upsilon_j <- hyperbolic Householder over the nu input pivots;
//              the state rows of the result are Phi_j;  L^Q_j <- hyh(L^Q_j, Phi_j)   (j >= 1)
// where hyh(L, Y) is the factor of L L^T + Y S Y^T obtained by one hyperbolic Householder
// reflector per pivot (J-orthogonal for J = diag(1, S)): for pivot i with a = L_ii and b = Y_i,:
//   r^2 = a^2 + b S b^T (must be > 0: the updated matrix is positive definite),
//   w = [a + r, b],  every row [l, y] <- [l, y] - (2 ([l, y] J w) / (w^T J w)) w^T,
// then the sign of the pivot column is flipped (so the new diagonal is +r).  The width of Upsilon
// grows by the nonzero rows of every stage; the kernel refuses instances whose total exceeds its
// LDS capacity (the paper's rule: refactor when the rank of the change is large).
//
// The right-hand-side sweep of the factorisation (rbar, p, the vectors lq_solve starts from) is
// recomputed in the same backward pass from the updated factors and the data's q, r, f, so the
// updated workspace solves the modified problem exactly as a fresh lq_factor would.  Without update
// rows the kernel only recomputes that sweep (a new right-hand side for the stored factors).
#include <float.h>
#include <math.h>

#include "lq_internal.hpp"
#include "lqupdate.h"

namespace lq {

// ---------------------------------------------------------------------------------------------
// Modification of the data: R_j += D_j^T dS_j D_j, S_j += D_j^T dS_j C_j, Q_j += C_j^T dS_j C_j.
// One workgroup per (instance, group of `spb` stages).
__global__ __launch_bounds__(256) void k_update_data(const Desc* __restrict__ desc, lq_update u, double* Q,
                                                     double* R, double* S, int spb) {
  const Desc D = desc[blockIdx.x];
  const int N = D.N, nx = D.nx, nu = D.nu, m = u.m;
  const int j0 = blockIdx.y * spb;
  for (int j = j0; j < j0 + spb && j <= N; ++j) {
    const double* Cj = u.C + (int64_t)m * D.oq + (int64_t)j * m * nx;
    const double* sj = u.dsig + (int64_t)m * D.oK + (int64_t)j * m;
    bool any = false;
    for (int i = 0; i < m; ++i) any |= sj[i] != 0.0;
    if (!any) continue;  // the stage keeps its matrices
    double* Qj = Q + D.oQ + (int64_t)j * nx * nx;
    for (int e = threadIdx.x; e < nx * nx; e += blockDim.x) {
      const int p = e / nx, q = e % nx;
      double s = 0.0;
      for (int i = 0; i < m; ++i)
        if (sj[i] != 0.0) s += sj[i] * Cj[i * nx + p] * Cj[i * nx + q];
      Qj[e] += s;
    }
    if (j == N) continue;
    const double* Dj = u.D + (int64_t)m * D.or_ + (int64_t)j * m * nu;
    double* Rj = R + D.oR + (int64_t)j * nu * nu;
    for (int e = threadIdx.x; e < nu * nu; e += blockDim.x) {
      const int p = e / nu, q = e % nu;
      double s = 0.0;
      for (int i = 0; i < m; ++i)
        if (sj[i] != 0.0) s += sj[i] * Dj[i * nu + p] * Dj[i * nu + q];
      Rj[e] += s;
    }
    double* Sj = S + D.oS + (int64_t)j * nu * nx;
    for (int e = threadIdx.x; e < nu * nx; e += blockDim.x) {
      const int p = e / nx, q = e % nx;
      double s = 0.0;
      for (int i = 0; i < m; ++i)
        if (sj[i] != 0.0) s += sj[i] * Dj[i * nu + p] * Cj[i * nx + q];
      Sj[e] += s;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Factor update: one workgroup of 256 threads per instance.
constexpr int UT = 256;
constexpr int UCH = 8;  // columns per thread in the Upsilon products

struct UpdArgs {
  const Desc* desc;
  lq_data d;
  double* F;     // factor region (float64 plan)
  double* V;     // right-hand-side sweep (rbar, p)
  lq_update u;
  double* Phi;   // update workspace: Phi_k of stages 1..N, [nx][wmax] each (instance at wmax * olam)
  double* Sg;    // signs of the columns of Phi_k, [wmax] per stage 0..N (instance at wmax * oK)
  int32_t* Wk;   // columns of Phi_k per stage 0..N (instance at oK)
  int32_t* st;   // per instance: -1 width above wmax, else max over failures of 2 (k + 1) + non-finite
  int32_t wmax, ldy, lrsmax, lqmax, fsmax, nuxmax, nxmax;
  int32_t* info;
};

template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

// Hyperbolic Householder update of the factor rows [0, nrows), pivots [0, npiv) (row r of L
// starts at row(r)) with the W columns of Y (row stride ldy, signature sg).  G lanes share a
// row (they split its columns and reduce by shuffles); UT / G rows are rewritten at once.  Rows
// below each pivot are rewritten; the pivot rows of Y are left stale (they are zero in exact
// terms).  The first failing pivot (r^2 not positive: kind 1, not finite: kind 2) is recorded in
// bad/kind and its r replaced by 1.
template <int G, class RowF>
__device__ void hyh_g(RowF row, int nrows, int npiv, double* Y, int ldy, int W, const double* sg, double* dg,
                      int& bad, int& kind) {
  constexpr int NG = UT / G;
  const int tid = threadIdx.x, g = tid / G, l = tid % G;
  for (int i = 0; i < npiv; ++i) {
    const double* yi = Y + (int64_t)i * ldy;
    const double a = row(i)[i];
    double part = 0.0;
    for (int c = l; c < W; c += G) {
      const double b = yi[c];
      part += sg[c] * b * b;
    }
    const double r2 = a * a + group_sum<G>(part);
    const bool ok = r2 > 0.0 && r2 <= DBL_MAX;
    const double rn = ok ? sqrt(r2) : 1.0;
    const double w1 = fabs(a) + rn;
    const double tinv = 1.0 / (rn * w1);  // 2 / (w^T J w)
    for (int r = i + 1 + g; r < nrows; r += NG) {
      double* lr = row(r);
      double* yr = Y + (int64_t)r * ldy;
      double gp = 0.0;
      for (int c = l; c < W; c += G) gp += yr[c] * sg[c] * yi[c];
      gp = group_sum<G>(gp);
      const double li = lr[i];
      const double coef = (li * w1 + gp) * tinv;
      for (int c = l; c < W; c += G) yr[c] -= coef * yi[c];
      if (l == 0) lr[i] = coef * w1 - li;
    }
    if (tid == 0) {
      dg[i] = rn;
      if (!ok && bad < 0) {
        bad = i;
        kind = r2 != r2 || r2 > DBL_MAX ? 2 : 1;
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < npiv; i += UT) row(i)[i] = dg[i];
  __syncthreads();
}

template <class RowF>
__device__ void hyh(RowF row, int nrows, int npiv, double* Y, int ldy, int W, const double* sg, double* dg,
                    int& bad, int& kind) {
  if (W <= 16) hyh_g<4>(row, nrows, npiv, Y, ldy, W, sg, dg, bad, kind);
  else hyh_g<16>(row, nrows, npiv, Y, ldy, W, sg, dg, bad, kind);
}

// Appends the nonzero rows of stage j as columns W0.. of Y (u rows from D_j, x rows from C_j,
// scaled by sqrt|dSigma|) and their signs to sg; returns the new width (uniform over the block).
__device__ int stage_columns(const UpdArgs& a, const Desc& D, int j, double* Y, double* sg, int W0, int* cmap,
                             int& cnt) {
  const int m = a.u.m, nx = D.nx, nu = D.nu, nux = nx + nu, tid = threadIdx.x;
  if (m == 0) return W0;
  const double* sj = a.u.dsig + (int64_t)m * D.oK + (int64_t)j * m;
  if (tid < m) cmap[tid] = sj[tid] != 0.0;
  __syncthreads();
  if (tid == 0) {
    int c = W0;
    for (int i = 0; i < m; ++i) cmap[i] = cmap[i] ? c++ : -1;
    cnt = c;
  }
  __syncthreads();
  const double* Cj = a.u.C + (int64_t)m * D.oq + (int64_t)j * m * nx;
  const double* Dj = j < D.N ? a.u.D + (int64_t)m * D.or_ + (int64_t)j * m * nu : nullptr;
  for (int e = tid; e < nux * m; e += UT) {
    const int r = e % nux, i = e / nux, c = cmap[i];
    if (c < 0) continue;
    const double s = sj[i];
    const double v = r < nu ? (Dj ? Dj[i * nu + r] : 0.0) : Cj[i * nx + (r - nu)];
    Y[(int64_t)r * a.ldy + c] = sqrt(fabs(s)) * v;
    if (r == 0) sg[c] = s > 0.0 ? 1.0 : -1.0;
  }
  const int W = cnt;
  __syncthreads();
  return W;
}

// Ynew[r][c] = sum_m M[m][r'] Phi[m][c] for c < W: the input rows from B_j (r < nu), the state
// rows from A_j (r' = r - nu); Phi = state rows of the current Upsilon.
__device__ void upsilon_products(const UpdArgs& a, const Desc& D, int j, const double* Phi, double* Ynew, int W) {
  const int nx = D.nx, nu = D.nu, nux = nx + nu, tid = threadIdx.x, ldy = a.ldy;
  const double* Aj = a.d.A + D.oA + (int64_t)j * nx * nx;
  const double* Bj = a.d.B + D.oB + (int64_t)j * nx * nu;
  const int nch = (W + UCH - 1) / UCH;
  for (int e = tid; e < nux * nch; e += UT) {
    const int r = e % nux, c0 = (e / nux) * UCH;
    const double* Mc = r < nu ? Bj + r : Aj + (r - nu);
    const int ldm = r < nu ? nu : nx;
    double acc[UCH];
#pragma unroll
    for (int t = 0; t < UCH; ++t) acc[t] = 0.0;
#pragma unroll 4
    for (int mm = 0; mm < nx; ++mm) {
      const double mv = Mc[(int64_t)mm * ldm];
      const double* ph = Phi + (int64_t)mm * ldy + c0;
#pragma unroll
      for (int t = 0; t < UCH; ++t) acc[t] += mv * ph[t];
    }
#pragma unroll
    for (int t = 0; t < UCH; ++t)
      if (c0 + t < W) Ynew[(int64_t)r * ldy + c0 + t] = acc[t];
  }
}

// Inputs of the next stage's Upsilon, loaded into registers while the current stage's pivots run:
// the operand columns of the products (thread t < P nux holds M[mm][r], M = [B_j A_j], for
// r = t / P and its share mm in [p S, p S + S), p = t % P, P a power of two so that the P partial
// sums of a row reduce by shuffles), entries of the stage's rows and its penalty changes.
constexpr int PMAX = 32;
struct StagePrefetch {
  double mc[PMAX];
  double rv[2];  // row entries e = tid, tid + UT of (r, i) = (e % nux, e / nux)
  double ds;     // dsig_j[tid] (tid < m)
};

__host__ __device__ inline int parts_of(int nux) {
  int P = 1;
  while (P < 64 && 2 * P * nux <= UT) P *= 2;
  return P;
}

__device__ void prefetch_stage(const UpdArgs& a, const Desc& D, int j, StagePrefetch& pf) {
  const int nx = D.nx, nu = D.nu, nux = nx + nu, m = a.u.m, tid = threadIdx.x;
  const int P = parts_of(nux), S = (nx + P - 1) / P, r = tid / P, p = tid % P;
  const double* Aj = a.d.A + D.oA + (int64_t)j * nx * nx;
  const double* Bj = a.d.B + D.oB + (int64_t)j * nx * nu;
#pragma unroll
  for (int q = 0; q < PMAX; ++q) {
    const int mm = p * S + q;
    pf.mc[q] = (r < nux && q < S && mm < nx) ? (r < nu ? Bj[mm * nu + r] : Aj[mm * nx + (r - nu)]) : 0.0;
  }
  const double* Cj = a.u.C + (int64_t)m * D.oq + (int64_t)j * m * nx;
  const double* Dj = j < D.N ? a.u.D + (int64_t)m * D.or_ + (int64_t)j * m * nu : nullptr;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = tid + q * UT, rr = e % nux, i = e / nux;
    pf.rv[q] = e < nux * m ? (rr < nu ? (Dj ? Dj[i * nu + rr] : 0.0) : Cj[i * nx + (rr - nu)]) : 0.0;
  }
  pf.ds = tid < m ? a.u.dsig[(int64_t)m * D.oK + (int64_t)j * m + tid] : 0.0;
}

// Ynew[r][c] = sum_mm M[mm][r] Phi[mm][c] for c < W from the prefetched columns.
__device__ void upsilon_products_pf(const Desc& D, const StagePrefetch& pf, const double* Phi, int ldy, double* Ynew,
                                    int W) {
  const int nx = D.nx, nux = nx + D.nu, tid = threadIdx.x;
  const int P = parts_of(nux), S = (nx + P - 1) / P, r = tid / P, p = tid % P;
  for (int c0 = 0; c0 < W; c0 += UCH) {
    double acc[UCH];
#pragma unroll
    for (int t = 0; t < UCH; ++t) acc[t] = 0.0;
    if (r < nux)
#pragma unroll
      for (int q = 0; q < PMAX; ++q) {
        const int mm = p * S + q;
        if (q < S && mm < nx) {
          const double* ph = Phi + (int64_t)mm * ldy + c0;
#pragma unroll
          for (int t = 0; t < UCH; ++t) acc[t] += pf.mc[q] * ph[t];
        }
      }
    for (int o = 1; o < P; o <<= 1)
#pragma unroll
      for (int t = 0; t < UCH; ++t) acc[t] += __shfl_xor(acc[t], o);
    if (r < nux && p == 0)
#pragma unroll
      for (int t = 0; t < UCH; ++t)
        if (c0 + t < W) Ynew[(int64_t)r * ldy + c0 + t] = acc[t];
  }
}

// stage_columns from the prefetched row entries and penalty changes.
__device__ int commit_columns(const UpdArgs& a, const Desc& D, const StagePrefetch& pf, double* Y, double* sg, int W0,
                              int* cmap, double* sds, int& cnt) {
  const int m = a.u.m, nux = D.nx + D.nu, tid = threadIdx.x;
  if (tid < m) {
    sds[tid] = pf.ds;
    cmap[tid] = pf.ds != 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    int c = W0;
    for (int i = 0; i < m; ++i) cmap[i] = cmap[i] ? c++ : -1;
    cnt = c;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = tid + q * UT, r = e % nux, i = e / nux;
    if (e < nux * m && cmap[i] >= 0) {
      const double s = sds[i];
      Y[(int64_t)r * a.ldy + cmap[i]] = sqrt(fabs(s)) * pf.rv[q];
      if (r == 0) sg[cmap[i]] = s > 0.0 ? 1.0 : -1.0;
    }
  }
  const int W = cnt;
  __syncthreads();
  return W;
}

// Pass 1, one workgroup per instance, backward in time: the input pivots of every stage
// ([L^R_k; L^S_k] with Upsilon_k), which leave Phi_k (the state rows), and the products that form
// Upsilon_{k-1} from Phi_k.  Phi_k and its signs go to the update workspace for pass 2.
template <bool PF>
__global__ __launch_bounds__(UT) void k_update_inputs(UpdArgs a) {
  extern __shared__ double sm[];
  __shared__ int s_cmap[LQ_UPDATE_MAX_ROWS];
  __shared__ double s_ds[LQ_UPDATE_MAX_ROWS];
  __shared__ int s_cnt, s_tot, s_bad, s_kind, s_code;
  const int b = blockIdx.x, tid = threadIdx.x;
  const Desc D = a.desc[b];
  const int N = D.N, nx = D.nx, nu = D.nu, nux = nx + nu, m = a.u.m, ldy = a.ldy, wmax = a.wmax;
  const int64_t fs = stage_factor_elems(nx, nu), lrs = off_LQ(nx, nu);

  // total width of Upsilon at stage 0 = all nonzero rows of the instance
  if (tid == 0) { s_tot = 0; s_code = 0; }
  __syncthreads();
  {
    const double* ds = a.u.dsig + (int64_t)m * D.oK;
    int c = 0;
    for (int64_t e = tid; e < (int64_t)(N + 1) * m; e += UT) c += ds[e] != 0.0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((tid & 63) == 0 && c) atomicAdd(&s_tot, c);
    __syncthreads();
    if (s_tot > wmax) {
      if (tid == 0) a.st[b] = -1;
      return;
    }
  }
  double* blk = sm;  // L^R, 1/diag L^R, L^S of the stage
  double* Yc = blk + a.lrsmax;
  double* Yn = Yc + (int64_t)a.nuxmax * ldy;
  double* sgc = Yn + (int64_t)a.nuxmax * ldy;
  double* sgn = sgc + ldy;
  double* dg = sgn + ldy;
  double* Fi = a.F + D.oF;
  double* Phi_i = a.Phi + (int64_t)wmax * D.olam;
  double* Sg_i = a.Sg + (int64_t)wmax * D.oK;
  int32_t* Wk_i = a.Wk + D.oK;
  double* LR = blk;
  double* dR = blk + off_dR(nx, nu);
  double* LS = blk + off_LS(nx, nu);
  auto rowU = [&](int rr) -> double* { return rr < nu ? LR + rr * (rr + 1) / 2 : LS + (rr - nu) * nu; };
  // Phi_k (state rows of the current Upsilon) and its signs to the workspace
  auto save_phi = [&](int k, int W) {
    if (tid == 0) Wk_i[k] = W;
    double* dst = Phi_i + (int64_t)(k - 1) * nx * wmax;
    for (int e = tid; e < nx * W; e += UT) {
      const int r = e / W, c = e % W;
      dst[(int64_t)r * wmax + c] = Yc[(int64_t)(nu + r) * ldy + c];
    }
    for (int c = tid; c < W; c += UT) Sg_i[(int64_t)k * wmax + c] = sgc[c];
  };

  // stage N: Phi_N from the terminal rows
  StagePrefetch pf;
  int Wc = 0;
  // Upsilon_{j} from Phi_{j+1} (current state rows, width Wc) and stage j's own rows
  auto next_upsilon = [&](int j) {
    int W = 0;
    if (Wc > 0) {
      if constexpr (PF) upsilon_products_pf(D, pf, Yc + (int64_t)nu * ldy, ldy, Yn, Wc);
      else upsilon_products(a, D, j, Yc + (int64_t)nu * ldy, Yn, Wc);
      for (int c = tid; c < Wc; c += UT) sgn[c] = sgc[c];
      W = Wc;
    }
    if constexpr (PF) return commit_columns(a, D, pf, Yn, sgn, W, s_cmap, s_ds, s_cnt);
    else return stage_columns(a, D, j, Yn, sgn, W, s_cmap, s_cnt);
  };
  Wc = stage_columns(a, D, N, Yc, sgc, 0, s_cmap, s_cnt);
  save_phi(N, Wc);
  if constexpr (PF) prefetch_stage(a, D, N - 1, pf);
  int Wn = next_upsilon(N - 1);
  for (int k = N - 1; k >= 0; --k) {
    {
      double* t = Yc; Yc = Yn; Yn = t;
      t = sgc; sgc = sgn; sgn = t;
      Wc = Wn;
    }
    if constexpr (PF)
      if (k > 0) prefetch_stage(a, D, k - 1, pf);  // in flight during this stage's pivots
    if (Wc > 0) {
      const double* src = Fi + (int64_t)k * fs;
#pragma unroll 8
      for (int e = tid; e < lrs; e += UT) blk[e] = src[e];
      if (tid == 0) { s_bad = -1; s_kind = 0; }
      __syncthreads();
      hyh(rowU, nux, nu, Yc, ldy, Wc, sgc, dg, s_bad, s_kind);
      if (tid == 0 && s_bad >= 0) s_code = max(s_code, 2 * (k + 1) + (s_kind == 2));
      for (int i = tid; i < nu; i += UT) dR[i] = 1.0 / dg[i];
      __syncthreads();
      double* dst = Fi + (int64_t)k * fs;
      for (int e = tid; e < lrs; e += UT) dst[e] = blk[e];
    }
    if (k > 0) {
      save_phi(k, Wc);
      Wn = next_upsilon(k - 1);
    }
    __syncthreads();
  }
  if (tid == 0) a.st[b] = s_code;
}

// Pass 2: L^Q_k <- hyh(L^Q_k, Phi_k) for every stage k = 1..N at once (the stages are independent
// once pass 1 has produced their Phi_k).  A workgroup takes `ns` consecutive stages of one instance,
// one team of nx groups of 4 lanes per stage (R = 1; R = 2: one stage, groups own rows g and g + 64).
// Each group keeps its Phi row in registers (CPL columns per lane); the row that is the next pivot
// is published to the team's double-buffered LDS row after its own update, so LDS holds only the
// teams' L^Q_k.
template <int R, int CPL>
__device__ void states_pivots(double (&y)[R][CPL], double* LQ, double* piv, const double* sg, double* dg, int nx,
                              int W, int rr, int l, bool lead, int& bad, int& kind) {
  constexpr int G = 4, NG = UT / G;
  for (int i = 0; i < nx; ++i) {
    if (W > 0) {
      const double* yi = piv + (i & 1) * LQ_UPDATE_MAX_ROWS;
      double* ynext = piv + ((i + 1) & 1) * LQ_UPDATE_MAX_ROWS;
      const double a0 = LQ[i * (i + 1) / 2 + i];
      double part = 0.0;
#pragma unroll
      for (int j = 0; j < CPL; ++j) {
        const int c = l + G * j;
        if (c < W) part += sg[c] * yi[c] * yi[c];
      }
      const double r2 = a0 * a0 + group_sum<G>(part);
      const bool ok = r2 > 0.0 && r2 <= DBL_MAX;
      const double rn = ok ? sqrt(r2) : 1.0;
      const double w1 = fabs(a0) + rn;
      const double tinv = 1.0 / (rn * w1);
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int r = rr + NG * t;
        if (r > i && r < nx) {
          double gp = 0.0;
#pragma unroll
          for (int j = 0; j < CPL; ++j) {
            const int c = l + G * j;
            if (c < W) gp += y[t][j] * sg[c] * yi[c];
          }
          gp = group_sum<G>(gp);
          double* lr = LQ + r * (r + 1) / 2;
          const double li = lr[i];
          const double coef = (li * w1 + gp) * tinv;
#pragma unroll
          for (int j = 0; j < CPL; ++j) {
            const int c = l + G * j;
            if (c < W) y[t][j] -= coef * yi[c];
          }
          if (l == 0) lr[i] = coef * w1 - li;
          if (r == i + 1)
#pragma unroll
            for (int j = 0; j < CPL; ++j)
              if (l + G * j < W) ynext[l + G * j] = y[t][j];
        }
      }
      if (lead) {
        dg[i] = rn;
        if (!ok && bad < 0) {
          bad = i;
          kind = r2 != r2 || r2 > DBL_MAX ? 2 : 1;
        }
      }
    }
    __syncthreads();
  }
}

template <int R, int CPL>
__device__ void states_body(const UpdArgs& a, const Desc& D, int k, int W, double* LQ, double* piv, double* sg,
                            double* dg, int rr, int l, int tt, int nthr_team, int& bad, int& kind) {
  constexpr int G = 4, NG = UT / G;
  const int nx = D.nx, wmax = a.wmax;
  double y[R][CPL];
  const double* Ph = a.Phi + (int64_t)wmax * D.olam + (int64_t)(k - 1) * nx * wmax;
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int r = rr + NG * t;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const int c = l + G * j;
      y[t][j] = (W > 0 && r < nx && c < W) ? Ph[(int64_t)r * wmax + c] : 0.0;
    }
    if (W > 0 && r == 0)
#pragma unroll
      for (int j = 0; j < CPL; ++j)
        if (l + G * j < W) piv[l + G * j] = y[t][j];
  }
  if (W > 0)
    for (int c = tt; c < W; c += nthr_team) sg[c] = a.Sg[(int64_t)wmax * D.oK + (int64_t)k * wmax + c];
  __syncthreads();
  states_pivots<R, CPL>(y, LQ, piv, sg, dg, nx, W, rr, l, rr == 0 && l == 0, bad, kind);
}

template <int R>
__global__ __launch_bounds__(UT) void k_update_states(UpdArgs a, int ns) {
  constexpr int G = 4, NG = UT / G;
  extern __shared__ double sm[];
  __shared__ int s_wmax;
  const int b = blockIdx.y, tid = threadIdx.x, g = tid / G, l = tid % G;
  const Desc D = a.desc[b];
  if (a.st[b] < 0 || (int64_t)blockIdx.x * ns + 1 > D.N) return;
  const int nx = D.nx, nu = D.nu;
  const int gpt = R == 1 ? nx : NG;         // groups per team (one team per stage)
  const int team = g / gpt, rr = g % gpt;   // this group's stage slot and row
  const int nthr_team = gpt * G, tt = tid - team * nthr_team;
  const int k = blockIdx.x * ns + 1 + team;
  const bool active = team < ns && k <= D.N;
  const int W = active ? a.Wk[D.oK + k] : 0;
  if (tid == 0) s_wmax = 0;
  __syncthreads();
  if (W > 0 && tt == 0) atomicMax(&s_wmax, W);
  __syncthreads();
  const int wg_w = s_wmax;
  if (wg_w == 0) return;  // no stage of this workgroup changes
  const int64_t lq = (int64_t)nx * (nx + 1) / 2 + nx;
  const int64_t per = lq + nx + 3 * LQ_UPDATE_MAX_ROWS;  // L^Q and 1/diag, new diagonal, pivot rows, signs
  double* LQ = sm + (active ? team : 0) * per;
  double* dQ = LQ + (int64_t)nx * (nx + 1) / 2;
  double* dg = LQ + lq;
  double* piv = dg + nx;
  double* sg = piv + 2 * LQ_UPDATE_MAX_ROWS;
  double* blkQ = active ? a.F + D.oF + (int64_t)k * stage_factor_elems(nx, nu) + off_LQ(nx, nu) : nullptr;
  if (W > 0)
#pragma unroll 4
    for (int64_t e = tt; e < lq; e += nthr_team) LQ[e] = blkQ[e];
  int bad = -1, kind = 0;
  if (wg_w <= 16) states_body<R, 4>(a, D, k, W, LQ, piv, sg, dg, rr, l, tt, nthr_team, bad, kind);
  else states_body<R, 16>(a, D, k, W, LQ, piv, sg, dg, rr, l, tt, nthr_team, bad, kind);
  if (W > 0) {
    for (int i = tt; i < nx; i += nthr_team) {
      LQ[i * (i + 1) / 2 + i] = dg[i];
      dQ[i] = 1.0 / dg[i];
    }
  }
  __syncthreads();
  if (W > 0) {
    for (int64_t e = tt; e < lq; e += nthr_team) blkQ[e] = LQ[e];
    if (tt == 0 && bad >= 0) atomicMax(a.st + b, 2 * (k + 1) + (kind == 2));
  }
}

// Pass 3, one workgroup per instance: the right-hand-side sweep of the factorisation from the
// (updated) factors and the data's q, r, f (the vectors lq_solve starts from), and the status.
//   p_N = q_N;  w = L^Q_{k+1} L^Q_{k+1}^T f_k + p_{k+1};  rbar_k = (L^R_k)^{-1} (r_k + B_k^T w);
//   p_k = q_k + A_k^T w - L^S_k rbar_k
__global__ __launch_bounds__(UT) void k_update_sweep(UpdArgs a, int with_rows) {
  extern __shared__ double sm[];
  const int b = blockIdx.x, tid = threadIdx.x;
  const Desc D = a.desc[b];
  const int N = D.N, nx = D.nx, nu = D.nu, nux = nx + nu;
  const int64_t fs = stage_factor_elems(nx, nu);
  if (with_rows) {
    const int code = a.st[b];
    if (code < 0) {
      if (tid == 0) a.info[b] = LQ_INFO_UPDATE_RANK;
      return;
    }
    if (tid == 0) a.info[b] = code == 0 ? 0 : ((code & 1) ? LQ_INFO_NONFINITE : code / 2);
  } else if (tid == 0) {
    a.info[b] = 0;
  }
  double* blk = sm;
  double* pn = blk + a.fsmax;
  double* wv = pn + a.nxmax;
  double* tv = wv + a.nxmax;
  double* tq = tv + a.nxmax;
  const double* Fi = a.F + D.oF;
  double* rbar = a.V + D.oV;
  double* pv = rbar + (int64_t)N * nu;
  const double* q = a.d.q + D.oq;
  const double* r = a.d.r + D.or_;
  const double* f = a.d.f ? a.d.f + D.of : nullptr;
  const double* LR = blk;
  const double* dR = blk + off_dR(nx, nu);
  const double* LS = blk + off_LS(nx, nu);
  const double* LQ = blk + off_LQ(nx, nu);
  auto load_block = [&](int k) {
    const double* src = Fi + (int64_t)k * fs;
#pragma unroll 8
    for (int e = tid; e < fs; e += UT) blk[e] = src[e];
  };
  // w = L^Q (L^Q)^T f_{k-1} + p_k with the block of stage k in LDS
  auto next_w = [&](int k) {
    if (f) {
      for (int i = tid; i < nx; i += UT) tq[i] = f[(int64_t)(k - 1) * nx + i];
      __syncthreads();
      for (int j = tid; j < nx; j += UT) {
        double s = 0.0;
        for (int mm = j; mm < nx; ++mm) s += LQ[mm * (mm + 1) / 2 + j] * tq[mm];
        tv[j] = s;
      }
      __syncthreads();
    }
    for (int i = tid; i < nx; i += UT) {
      double s = pn[i];
      if (f)
        for (int j = 0; j <= i; ++j) s += LQ[i * (i + 1) / 2 + j] * tv[j];
      wv[i] = s;
    }
    __syncthreads();
  };
  load_block(N);
  for (int i = tid; i < nx; i += UT) {
    const double v = q[(int64_t)N * nx + i];
    pn[i] = v;
    pv[(int64_t)N * nx + i] = v;
  }
  __syncthreads();
  next_w(N);
  for (int k = N - 1; k >= 0; --k) {
    load_block(k);
    __syncthreads();
    const double* Ak = a.d.A + D.oA + (int64_t)k * nx * nx;
    const double* Bk = a.d.B + D.oB + (int64_t)k * nx * nu;
    const int nrow = k > 0 ? nux : nu;
    for (int j = tid; j < nrow; j += UT) {
      double s;
      const double* Mc;
      int ldm;
      if (j < nu) { s = r[(int64_t)k * nu + j]; Mc = Bk + j; ldm = nu; }
      else { s = q[(int64_t)k * nx + (j - nu)]; Mc = Ak + (j - nu); ldm = nx; }
#pragma unroll 4
      for (int mm = 0; mm < nx; ++mm) s += Mc[(int64_t)mm * ldm] * wv[mm];
      tq[j] = s;
    }
    __syncthreads();
    if (nu <= 64) {
      // wave 0, lane i holds entry i: column-oriented forward substitution with lane broadcasts
      if (tid < 64) {
        const int ln = tid;
        double v = ln < nu ? tq[ln] : 0.0;
        for (int j = 0; j < nu; ++j) {
          const double xj = __shfl(v, j) * dR[j];
          if (ln == j) v = xj;
          else if (ln > j && ln < nu) v -= LR[ln * (ln + 1) / 2 + j] * xj;
        }
        if (ln < nu) tq[ln] = v;
      }
    } else if (tid == 0) {
      for (int i = 0; i < nu; ++i) {
        double s = tq[i];
        for (int j = 0; j < i; ++j) s -= LR[i * (i + 1) / 2 + j] * tq[j];
        tq[i] = s * dR[i];
      }
    }
    __syncthreads();
    for (int i = tid; i < nu; i += UT) rbar[(int64_t)k * nu + i] = tq[i];
    if (k > 0)
      for (int i = tid; i < nx; i += UT) {
        double s = tq[nu + i];
        for (int j = 0; j < nu; ++j) s -= LS[i * nu + j] * tq[j];
        pn[i] = s;
        pv[(int64_t)k * nx + i] = s;
      }
    __syncthreads();
    if (k > 0) next_w(k);
  }
}

// LDS doubles of the three passes for the plan's largest stage and a width cap (row stride ldy).
static size_t inputs_lds_doubles(int lrsmax, int nuxmax, int ldy) {
  return (size_t)lrsmax + 2 * (size_t)nuxmax * ldy + 2 * (size_t)ldy + nuxmax;
}
static int states_per_wg(int nxmax) { return nxmax <= UT / 4 ? (UT / 4) / nxmax : 1; }
static size_t states_lds_doubles(int lqmax, int nxmax) {
  return (size_t)states_per_wg(nxmax) * ((size_t)lqmax + nxmax + 3 * LQ_UPDATE_MAX_ROWS);
}
static size_t sweep_lds_doubles(int fsmax, int nuxmax, int nxmax) { return (size_t)fsmax + 3 * (size_t)nxmax + nuxmax; }

// Width cap of Upsilon: the largest multiple of 8 up to LQ_UPDATE_MAX_ROWS whose first pass fits two
// workgroups per CU if that still allows 32 columns, else one; the second pass must fit too.
int update_width(int lrsmax, int lqmax, int nuxmax, int nxmax, int* ldy_out) {
  const size_t lds_cu = 160 * 1024, stat = 1024;  // LDS per CU; static arrays of the kernels
  for (int per_cu : {2, 1}) {
    const size_t cap = lds_cu / per_cu - stat;
    for (int w = LQ_UPDATE_MAX_ROWS; w >= (per_cu == 2 ? 32 : UCH); w -= UCH) {
      const int ldy = w + 1;
      if (inputs_lds_doubles(lrsmax, nuxmax, ldy) * sizeof(double) <= cap &&
          states_lds_doubles(lqmax, nxmax) * sizeof(double) <= lds_cu - stat && nxmax <= 2 * (UT / 4)) {
        if (ldy_out) *ldy_out = ldy;
        return w;
      }
    }
  }
  if (ldy_out) *ldy_out = 0;
  return 0;
}

bool update_sweep_fits(int fsmax, int nuxmax, int nxmax) {
  return sweep_lds_doubles(fsmax, nuxmax, nxmax) * sizeof(double) <= 160 * 1024 - 1024;
}

hipError_t launch_update_data(const Desc* desc, int batch, int maxN, const lq_update& u, double* Q, double* R,
                              double* S, hipStream_t st) {
  const int spb = (maxN + 1 + 65534) / 65535 > 4 ? (maxN + 1 + 65534) / 65535 : 4;
  const dim3 grid(batch, (maxN + 1 + spb - 1) / spb);
  hipLaunchKernelGGL(k_update_data, grid, dim3(256), 0, st, desc, u, Q, R, S, spb);
  return hipGetLastError();
}

// Byte offsets of the update workspace: Phi (wmax * sum N nx doubles), signs (wmax * sum (N + 1)
// doubles), Wk (sum (N + 1) int32), st (batch int32).
void update_ws_layout(int wmax, int64_t sum_Nnx, int64_t sum_K, int batch, size_t* oSg, size_t* oWk, size_t* oSt,
                      size_t* total) {
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  *oSg = al(sizeof(double) * (size_t)wmax * sum_Nnx);
  *oWk = al(*oSg + sizeof(double) * (size_t)wmax * sum_K);
  *oSt = al(*oWk + sizeof(int32_t) * (size_t)sum_K);
  *total = al(*oSt + sizeof(int32_t) * (size_t)batch);
}

hipError_t launch_factor_update(const Desc* desc, int batch, int maxN, int lrsmax, int lqmax, int fsmax, int nuxmax,
                                int nxmax, int64_t sum_Nnx, int64_t sum_K, const lq_data& d, const lq_update& u,
                                double* F, double* V, void* uws, int32_t* info, hipStream_t st) {
  UpdArgs a = {};
  a.desc = desc;
  a.d = d;
  a.F = F;
  a.V = V;
  a.u = u;
  a.lrsmax = lrsmax;
  a.lqmax = lqmax;
  a.fsmax = fsmax;
  a.nuxmax = nuxmax;
  a.nxmax = nxmax;
  a.info = info;
  hipError_t e;
  const bool rows = u.m > 0;
  if (rows) {
    int ldy = 0;
    const int wmax = update_width(lrsmax, lqmax, nuxmax, nxmax, &ldy);
    if (wmax <= 0) return hipErrorInvalidValue;
    a.wmax = wmax;
    a.ldy = ldy;
    size_t oSg, oWk, oSt, tot;
    update_ws_layout(wmax, sum_Nnx, sum_K, batch, &oSg, &oWk, &oSt, &tot);
    char* w = (char*)uws;
    a.Phi = (double*)w;
    a.Sg = (double*)(w + oSg);
    a.Wk = (int32_t*)(w + oWk);
    a.st = (int32_t*)(w + oSt);
    const size_t l1 = inputs_lds_doubles(lrsmax, nuxmax, ldy) * sizeof(double);
    const size_t l2 = states_lds_doubles(lqmax, nxmax) * sizeof(double);
    const int ns = states_per_wg(nxmax);
    const void* k2 = nxmax <= UT / 4 ? (const void*)k_update_states<1> : (const void*)k_update_states<2>;
    // prefetching the products' columns costs registers (occupancy); it pays where each row's share
    // of the state dimension is long (few parts per row), not for small stages
    const bool pf = parts_of(nuxmax) <= 4 && (nxmax + parts_of(nuxmax) - 1) / parts_of(nuxmax) <= PMAX &&
                    (int64_t)nuxmax * u.m <= 2 * UT;
    const void* k1 = pf ? (const void*)k_update_inputs<true> : (const void*)k_update_inputs<false>;
    if ((e = raise_lds_limit(k1, l1)) != hipSuccess) return e;
    if ((e = raise_lds_limit(k2, l2)) != hipSuccess) return e;
    void* args1[] = {&a};
    if ((e = hipLaunchKernel(k1, dim3(batch), dim3(UT), args1, l1, st)) != hipSuccess) return e;
    void* args[] = {&a, (void*)&ns};
    if ((e = hipLaunchKernel(k2, dim3((maxN + ns - 1) / ns, batch), dim3(UT), args, l2, st)) != hipSuccess) return e;
  }
  const size_t l3 = sweep_lds_doubles(fsmax, nuxmax, nxmax) * sizeof(double);
  if ((e = raise_lds_limit((const void*)k_update_sweep, l3)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_update_sweep, dim3(batch), dim3(UT), l3, st, a, rows ? 1 : 0);
  return hipGetLastError();
}

}  // namespace lq
