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
// Factor update.  256 threads in 16 groups of 16 lanes: in a hyperbolic step each group owns
// factor rows, its lanes split the columns of Upsilon and reduce by 16-lane shuffles.
constexpr int UT = 256;
constexpr int UG = 16;
constexpr int UNG = UT / UG;
constexpr int UCH = 8;  // columns per thread in the Upsilon products

struct UpdArgs {
  const Desc* desc;
  lq_data d;
  double* F;  // factor region (float64 plan)
  double* V;  // right-hand-side sweep (rbar, p)
  lq_update u;
  int32_t wmax, ldy, fsmax, nuxmax, nxmax;
  int32_t* info;
};

__device__ __forceinline__ double sum16(double v) {
  v += __shfl_xor(v, 8, UG);
  v += __shfl_xor(v, 4, UG);
  v += __shfl_xor(v, 2, UG);
  v += __shfl_xor(v, 1, UG);
  return v;
}

// Hyperbolic Householder update of the factor rows [0, nrows), pivots [0, npiv) (row r of L
// starts at row(r)) with the W columns of Y (row stride ldy, signature sg).  Rows below each
// pivot are rewritten; the pivot rows of Y are left stale (they are zero in exact terms).  The
// first failing pivot (r^2 not positive: kind 1, not finite: kind 2) is recorded in bad/kind and
// its r replaced by 1.
template <class RowF>
__device__ void hyh(RowF row, int nrows, int npiv, double* Y, int ldy, int W, const double* sg, double* dg,
                    int& bad, int& kind) {
  const int tid = threadIdx.x, g = tid / UG, l = tid % UG;
  for (int i = 0; i < npiv; ++i) {
    const double* yi = Y + (int64_t)i * ldy;
    const double a = row(i)[i];
    double part = 0.0;
    for (int c = l; c < W; c += UG) {
      const double b = yi[c];
      part += sg[c] * b * b;
    }
    const double r2 = a * a + sum16(part);
    const bool ok = r2 > 0.0 && r2 <= DBL_MAX;
    const double rn = ok ? sqrt(r2) : 1.0;
    const double w1 = fabs(a) + rn;
    const double tinv = 1.0 / (rn * w1);  // 2 / (w^T J w)
    for (int r = i + 1 + g; r < nrows; r += UNG) {
      double* lr = row(r);
      double* yr = Y + (int64_t)r * ldy;
      double gp = 0.0;
      for (int c = l; c < W; c += UG) gp += yr[c] * sg[c] * yi[c];
      gp = sum16(gp);
      const double li = lr[i];
      const double coef = (li * w1 + gp) * tinv;
      for (int c = l; c < W; c += UG) yr[c] -= coef * yi[c];
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

// Appends the nonzero rows of stage j as columns W0.. of Y (u rows from D_j, x rows from C_j,
// scaled by sqrt|dSigma|) and their signs to sg; returns the new width (uniform over the block).
__device__ int stage_columns(const UpdArgs& a, const Desc& D, int j, double* Y, double* sg, int W0, int* cmap,
                             int& cnt) {
  const int m = a.u.m, nx = D.nx, nu = D.nu, nux = nx + nu, tid = threadIdx.x;
  if (m == 0) return W0;
  const double* sj = a.u.dsig + (int64_t)m * D.oK + (int64_t)j * m;
  if (tid == 0) {
    int c = W0;
    for (int i = 0; i < m; ++i) cmap[i] = sj[i] != 0.0 ? c++ : -1;
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

__global__ __launch_bounds__(UT) void k_factor_update(UpdArgs a) {
  extern __shared__ double sm[];
  __shared__ int s_cmap[LQ_UPDATE_MAX_ROWS];
  __shared__ int s_cnt, s_tot, s_bad, s_kind, s_info;
  const int b = blockIdx.x, tid = threadIdx.x;
  const Desc D = a.desc[b];
  const int N = D.N, nx = D.nx, nu = D.nu, nux = nx + nu, m = a.u.m, ldy = a.ldy;
  const int64_t fs = stage_factor_elems(nx, nu);

  // total width of Upsilon at stage 0 = all nonzero rows of the instance
  if (tid == 0) { s_tot = 0; s_info = 0; }
  __syncthreads();
  if (m > 0) {
    const double* ds = a.u.dsig + (int64_t)m * D.oK;
    int c = 0;
    for (int64_t e = tid; e < (int64_t)(N + 1) * m; e += UT) c += ds[e] != 0.0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((tid & 63) == 0 && c) atomicAdd(&s_tot, c);
    __syncthreads();
    if (s_tot > a.wmax) {
      if (tid == 0) a.info[b] = LQ_INFO_UPDATE_RANK;
      return;
    }
  }

  double* blk = sm;
  double* Yc = blk + a.fsmax;
  double* Yn = Yc + (int64_t)a.nuxmax * ldy;
  double* sgc = Yn + (int64_t)a.nuxmax * ldy;
  double* sgn = sgc + ldy;
  double* dg = sgn + ldy;
  double* pn = dg + a.nuxmax;  // p_{k+1}, then p_k
  double* wv = pn + a.nxmax;   // w = P_{k+1} f_k + p_{k+1}
  double* tv = wv + a.nxmax;
  double* tq = tv + a.nxmax;   // (rhat, qhat)

  double* Fi = a.F + D.oF;
  double* rbar = a.V + D.oV;
  double* pv = rbar + (int64_t)N * nu;
  const double* q = a.d.q + D.oq;
  const double* r = a.d.r + D.or_;
  const double* f = a.d.f ? a.d.f + D.of : nullptr;
  double* LR = blk;
  double* dR = blk + off_dR(nx, nu);
  double* LS = blk + off_LS(nx, nu);
  double* LQ = blk + off_LQ(nx, nu);
  double* dQ = blk + off_dQ(nx, nu);
  auto rowU = [&](int rr) -> double* { return rr < nu ? LR + rr * (rr + 1) / 2 : LS + (rr - nu) * nu; };
  auto rowQ = [&](int rr) -> double* { return LQ + rr * (rr + 1) / 2; };
  auto load_block = [&](int k) {
    const double* src = Fi + (int64_t)k * fs;
    for (int e = tid; e < fs; e += UT) blk[e] = src[e];
    if (tid == 0) { s_bad = -1; s_kind = 0; }
    __syncthreads();
  };
  auto store_block = [&](int k) {
    double* dst = Fi + (int64_t)k * fs;
    for (int e = tid; e < fs; e += UT) dst[e] = blk[e];
  };
  auto note_failure = [&](int stage) {
    // s_bad / s_kind are read after the barrier that ends hyh
    if (tid == 0 && s_bad >= 0 && s_info == 0) s_info = s_kind == 2 ? LQ_INFO_NONFINITE : stage + 1;
  };
  // w = L^Q_k (L^Q_k)^T f_{k-1} + p_k from the block in LDS and pn
  auto next_w = [&](int k) {
    const double* fk = f ? f + (int64_t)(k - 1) * nx : nullptr;
    if (fk) {
      for (int j = tid; j < nx; j += UT) {
        double s = 0.0;
        for (int mm = j; mm < nx; ++mm) s += LQ[mm * (mm + 1) / 2 + j] * fk[mm];
        tv[j] = s;
      }
      __syncthreads();
    }
    for (int i = tid; i < nx; i += UT) {
      double s = pn[i];
      if (fk)
        for (int j = 0; j <= i; ++j) s += LQ[i * (i + 1) / 2 + j] * tv[j];
      wv[i] = s;
    }
    __syncthreads();
  };

  // ---- stage N: Phi_N from the terminal rows, then L^Q_N
  load_block(N);
  int Wc = stage_columns(a, D, N, Yc, sgc, 0, s_cmap, s_cnt);
  int Wn = 0;
  if (Wc > 0) {
    upsilon_products(a, D, N - 1, Yc + (int64_t)nu * ldy, Yn, Wc);
    for (int c = tid; c < Wc; c += UT) sgn[c] = sgc[c];
    Wn = Wc;
    __syncthreads();
    hyh(rowQ, nx, nx, Yc + (int64_t)nu * ldy, ldy, Wc, sgc, dg, s_bad, s_kind);
    note_failure(N);
    for (int i = tid; i < nx; i += UT) dQ[i] = 1.0 / dg[i];
    __syncthreads();
    store_block(N);
  }
  Wn = stage_columns(a, D, N - 1, Yn, sgn, Wn, s_cmap, s_cnt);
  for (int i = tid; i < nx; i += UT) {
    const double v = q[(int64_t)N * nx + i];
    pn[i] = v;
    pv[(int64_t)N * nx + i] = v;
  }
  __syncthreads();
  next_w(N);

  for (int k = N - 1; k >= 0; --k) {
    {
      double* t = Yc; Yc = Yn; Yn = t;
      t = sgc; sgc = sgn; sgn = t;
      Wc = Wn;
    }
    load_block(k);
    if (Wc > 0) {
      hyh(rowU, nux, nu, Yc, ldy, Wc, sgc, dg, s_bad, s_kind);
      note_failure(k);
      for (int i = tid; i < nu; i += UT) dR[i] = 1.0 / dg[i];
      __syncthreads();
    }
    // (rhat, qhat) = (r_k, q_k) + [B_k A_k]^T w;  rbar_k = (L^R_k)^{-1} rhat;  p_k = qhat - L^S_k rbar_k
    {
      const double* Ak = a.d.A + D.oA + (int64_t)k * nx * nx;
      const double* Bk = a.d.B + D.oB + (int64_t)k * nx * nu;
      const int nrow = k > 0 ? nux : nu;
      for (int j = tid; j < nrow; j += UT) {
        double s;
        const double* Mc;
        int ldm;
        if (j < nu) { s = r[(int64_t)k * nu + j]; Mc = Bk + j; ldm = nu; }
        else { s = q[(int64_t)k * nx + (j - nu)]; Mc = Ak + (j - nu); ldm = nx; }
        for (int mm = 0; mm < nx; ++mm) s += Mc[(int64_t)mm * ldm] * wv[mm];
        tq[j] = s;
      }
      __syncthreads();
      if (tid == 0)
        for (int i = 0; i < nu; ++i) {
          double s = tq[i];
          for (int j = 0; j < i; ++j) s -= LR[i * (i + 1) / 2 + j] * tq[j];
          tq[i] = s * dR[i];
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
    }
    if (k > 0) {
      Wn = 0;
      if (Wc > 0) {
        upsilon_products(a, D, k - 1, Yc + (int64_t)nu * ldy, Yn, Wc);
        for (int c = tid; c < Wc; c += UT) sgn[c] = sgc[c];
        Wn = Wc;
        __syncthreads();
        hyh(rowQ, nx, nx, Yc + (int64_t)nu * ldy, ldy, Wc, sgc, dg, s_bad, s_kind);
        note_failure(k);
        for (int i = tid; i < nx; i += UT) dQ[i] = 1.0 / dg[i];
        __syncthreads();
      }
      Wn = stage_columns(a, D, k - 1, Yn, sgn, Wn, s_cmap, s_cnt);
      next_w(k);
    }
    if (Wc > 0) store_block(k);
    __syncthreads();
  }
  if (tid == 0) a.info[b] = s_info;
}

// LDS doubles of the update kernel for the plan's largest stage and a width cap.
static size_t update_lds_doubles(int fsmax, int nuxmax, int nxmax, int ldy) {
  return (size_t)fsmax + 2 * (size_t)nuxmax * ldy + 2 * (size_t)ldy + nuxmax + 3 * (size_t)nxmax + nuxmax;
}

int update_width(int fsmax, int nuxmax, int nxmax, int* ldy_out) {
  const size_t cap = 160 * 1024 - 1024;  // LDS per workgroup, less the static arrays
  for (int w = LQ_UPDATE_MAX_ROWS; w >= UCH; w -= UCH) {
    const int ldy = w + 1;
    if (update_lds_doubles(fsmax, nuxmax, nxmax, ldy) * sizeof(double) <= cap) {
      if (ldy_out) *ldy_out = ldy;
      return w;
    }
  }
  if (ldy_out) *ldy_out = 0;
  return 0;
}

hipError_t launch_update_data(const Desc* desc, int batch, int maxN, const lq_update& u, double* Q, double* R,
                              double* S, hipStream_t st) {
  const int spb = (maxN + 1 + 65534) / 65535 > 4 ? (maxN + 1 + 65534) / 65535 : 4;
  const dim3 grid(batch, (maxN + 1 + spb - 1) / spb);
  hipLaunchKernelGGL(k_update_data, grid, dim3(256), 0, st, desc, u, Q, R, S, spb);
  return hipGetLastError();
}

hipError_t launch_factor_update(const Desc* desc, int batch, int fsmax, int nuxmax, int nxmax, const lq_data& d,
                                const lq_update& u, double* F, double* V, int32_t* info, hipStream_t st) {
  int ldy = 0;
  const int wmax = update_width(fsmax, nuxmax, nxmax, &ldy);
  if (wmax <= 0) return hipErrorInvalidValue;
  UpdArgs a;
  a.desc = desc;
  a.d = d;
  a.F = F;
  a.V = V;
  a.u = u;
  a.wmax = wmax;
  a.ldy = ldy;
  a.fsmax = fsmax;
  a.nuxmax = nuxmax;
  a.nxmax = nxmax;
  a.info = info;
  const size_t lds = update_lds_doubles(fsmax, nuxmax, nxmax, ldy) * sizeof(double);
  hipError_t e = raise_lds_limit((const void*)k_factor_update, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_factor_update, dim3(batch), dim3(UT), lds, st, a);
  return hipGetLastError();
}

}  // namespace lq
