// Parallel-in-time factorisation and solution of the LQ-OCP KKT system (paper, Sec. "Cyqlone:
// parallel factorization and solution of KKT systems with optimal control structure"), for uniform
// batches; the formulation and the entry points are described in include/lqpit.h.
//
// Kernels (one workgroup of wg::NT threads per (interval, instance) unless noted):
//   k_pit_factor  the interval's Riccati recursion with the propagated coupling of its outgoing
//                 dynamics constraint (Alg. "factor-block-column-riccati"): stage factors, L^B,
//                 A^cl, and at the interval's first stage L^A; accumulates M^fwd
//   k_pit_schur   Schur complement blocks of one boundary (Sec. "Computation of the Schur
//                 complement"); then the cyclic-reduction factorisation of lqblocktri.h
//   k_pit_bwd     backward vector sweep of an interval (boundary multipliers zero, or given)
//   k_pit_fwd     forward rollout of an interval from its free first state; with zero multipliers
//                 it yields the interval's part of the Schur right-hand side, with the solved
//                 multipliers the solution x, u, lam
//   k_pit_rhs     Schur right-hand side (one workgroup per instance); then the CR solve
//   k_pit_resid   float64 KKT residual rows of a chunk of stages (eq. opt-cond-ocp-eq), maxima by
//                 atomics; k_pit_relres turns them into rel_res and the non-finite status.
#include <stdio.h>
#include <string.h>

#include "lq_internal.hpp"
#include "lq_wgblas.hpp"
#include "lqblocktri.h"
#include "lqpit.h"

namespace lq {
namespace {

using wg::NT;

struct PG {
  int32_t batch, N, nx, nu, nux, P;
  int64_t FS;                         // packed stage block (elements)
  // workspace regions (double offsets)
  int64_t oF, oLQs, oLA, oMf, oScr, oMs, oKs, oCR, oRb, oPv, oG, oRhs, oMu, oAcc, oSinfo, total;
  int64_t SC;                         // scratch doubles per (instance, interval)
  const double *A, *B, *Q, *R, *S, *q, *r, *f, *x0;
};

__host__ __device__ inline int64_t a256(int64_t v) { return (v + 31) & ~(int64_t)31; }  // 256-byte steps of doubles

// first stage of interval p (1-based stages; s_P = N + 1)
__host__ __device__ inline int stage_begin(const PG& g, int p) { return 1 + (int)(((int64_t)p * g.N) / g.P); }

PG layout(int32_t batch, int32_t N, int32_t nx, int32_t nu, int32_t P) {
  PG g;
  memset(&g, 0, sizeof g);
  g.batch = batch; g.N = N; g.nx = nx; g.nu = nu; g.nux = nx + nu; g.P = P;
  g.FS = stage_factor_elems(nx, nu);
  const int64_t nn = (int64_t)nx * nx, bp = (int64_t)batch * P;
  g.SC = (int64_t)g.nux * g.nux + nn + 2 * (int64_t)nx * g.nux + nn + (int64_t)nx * nu + 8 * (int64_t)(g.nux + 8);
  int64_t o = 0;
  g.oF = o; o = a256(o + (int64_t)batch * N * g.FS);
  g.oLQs = o; o = a256(o + bp * nn);
  g.oLA = o; o = a256(o + bp * nn);
  g.oMf = o; o = a256(o + bp * nn);
  g.oScr = o; o = a256(o + bp * g.SC);
  g.oMs = o; o = a256(o + bp * nn);
  g.oKs = o; o = a256(o + (int64_t)batch * (P > 1 ? P - 1 : 1) * nn);
  g.oCR = o; o = a256(o + (int64_t)(lq_bt_workspace_bytes(batch, P, nx, LQ_BT_CR) / sizeof(double)) + 1);
  g.oRb = o; o = a256(o + (int64_t)batch * N * nu);
  g.oPv = o; o = a256(o + (int64_t)batch * N * nx);
  g.oG = o; o = a256(o + bp * 2 * nx);
  g.oRhs = o; o = a256(o + bp * nx);
  g.oMu = o; o = a256(o + bp * nx);
  g.oAcc = o; o = a256(o + 2 * (int64_t)batch);
  g.oSinfo = o; o = a256(o + batch);  // int32 per instance (counted in doubles)
  g.total = o;
  return g;
}

// ---- data access (uniform packed layout of lqkkt.h) --------------------------------------------
__device__ inline const double* mA(const PG& g, int b, int k) { return g.A + ((int64_t)b * g.N + k) * g.nx * g.nx; }
__device__ inline const double* mB(const PG& g, int b, int k) { return g.B + ((int64_t)b * g.N + k) * g.nx * g.nu; }
__device__ inline const double* mQ(const PG& g, int b, int k) { return g.Q + ((int64_t)b * (g.N + 1) + k) * g.nx * g.nx; }
__device__ inline const double* mR(const PG& g, int b, int k) { return g.R + ((int64_t)b * g.N + k) * g.nu * g.nu; }
__device__ inline const double* mS(const PG& g, int b, int k) { return g.S + ((int64_t)b * g.N + k) * g.nu * g.nx; }
__device__ inline const double* vq(const PG& g, int b, int k) { return g.q + ((int64_t)b * (g.N + 1) + k) * g.nx; }
__device__ inline const double* vr(const PG& g, int b, int k) { return g.r + ((int64_t)b * g.N + k) * g.nu; }
__device__ inline const double* vf(const PG& g, int b, int k) { return g.f + ((int64_t)b * g.N + k) * g.nx; }
__device__ inline const double* vx0(const PG& g, int b) { return g.x0 + (int64_t)b * g.nx; }

// Packed stage block j (1..N) of instance b.
__device__ inline double* fblk(const PG& g, double* ws, int b, int j) { return ws + g.oF + ((int64_t)b * g.N + (j - 1)) * g.FS; }

// ---- packed-triangle vector helpers (one workgroup) -----------------------------------------
// Lp: packed lower triangle (row i starts at i(i+1)/2), dinv: 1 / diagonal.

// x <- L^{-1} x (TR = false) or L^{-T} x (TR = true), n <= NT; x in global memory.
template <bool TR>
__device__ void pk_trsv(int n, const double* Lp, const double* dinv, double* x, wg::Smem& sm) {
  wg::trsv_blocked<TR>(
      n, [&](int i, int j) { return Lp[(int64_t)i * (i + 1) / 2 + j]; }, [&](int i) { return dinv[i]; }, x, sm);
}

// y = L x (TR = false) or y = L^T x (TR = true) (+ y when ACC); x and y must not overlap.  Both
// read the packed rows coalesced: L x with a wavefront per row; L^T x with the rows dealt over the
// wavefronts (lanes over the columns) and the partial sums added through LDS.
template <bool TR, bool ACC>
__device__ void pk_trmv(int n, const double* Lp, const double* x, double* y, wg::Smem& sm) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  wg::sync();
  if (!TR) {
    for (int i = w; i < n; i += NW) {
      const double* row = Lp + (int64_t)i * (i + 1) / 2;
      double s = 0.0;
      for (int t = lane; t <= i; t += 64) s = fma(row[t], x[t], s);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
      if (lane == 0) y[i] = ACC ? y[i] + s : s;
    }
    wg::sync();
  } else {
    double* part = &sm.d[0][0];
    for (int i0 = 0; i0 < n; i0 += 64) {
      const int i = i0 + lane;
      double s = 0.0;
      if (i < n) {
#pragma unroll 4
        for (int t = i0 + ((w - i0) % NW + NW) % NW; t < n; t += NW)  // rows t >= i0, t = w mod NW
          if (t >= i) s = fma(Lp[(int64_t)t * (t + 1) / 2 + i], x[t], s);
        part[w * n + i] = s;
      }
    }
    wg::sync();
    for (int i = threadIdx.x; i < n; i += NT) {
      double s = ACC ? y[i] : 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) s += part[q * n + i];
      y[i] = s;
    }
    wg::sync();
  }
}

__device__ inline void vcopy(int n, const double* x, double* y) {
  wg::sync();
  for (int i = threadIdx.x; i < n; i += NT) y[i] = x[i];
  wg::sync();
}

__device__ inline void report(int32_t* info, int b, int code) {
  if (threadIdx.x == 0 && code) atomicCAS(info + b, 0, code);
}

// ---- factorisation ------------------------------------------------------------------------

__global__ void __launch_bounds__(NT, 2) k_pit_factor(PG g, double* ws, int32_t* info) {
  extern __shared__ __align__(16) unsigned char smraw[];
  wg::Smem& sm = *reinterpret_cast<wg::Smem*>(smraw);
  const int p = blockIdx.x, b = blockIdx.y;
  const int nx = g.nx, nu = g.nu, nux = g.nux, N = g.N;
  const int s = stage_begin(g, p), e = stage_begin(g, p + 1) - 1;
  double* scr = ws + g.oScr + ((int64_t)b * g.P + p) * g.SC;
  double* Hh = scr;                                  // nux x nux
  double* LQ = Hh + (int64_t)nux * nux;              // nx x nx (dense lower, zero upper)
  double* W = LQ + (int64_t)nx * nx;                 // nx x nux
  double* Ch = W + (int64_t)nx * nux;                // nx x nux: [B^ A^]
  double* Acl = Ch + (int64_t)nx * nux;              // nx x nx
  double* LB = Acl + (int64_t)nx * nx;               // nx x nu
  double* Mf = ws + g.oMf + ((int64_t)b * g.P + p) * nx * nx;
  double* LA = ws + g.oLA + ((int64_t)b * g.P + p) * nx * nx;
  double* LQs = ws + g.oLQs + ((int64_t)b * g.P + p) * nx * nx;
  wg::fill(nx, nx, 0.0, Mf, nx);
  // coupling of the outgoing dynamics constraint of stage e: (B_e, A_e), or (B_0, 0) for the wrap stage
  {
    const int ce = e < N ? e : 0;
    wg::copy(nx, nu, mB(g, b, ce), nu, Ch, nux);
    if (e < N) wg::copy(nx, nx, mA(g, b, e), nx, Ch + nu, nux);
    else wg::fill(nx, nx, 0.0, Ch + nu, nux);
  }
  for (int j = e; j >= s; --j) {
    const bool wrap = j == N;
    const double* Rj = mR(g, b, wrap ? 0 : j);
    const double* Qj = mQ(g, b, j);
    const double* Sj = (g.S && !wrap) ? mS(g, b, j) : nullptr;
    // stage matrix (lower part): [[sym R, S], [S^T, sym Q]]
    wg::sync();
    for (int el = threadIdx.x; el < nux * nux; el += NT) {
      const int i = el / nux, c = el % nux;
      if (c > i) continue;
      double v;
      if (i < nu) v = 0.5 * (Rj[i * nu + c] + Rj[c * nu + i]);
      else if (c < nu) v = Sj ? Sj[(int64_t)c * nx + (i - nu)] : 0.0;
      else v = 0.5 * (Qj[(int64_t)(i - nu) * nx + (c - nu)] + Qj[(int64_t)(c - nu) * nx + (i - nu)]);
      Hh[(int64_t)i * nux + c] = v;
    }
    wg::sync();
    if (j < e) wg::gemm<true, false, 1>(nux, nux, nx, 1.0, W, nux, W, nux, 1.0, Hh, nux, sm);  // + V V^T
    const int f = wg::potrf(nux, Hh, nux, sm);
    report(info, b, f ? j : 0);
    // packed stage block: L^R, 1/diag L^R, L^S, L^Q, 1/diag L^Q
    double* F = fblk(g, ws, b, j);
    for (int el = threadIdx.x; el < nux * nux; el += NT) {
      const int i = el / nux, c = el % nux;
      if (c > i) continue;
      const double v = Hh[(int64_t)i * nux + c];
      if (i < nu) {
        F[i * (i + 1) / 2 + c] = v;
        if (c == i) F[off_dR(nx, nu) + i] = 1.0 / v;
      } else if (c < nu) {
        F[off_LS(nx, nu) + (int64_t)(i - nu) * nu + c] = v;
      } else {
        const int ii = i - nu, cc = c - nu;
        F[off_LQ(nx, nu) + (int64_t)ii * (ii + 1) / 2 + cc] = v;
        if (cc == ii) F[off_dQ(nx, nu) + ii] = 1.0 / v;
      }
    }
    for (int el = threadIdx.x; el < nx * nx; el += NT) {
      const int i = el / nx, c = el % nx;
      LQ[el] = c <= i ? Hh[(int64_t)(i + nu) * nux + (c + nu)] : 0.0;
    }
    wg::sync();
    // L^B = B^ (L^R)^{-T};  A^cl = A^ - L^B (L^S)^T;  M^fwd += L^B (L^B)^T
    wg::copy(nx, nu, Ch, nux, LB, nu);
    wg::trsm_rlt(nx, nu, Hh, nux, LB, nu, sm);
    wg::copy(nx, nx, Ch + nu, nux, Acl, nx);
    wg::gemm<false, true, 0>(nx, nx, nu, -1.0, LB, nu, Hh + (int64_t)nu * nux, nux, 1.0, Acl, nx, sm);
    wg::gemm<false, true, 1>(nx, nx, nu, 1.0, LB, nu, LB, nu, 1.0, Mf, nx, sm);
    if (j > s) {
      // previous stage: W = (L^Q_j)^T [B_{j-1} A_{j-1}],  (B^, A^) = A^cl [B_{j-1} A_{j-1}]
      const double* Bp = mB(g, b, j - 1);
      const double* Ap = mA(g, b, j - 1);
      wg::gemm<true, false, 0, true>(nx, nu, nx, 1.0, LQ, nx, Bp, nu, 0.0, W, nux, sm);  // (L^Q)^T upper
      wg::gemm<true, false, 0, true>(nx, nx, nx, 1.0, LQ, nx, Ap, nx, 0.0, W + nu, nux, sm);
      wg::gemm<false, false, 0>(nx, nu, nx, 1.0, Acl, nx, Bp, nu, 0.0, Ch, nux, sm);
      wg::gemm<false, false, 0>(nx, nx, nx, 1.0, Acl, nx, Ap, nx, 0.0, Ch + nu, nux, sm);
    } else {
      // first stage of the interval: L^A = A^cl (L^Q_s)^{-T}, M^fwd += L^A (L^A)^T
      wg::copy(nx, nx, Acl, nx, LA, nx);
      wg::trsm_rlt(nx, nx, LQ, nx, LA, nx, sm);
      wg::gemm<false, true, 1>(nx, nx, nx, 1.0, LA, nx, LA, nx, 1.0, Mf, nx, sm);
      wg::copy(nx, nx, LQ, nx, LQs, nx);
    }
  }
}

// Schur complement blocks of boundary p: D_p = (L^Q_{s_p})^{-T} (L^Q_{s_p})^{-1} + M^fwd_{p-1 mod P}
// (lower part), K_p = -L^A_(p) (L^Q_{s_p})^{-1} (p <= P - 2).
__global__ void __launch_bounds__(NT, 2) k_pit_schur(PG g, double* ws) {
  extern __shared__ __align__(16) unsigned char smraw[];
  wg::Smem& sm = *reinterpret_cast<wg::Smem*>(smraw);
  const int p = blockIdx.x, b = blockIdx.y, nx = g.nx, P = g.P;
  const int64_t nn = (int64_t)nx * nx;
  double* X = ws + g.oScr + ((int64_t)b * P + p) * g.SC;  // scratch: X = (L^Q_s)^{-T}
  const double* LQs = ws + g.oLQs + ((int64_t)b * P + p) * nn;
  wg::sync();
  for (int el = threadIdx.x; el < nx * nx; el += NT) X[el] = (el / nx == el % nx) ? 1.0 : 0.0;
  wg::sync();
  wg::trsm_rlt(nx, nx, LQs, nx, X, nx, sm);
  double* D = ws + g.oMs + ((int64_t)b * P + p) * nn;
  const int pm = (p + P - 1) % P;
  wg::copy(nx, nx, ws + g.oMf + ((int64_t)b * P + pm) * nn, nx, D, nx);
  wg::gemm<false, true, 1>(nx, nx, nx, 1.0, X, nx, X, nx, 1.0, D, nx, sm);
  if (p + 1 < P) {
    double* K = ws + g.oKs + ((int64_t)b * (P - 1) + p) * nn;
    wg::gemm<false, true, 0>(nx, nx, nx, -1.0, ws + g.oLA + ((int64_t)b * P + p) * nn, nx, X, nx, 0.0, K, nx, sm);
  }
}

// info[b] <- N + code of the Schur factorisation (code = block row + 1), unless info[b] is set.
__global__ void k_pit_merge_info(PG g, const int32_t* sinfo, int32_t* info) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < g.batch && sinfo[b] != 0 && info[b] == 0) info[b] = g.N + sinfo[b];
}

// ---- solution -----------------------------------------------------------------------------

// Right-hand-side vector of stage j: r (r_0 + S_0 x_init for the wrap stage) and q.
__device__ void stage_rhs(const PG& g, int b, int j, double* rh, double* qh) {
  const int nx = g.nx, nu = g.nu;
  wg::sync();
  if (j < g.N) {
    for (int i = threadIdx.x; i < nu; i += NT) rh[i] = vr(g, b, j)[i];
  } else {
    const double* x0 = vx0(g, b);
    for (int i = threadIdx.x; i < nu; i += NT) {
      double v = vr(g, b, 0)[i];
      if (g.S) {
        const double* S0 = mS(g, b, 0) + (int64_t)i * nx;
        for (int c = 0; c < nx; ++c) v = fma(S0[c], x0[c], v);
      }
      rh[i] = v;
    }
  }
  for (int i = threadIdx.x; i < nx; i += NT) qh[i] = vq(g, b, j)[i];
  wg::sync();
}

// Backward vector sweep of interval p: rbar_j = (L^R_j)^{-1} rhat_j, p_j = qhat_j - L^S_j rbar_j
// with (rhat, qhat) = (r, q) + [B A]^T w, w = L^Q_{j+1} (L^Q_{j+1})^T f_j + p_{j+1} inside the
// interval, and at its last stage the outgoing coupling times the boundary multiplier (USE_MU).
template <bool USE_MU>
__global__ void __launch_bounds__(NT, 2) k_pit_bwd(PG g, double* ws) {
  extern __shared__ __align__(16) unsigned char smraw[];
  wg::Smem& sm = *reinterpret_cast<wg::Smem*>(smraw);
  const int p = blockIdx.x, b = blockIdx.y, nx = g.nx, nu = g.nu, N = g.N;
  const int s = stage_begin(g, p), e = stage_begin(g, p + 1) - 1;
  double* v = ws + g.oScr + ((int64_t)b * g.P + p) * g.SC;  // vector scratch
  double* rh = v;
  double* qh = rh + nu;
  double* w = qh + nx;
  double* t = w + nx;
  for (int j = e; j >= s; --j) {
    stage_rhs(g, b, j, rh, qh);
    if (j < e) {
      const double* Fn = fblk(g, ws, b, j + 1);
      const double* pn = ws + g.oPv + ((int64_t)b * N + j) * nx;  // p_{j+1}
      if (g.f) {
        pk_trmv<true, false>(nx, Fn + off_LQ(nx, nu), vf(g, b, j), t, sm);
        vcopy(nx, pn, w);
        pk_trmv<false, true>(nx, Fn + off_LQ(nx, nu), t, w, sm);
      } else {
        vcopy(nx, pn, w);
      }
      wg::gemv<true>(nx, nu, 1.0, mB(g, b, j), nu, w, 1.0, rh, sm);
      wg::gemv<true>(nx, nx, 1.0, mA(g, b, j), nx, w, 1.0, qh, sm);
    } else if (USE_MU) {
      const double* mu = ws + g.oMu + ((int64_t)b * g.P + (p + 1) % g.P) * nx;
      wg::gemv<true>(nx, nu, 1.0, mB(g, b, j < N ? j : 0), nu, mu, 1.0, rh, sm);
      if (j < N) wg::gemv<true>(nx, nx, 1.0, mA(g, b, j), nx, mu, 1.0, qh, sm);
    }
    const double* F = fblk(g, ws, b, j);
    pk_trsv<false>(nu, F, F + off_dR(nx, nu), rh, sm);
    wg::gemv<false>(nx, nu, -1.0, F + off_LS(nx, nu), nu, rh, 1.0, qh, sm);
    vcopy(nu, rh, ws + g.oRb + ((int64_t)b * N + (j - 1)) * nu);
    vcopy(nx, qh, ws + g.oPv + ((int64_t)b * N + (j - 1)) * nx);
  }
}

// Forward rollout of interval p from x_s = P_s^{-1} (mu_b - p_s):
//   u_j = -(L^R_j)^{-T} ((L^S_j)^T x_j + rbar_j),  x_{j+1} = A_j x_j + B_j u_j + f_j,
//   lam_j = L^Q_{j+1} (L^Q_{j+1})^T x_{j+1} + p_{j+1}.
// SOLVE = false (zero multipliers): the interval's part of the Schur right-hand side, the value
// of its outgoing coupling (B^ u + A^ x at the last stage) and -x_s.  SOLVE = true: x, u, lam.
template <bool SOLVE>
__global__ void __launch_bounds__(NT, 2) k_pit_fwd(PG g, double* ws, double* X, double* U, double* LAM) {
  extern __shared__ __align__(16) unsigned char smraw[];
  wg::Smem& sm = *reinterpret_cast<wg::Smem*>(smraw);
  const int p = blockIdx.x, b = blockIdx.y, nx = g.nx, nu = g.nu, N = g.N;
  const int s = stage_begin(g, p), e = stage_begin(g, p + 1) - 1;
  double* v = ws + g.oScr + ((int64_t)b * g.P + p) * g.SC;
  double* xv = v;
  double* xn = xv + nx;
  double* uv = xn + nx;
  double* t = uv + nu;
  double* gf = ws + g.oG + ((int64_t)b * g.P + p) * 2 * nx;
  // x_s
  {
    const double* Fs = fblk(g, ws, b, s);
    const double* ps = ws + g.oPv + ((int64_t)b * N + (s - 1)) * nx;
    wg::sync();
    for (int i = threadIdx.x; i < nx; i += NT)
      xv[i] = (SOLVE ? ws[g.oMu + ((int64_t)b * g.P + p) * nx + i] : 0.0) - ps[i];
    wg::sync();
    pk_trsv<false>(nx, Fs + off_LQ(nx, nu), Fs + off_dQ(nx, nu), xv, sm);
    pk_trsv<true>(nx, Fs + off_LQ(nx, nu), Fs + off_dQ(nx, nu), xv, sm);
    if (!SOLVE)
      for (int i = threadIdx.x; i < nx; i += NT) gf[nx + i] = -xv[i];
    if (SOLVE) {  // the boundary multiplier at this interval's start
      const int lj = p == 0 ? 0 : s - 1;
      for (int i = threadIdx.x; i < nx; i += NT)
        LAM[((int64_t)b * N + lj) * nx + i] = ws[g.oMu + ((int64_t)b * g.P + p) * nx + i];
    }
    wg::sync();
  }
  for (int j = s; j <= e; ++j) {
    const bool wrap = j == N;
    const double* F = fblk(g, ws, b, j);
    const double* rb = ws + g.oRb + ((int64_t)b * N + (j - 1)) * nu;
    wg::gemv<true>(nx, nu, 1.0, F + off_LS(nx, nu), nu, xv, 0.0, uv, sm);
    wg::sync();
    for (int i = threadIdx.x; i < nu; i += NT) uv[i] = -(uv[i] + rb[i]);
    wg::sync();
    pk_trsv<true>(nu, F, F + off_dR(nx, nu), uv, sm);
    if (SOLVE) {
      const int uj = wrap ? 0 : j;
      for (int i = threadIdx.x; i < nu; i += NT) U[((int64_t)b * N + uj) * nu + i] = uv[i];
      for (int i = threadIdx.x; i < nx; i += NT) X[((int64_t)b * N + (j - 1)) * nx + i] = xv[i];
    }
    if (j < e) {
      wg::gemv<false>(nx, nx, 1.0, mA(g, b, j), nx, xv, 0.0, xn, sm);
      wg::gemv<false>(nx, nu, 1.0, mB(g, b, j), nu, uv, 1.0, xn, sm);
      if (g.f) {
        wg::sync();
        for (int i = threadIdx.x; i < nx; i += NT) xn[i] += vf(g, b, j)[i];
      }
      if (SOLVE) {
        const double* Fn = fblk(g, ws, b, j + 1);
        const double* pn = ws + g.oPv + ((int64_t)b * N + j) * nx;
        pk_trmv<true, false>(nx, Fn + off_LQ(nx, nu), xn, t, sm);
        double* lam = LAM + ((int64_t)b * N + j) * nx;
        vcopy(nx, pn, lam);
        pk_trmv<false, true>(nx, Fn + off_LQ(nx, nu), t, lam, sm);
      }
      vcopy(nx, xn, xv);
    } else if (!SOLVE) {
      // value of the outgoing coupling at the interval's end: B^ u + A^ x
      wg::gemv<false>(nx, nu, 1.0, mB(g, b, wrap ? 0 : j), nu, uv, 0.0, gf, sm);
      if (!wrap) wg::gemv<false>(nx, nx, 1.0, mA(g, b, j), nx, xv, 1.0, gf, sm);
    }
  }
}

// Schur right-hand side of boundary p: g^fwd_{p-1 mod P} + g^bwd_p + f of the boundary's
// constraint (f_{s_p - 1}, or f_0 + A_0 x_init for p = 0).
__global__ void __launch_bounds__(NT, 2) k_pit_rhs(PG g, double* ws) {
  const int b = blockIdx.x, nx = g.nx, P = g.P;
  const double* x0 = vx0(g, b);
  for (int el = threadIdx.x; el < P * nx; el += NT) {
    const int p = el / nx, i = el % nx;
    const int pm = (p + P - 1) % P;
    double v = ws[g.oG + ((int64_t)b * P + pm) * 2 * nx + i] + ws[g.oG + ((int64_t)b * P + p) * 2 * nx + nx + i];
    if (p == 0) {
      if (g.f) v += vf(g, b, 0)[i];
      const double* A0 = mA(g, b, 0) + (int64_t)i * nx;
      for (int c = 0; c < nx; ++c) v = fma(A0[c], x0[c], v);
    } else if (g.f) {
      v += vf(g, b, stage_begin(g, p) - 1)[i];
    }
    ws[g.oRhs + ((int64_t)b * P + p) * nx + i] = v;
  }
}

// Residual rows of stages c*CH .. c*CH + CH - 1 (k = 0..N-1 rows u_k, lam_k; k = 1..N rows x_k):
//   rho_u,k = -r_k - (sym(R_k) u_k + S_k x_k + B_k^T lam_k)            (x_0 = x_init)
//   rho_x,k = -q_k - (S_k^T u_k + sym(Q_k) x_k + A_k^T lam_k - lam_{k-1}) (k < N; k = N: Q_N x_N - lam_{N-1})
//   rho_l,k = -f_k - (A_k x_k + B_k u_k - x_{k+1})
// and the right-hand side entries (-(r_0 + S_0 x_init), -(f_0 + A_0 x_init) for k = 0).  The
// products use the coalesced workgroup matrix-vector routines; the vectors stay in LDS.
constexpr int RCH = 8;
__global__ void __launch_bounds__(NT, 2) k_pit_resid(PG g, const double* X, const double* U, const double* LAM,
                                                     double* ws) {
  extern __shared__ __align__(16) unsigned char smraw[];
  wg::Smem& sm = *reinterpret_cast<wg::Smem*>(smraw);
  __shared__ double tv[3][256];
  const int c = blockIdx.x, b = blockIdx.y, nx = g.nx, nu = g.nu, N = g.N;
  double mr = 0.0, mb = 0.0;
  auto up = [&](double rho, double bv) {
    const double a = fabs(rho), bb = fabs(bv);
    mr = (a > mr || a != a) ? a : mr;
    mb = (bb > mb || bb != bb) ? bb : mb;
  };
  const double* x0 = vx0(g, b);
  for (int k = c * RCH; k < (c + 1) * RCH && k <= N; ++k) {
    const double* xk = k == 0 ? x0 : X + ((int64_t)b * N + (k - 1)) * nx;
    if (k < N) {
      const double* uk = U + ((int64_t)b * N + k) * nu;
      const double* lk = LAM + ((int64_t)b * N + k) * nx;
      const double* Rk = mR(g, b, k);
      const double* Bk = mB(g, b, k);
      // tv0 = sym(R) u + B^T lam, tv1 = S x
      wg::gemv<false>(nu, nu, 0.5, Rk, nu, uk, 0.0, tv[0], sm);
      wg::gemv<true>(nu, nu, 0.5, Rk, nu, uk, 1.0, tv[0], sm);
      wg::gemv<true>(nx, nu, 1.0, Bk, nu, lk, 1.0, tv[0], sm);
      if (g.S) wg::gemv<false>(nu, nx, 1.0, mS(g, b, k), nx, xk, 0.0, tv[1], sm);
      for (int i = threadIdx.x; i < nu; i += NT) {
        const double rk = vr(g, b, k)[i], sx = g.S ? tv[1][i] : 0.0;
        up(-rk - (tv[0][i] + sx), k == 0 ? rk + sx : rk);
      }
      // tv2 = A x (tv1 keeps A x for k = 0), then + B u
      wg::gemv<false>(nx, nx, 1.0, mA(g, b, k), nx, xk, 0.0, tv[2], sm);
      if (k == 0)
        for (int i = threadIdx.x; i < nx; i += NT) tv[1][i] = tv[2][i];
      wg::gemv<false>(nx, nu, 1.0, Bk, nu, uk, 1.0, tv[2], sm);
      const double* xn = X + ((int64_t)b * N + k) * nx;
      for (int i = threadIdx.x; i < nx; i += NT) {
        const double fk = g.f ? vf(g, b, k)[i] : 0.0;
        up(-fk - (tv[2][i] - xn[i]), k == 0 ? fk + tv[1][i] : fk);
      }
    }
    if (k >= 1) {
      const double* Qk = mQ(g, b, k);
      const double* lm = LAM + ((int64_t)b * N + (k - 1)) * nx;
      wg::gemv<false>(nx, nx, 0.5, Qk, nx, xk, 0.0, tv[0], sm);
      wg::gemv<true>(nx, nx, 0.5, Qk, nx, xk, 1.0, tv[0], sm);
      if (k < N) {
        const double* uk = U + ((int64_t)b * N + k) * nu;
        const double* lk = LAM + ((int64_t)b * N + k) * nx;
        if (g.S) wg::gemv<true>(nu, nx, 1.0, mS(g, b, k), nx, uk, 1.0, tv[0], sm);
        wg::gemv<true>(nx, nx, 1.0, mA(g, b, k), nx, lk, 1.0, tv[0], sm);
      }
      for (int i = threadIdx.x; i < nx; i += NT) {
        const double qk = vq(g, b, k)[i];
        up(-qk - (tv[0][i] - lm[i]), qk);
      }
    }
    wg::sync();
  }
  // workgroup maxima, then atomic maxima on the bit patterns (non-negative doubles order as
  // integers; a NaN's pattern is above every number's)
  sm.red[threadIdx.x] = mr;
  __syncthreads();
  for (int st = NT / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      const double o = sm.red[threadIdx.x + st], cur = sm.red[threadIdx.x];
      sm.red[threadIdx.x] = (o > cur || o != o) ? o : cur;
    }
    __syncthreads();
  }
  const double rmax = sm.red[0];
  __syncthreads();
  sm.red[threadIdx.x] = mb;
  __syncthreads();
  for (int st = NT / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      const double o = sm.red[threadIdx.x + st], cur = sm.red[threadIdx.x];
      sm.red[threadIdx.x] = (o > cur || o != o) ? o : cur;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(ws + g.oAcc) + 2 * (int64_t)b;
    atomicMax(acc, (unsigned long long)__double_as_longlong(fabs(rmax)));
    atomicMax(acc + 1, (unsigned long long)__double_as_longlong(fabs(sm.red[0])));
  }
}

__global__ void k_pit_zero_acc(PG g, double* ws) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 2 * g.batch) reinterpret_cast<unsigned long long*>(ws + g.oAcc)[i] = 0ull;
}

__global__ void k_pit_relres(PG g, double* ws, double* rel_res, int32_t* info) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= g.batch) return;
  const unsigned long long* acc = reinterpret_cast<const unsigned long long*>(ws + g.oAcc) + 2 * (int64_t)b;
  const double mr = __longlong_as_double((long long)acc[0]), mb = __longlong_as_double((long long)acc[1]);
  const double rel = mb != mb ? mb : (mb > 0.0 ? mr / mb : mr);
  if (rel_res) rel_res[b] = rel;
  if (info[b] == 0 && !isfinite(rel)) info[b] = LQ_INFO_NONFINITE;
}

__global__ void k_pit_zero_i32(int32_t* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

int check_args(int32_t batch, int32_t N, int32_t nx, int32_t nu, int32_t P, const lq_data* d, void* ws,
               const char* fn) {
  if (batch <= 0 || N <= 0 || nx <= 0 || nu <= 0 || P <= 0)
    return set_error(LQ_EINVAL, "%s: batch, N, nx, nu, P must be positive", fn);
  if (P > N) return set_error(LQ_EINVAL, "%s: P (%d) must not exceed N (%d)", fn, P, N);
  if (nx > 256 || nu > 256 || batch > 65535)
    return set_error(LQ_EUNSUPPORTED, "%s: sizes above the limits (nx <= 256, nu <= 256, batch <= 65535)", fn);
  if (!d || !d->A || !d->B || !d->Q || !d->R || !d->q || !d->r || !d->x0)
    return set_error(LQ_EINVAL, "%s: A, B, Q, R, q, r, x0 are required", fn);
  if (!ws || ((uintptr_t)ws & 255)) return set_error(LQ_EINVAL, "%s: workspace must be non-NULL and 256-byte aligned", fn);
  return LQ_OK;
}

PG with_data(PG g, const lq_data* d) {
  g.A = d->A; g.B = d->B; g.Q = d->Q; g.R = d->R; g.S = d->S; g.q = d->q; g.r = d->r; g.f = d->f; g.x0 = d->x0;
  return g;
}

int rc_of(hipError_t e, const char* fn) {
  if (e != hipSuccess) return set_error(LQ_EHIP, "%s: launch failed: %s", fn, hipGetErrorString(e));
  return LQ_OK;
}

}  // namespace
}  // namespace lq

using namespace lq;

extern "C" size_t lq_pit_workspace_bytes(int32_t batch, int32_t N, int32_t nx, int32_t nu, int32_t P) {
  if (batch <= 0 || N <= 0 || nx <= 0 || nu <= 0 || P <= 0 || P > N) return 0;
  return (size_t)layout(batch, N, nx, nu, P).total * sizeof(double);
}

extern "C" int lq_pit_factor(int32_t batch, int32_t N, int32_t nx, int32_t nu, int32_t P, const lq_data* d,
                             void* ws, int32_t* info, hipStream_t st) {
  clear_error();
  const char* fn = "lq_pit_factor";
  int rc = check_args(batch, N, nx, nu, P, d, ws, fn);
  if (rc) return rc;
  if (!info) return set_error(LQ_EINVAL, "%s: info is required", fn);
  const PG g = with_data(layout(batch, N, nx, nu, P), d);
  double* w = (double*)ws;
  const size_t lds = sizeof(wg::Smem);
  hipError_t e = raise_lds_limit((const void*)k_pit_factor, lds);
  if (e == hipSuccess) e = raise_lds_limit((const void*)k_pit_schur, lds);
  if (e != hipSuccess) return rc_of(e, fn);
  hipLaunchKernelGGL(k_pit_zero_i32, dim3((batch + 255) / 256), dim3(256), 0, st, info, batch);
  hipLaunchKernelGGL(k_pit_factor, dim3(P, batch), dim3(NT), lds, st, g, w, info);
  hipLaunchKernelGGL(k_pit_schur, dim3(P, batch), dim3(NT), lds, st, g, w);
  if ((e = hipGetLastError()) != hipSuccess) return rc_of(e, fn);
  int32_t* sinfo = reinterpret_cast<int32_t*>(w + g.oSinfo);
  rc = lq_bt_cr_factor(batch, P, nx, w + g.oMs, P > 1 ? w + g.oKs : nullptr, w + g.oCR, sinfo, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_pit_merge_info, dim3((batch + 255) / 256), dim3(256), 0, st, g, sinfo, info);
  return rc_of(hipGetLastError(), fn);
}

extern "C" int lq_pit_solve(int32_t batch, int32_t N, int32_t nx, int32_t nu, int32_t P, const lq_data* d, void* ws,
                            double* x, double* u, double* lam, double* rel_res, int32_t* info, hipStream_t st) {
  clear_error();
  const char* fn = "lq_pit_solve";
  int rc = check_args(batch, N, nx, nu, P, d, ws, fn);
  if (rc) return rc;
  if (!x || !u || !lam || !info) return set_error(LQ_EINVAL, "%s: x, u, lam, info are required", fn);
  const PG g = with_data(layout(batch, N, nx, nu, P), d);
  double* w = (double*)ws;
  const size_t lds = sizeof(wg::Smem);
  hipError_t e = hipSuccess;
  for (const void* k : {(const void*)k_pit_bwd<false>, (const void*)k_pit_bwd<true>, (const void*)k_pit_fwd<false>,
                        (const void*)k_pit_fwd<true>, (const void*)k_pit_resid})
    if (e == hipSuccess) e = raise_lds_limit(k, lds);
  if (e != hipSuccess) return rc_of(e, fn);
  const dim3 grid(P, batch);
  hipLaunchKernelGGL(k_pit_bwd<false>, grid, dim3(NT), lds, st, g, w);
  hipLaunchKernelGGL(k_pit_fwd<false>, grid, dim3(NT), lds, st, g, w, x, u, lam);
  hipLaunchKernelGGL(k_pit_rhs, dim3(batch), dim3(NT), 0, st, g, w);
  if ((e = hipGetLastError()) != hipSuccess) return rc_of(e, fn);
  rc = lq_bt_cr_solve(batch, P, nx, w + g.oCR, w + g.oRhs, w + g.oMu, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_pit_bwd<true>, grid, dim3(NT), lds, st, g, w);
  hipLaunchKernelGGL(k_pit_fwd<true>, grid, dim3(NT), lds, st, g, w, x, u, lam);
  hipLaunchKernelGGL(k_pit_zero_acc, dim3((2 * batch + 255) / 256), dim3(256), 0, st, g, w);
  hipLaunchKernelGGL(k_pit_resid, dim3((N + RCH) / RCH, batch), dim3(NT), lds, st, g, x, u, lam, w);
  hipLaunchKernelGGL(k_pit_relres, dim3((batch + 255) / 256), dim3(256), 0, st, g, w, rel_res, info);
  return rc_of(hipGetLastError(), fn);
}
