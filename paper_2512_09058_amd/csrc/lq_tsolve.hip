// Solve kernel for medium and large stage sizes (nx <= 128, nu <= 64): forward rollout with the
// float64 KKT residual fused in, backward correction sweeps and the refinement loop, for the
// primal and the adjoint right-hand side.  The recursions are those of the generic solve kernel
// (sweeps of the block factorisation, eq. opt-cond-ocp-eq); what differs is how a stage's data
// reaches the arithmetic.
//
// One workgroup of W wavefronts per instance (a persistent grid for ragged batches).  Every
// dense stage matrix is read once per pass into registers with a fixed coalesced lane mapping:
// a row is spread over a group of CW consecutive lanes (CW = the padded column count, at most
// 64, two chunks of 64 for 128 columns), 64/CW rows per wavefront instruction, rows dealt round
// robin over the wavefronts.  From the same registers the kernel forms row sums M x (reduced in
// the lane group) and column sums M^T v (reduced across the groups and, through LDS, across the
// wavefronts), so A_k serves both A x_k and A^T lam_k, B_k both B u_k and B^T lam_k, and so on.
// The triangular factors L^Q_{k+1} and L^R_k pass through LDS (their products run over
// triangles).  Per stage the forward chain is: (L^S)^T x, the triangular solve with L^R (one
// wavefront, lane reads), A x + B u; lam_k and the residual rows follow from data already in
// registers.
//
// Float64 arithmetic throughout; factors stored in float32 (mixed mode) are widened on load.
#include <math.h>

#include <type_traits>

#include "lq_internal.hpp"

namespace lq {
namespace {

template <int W, int NXP, int NUP>
struct TS {
  static constexpr int NT = 64 * W;
  static constexpr int XW = NXP >= 64 ? 64 : NXP;  // lanes per row, nx-wide operands
  static constexpr int XC = NXP > 64 ? NXP / 64 : 1;  // column chunks of 64
  static constexpr int XG = 64 / XW;                  // rows per wavefront instruction
  static constexpr int UW = NUP;                      // lanes per row, nu-wide operands
  static constexpr int UG = 64 / UW;
  static constexpr int RXX = (NXP + W * XG - 1) / (W * XG);  // row slots: nx rows, nx wide
  static constexpr int RXU = (NXP + W * UG - 1) / (W * UG);  //            nx rows, nu wide
  static constexpr int RUX = (NUP + W * XG - 1) / (W * XG);  //            nu rows, nx wide
  static constexpr int RUU = (NUP + W * UG - 1) / (W * UG);  //            nu rows, nu wide
};

// A stage matrix in registers: slot t, chunk c of lane (wave w, group q, column c0) holds
// M[(t W + w) G + q][c0 + 64 c].
template <int R, int C, int CW>
struct Frag {
  double v[R][C];
  static constexpr int G = 64 / CW;
};

struct Lanes {
  int w, lane;
};

// Lane coordinates from an opaque copy of the thread index.  Called per stage, so the compiler
// recomputes the per-lane element offsets of the stage loads instead of hoisting all of them out
// of the stage loop (which costs more registers than the fragments themselves).
__device__ __forceinline__ Lanes lanes_now() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  Lanes L;
  L.w = __builtin_amdgcn_readfirstlane(t >> 6);
  L.lane = t & 63;
  return L;
}

template <int R, int C, int CW>
__device__ __forceinline__ int frag_row(const Lanes& L, int W, int t) {
  return (t * W + L.w) * (64 / CW) + L.lane / CW;
}
template <int CW>
__device__ __forceinline__ int frag_col(const Lanes& L, int c) {
  return (L.lane % CW) + 64 * c;
}

// Load rows [0, nr) x columns [0, nc) of the row-major matrix M (leading dimension ld); entries
// outside are zero (addresses are clamped, so every lane issues its loads).
template <int R, int C, int CW, typename T>
__device__ __forceinline__ void frag_load(Frag<R, C, CW>& f, const T* __restrict__ M, int nr, int nc, int ld,
                                          const Lanes& L, int W) {
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int r = frag_row<R, C, CW>(L, W, t);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = frag_col<CW>(L, c);
      const double e = (double)M[(r < nr ? r : nr - 1) * ld + (j < nc ? j : nc - 1)];
      f.v[t][c] = (r < nr && j < nc) ? e : 0.0;
    }
  }
}

__device__ __forceinline__ double xor_sum(double a, int from, int to) {
  for (int o = from; o < to; o <<= 1) a += __shfl_xor(a, o);
  return a;
}

// out(r, (M x)_r) for the rows held; x is a zero-padded LDS vector.
template <int R, int C, int CW, typename F>
__device__ __forceinline__ void frag_rows(const Frag<R, C, CW>& f, const double* x, int nr, const Lanes& L, int W,
                                          F&& out) {
#pragma unroll
  for (int t = 0; t < R; ++t) {
    double p = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) p = fma(f.v[t][c], x[frag_col<CW>(L, c)], p);
    p = xor_sum(p, 1, CW);
    const int r = frag_row<R, C, CW>(L, W, t);
    if ((L.lane % CW) == 0 && r < nr) out(r, p);
  }
}

// acc[c] += sum over the rows r < nr held of M[r][col] v[r].
template <int R, int C, int CW>
__device__ __forceinline__ void frag_cols(const Frag<R, C, CW>& f, const double* v, int nr, double (&acc)[C],
                                          const Lanes& L, int W) {
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int rr = frag_row<R, C, CW>(L, W, t);
    const double vr = rr < nr ? v[rr] : 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = fma(f.v[t][c], vr, acc[c]);
  }
}

// An nr x nr matrix streamed from global memory one row slot at a time (the fragment mapping,
// never resident as a whole): out(r, (M x)_r) for its rows and acc[c] += M[r][col] x_r.
template <int R, int C, int CW, typename F>
__device__ __forceinline__ void stream_sq(const double* __restrict__ M, int nr, const double* x, double (&acc)[C],
                                          const Lanes& L, int W, F&& out) {
#pragma unroll 4
  for (int t = 0; t < R; ++t) {
    const int r = frag_row<R, C, CW>(L, W, t);
    const int rc = r < nr ? r : nr - 1;
    double v[C];
    double p = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = frag_col<CW>(L, c);
      const double e = M[rc * nr + (j < nr ? j : nr - 1)];
      v[c] = (r < nr && j < nr) ? e : 0.0;
      p = fma(v[c], x[j], p);
    }
    p = xor_sum(p, 1, CW);
    if ((L.lane % CW) == 0 && r < nr) out(r, p);
    const double xr = r < nr ? x[r] : 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = fma(v[c], xr, acc[c]);
  }
}

// Column partials of every wavefront into part[w * pst + col]; after the barrier the caller sums
// over the wavefronts (colsum_total).
template <int C, int CW>
__device__ __forceinline__ void colsum_publish(double (&acc)[C], double* part, int pst, const Lanes& L) {
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const double s = xor_sum(acc[c], CW, 64);
    if (L.lane < CW) part[L.w * pst + frag_col<CW>(L, c)] = s;
  }
}
__device__ __forceinline__ double colsum_total(const double* part, int pst, int W, int col) {
  double s = 0.0;
  for (int w = 0; w < W; ++w) s += part[w * pst + col];
  return s;
}

// Packed lower triangle (rows [0, n), row i holds i + 1 entries) into LDS as float64.
template <typename T>
__device__ __forceinline__ void tri_to_lds(const T* __restrict__ P, int n, double* dst) {
  const int tot = n * (n + 1) / 2;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) dst[e] = (double)P[e];
}
__device__ __forceinline__ int tri(int i) { return i * (i + 1) / 2; }

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, l), hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __hiloint2double(hi, lo);
}

// Triangular solves with L^R (packed in LDS, reciprocal diagonal dr): wavefront 0, lane j keeps
// entry j.  TRANS: y = (L^R)^{-T} t, else y = (L^R)^{-1} t.  nu <= 64.
template <bool TRANS>
__device__ __forceinline__ void lr_solve(const double* LR, const double* dr, int nu, const double* t, double* y) {
  if (threadIdx.x >= 64) return;
  const int j = threadIdx.x;
  double a = j < nu ? t[j] : 0.0;
  for (int st = 0; st < nu; ++st) {
    const int i = TRANS ? nu - 1 - st : st;
    const double yi = readlane_d(a, i) * dr[i];
    if (j == 0) y[i] = yi;
    if (TRANS ? j < i : (j > i && j < nu)) a = fma(-(TRANS ? LR[tri(i) + j] : LR[tri(j) + i]), yi, a);
  }
}

template <typename F>
__device__ __forceinline__ void each_instance(int batch, const int32_t* order, int32_t* counter, F&& body) {
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

// LDS doubles of the kernel for the padded sizes.
__host__ __device__ constexpr int tsolve_lds_doubles(int W, int NXP, int NUP) {
  return NXP * (NXP + 1) / 2 + NUP * (NUP + 1) / 2 + W * (NXP + NUP) + 14 * NXP + 8 * NUP + 64 * W;
}

template <int W, int NXP, int NUP, typename TF>
__device__ __forceinline__ void tsolve_one(const SolveArgs& a, int b, double* sm) {
  typedef TS<W, NXP, NUP> S;
  const Desc D = a.desc[b];
  const int N = D.N, nx = D.nx, nu = D.nu, tid = threadIdx.x, nt = blockDim.x;
  Lanes L;
  L.w = __builtin_amdgcn_readfirstlane(tid >> 6);
  L.lane = tid & 63;
  // LDS
  double* LQ = sm;                          // packed L^Q_{k+1}
  double* LR = LQ + NXP * (NXP + 1) / 2;    // packed L^R_k
  double* px = LR + NUP * (NUP + 1) / 2;    // column partials, nx-wide  [W][NXP]
  double* pu = px + W * NXP;                //                   nu-wide  [W][NUP]
  double* xc = pu + W * NUP;                // chain state x_k (correction in mode 1)
  double* xn = xc + NXP;                    // x_{k+1}
  double* ct = xn + NXP;                    // t2 = (L^Q)^T x_{k+1}, then w in the backward pass
  double* xt = ct + NXP;                    // total iterate: x_k
  double* xt1 = xt + NXP;                   //                x_{k+1}
  double* lt = xt1 + NXP;                   //                lam_k
  double* ltm = lt + NXP;                   //                lam_{k-1}
  double* ax = ltm + NXP;                   // residual accumulators (nx rows)
  double* al = ax + NXP;
  double* a0 = al + NXP;                    // A x_init (part of b)
  double* pn = a0 + NXP;                    // p_{k+1} of the backward sweep
  double* fl = pn + NXP;                    // correction right-hand sides
  double* qv = fl + NXP;
  double* xs = qv + NXP;                    // scratch nx
  double* us = xs + NXP;                    // s = rbar + (L^S)^T x, then rhat
  double* uu = us + NUP;                    // u_k (chain)
  double* ut = uu + NUP;                    // total u_k
  double* au = ut + NUP;                    // residual accumulator (nu rows)
  double* s0 = au + NUP;                    // S x_init
  double* dr = s0 + NUP;                    // 1 / diag L^R_k
  double* rv = dr + NUP;                    // correction right-hand side r
  double* yb = rv + NUP;                    // rbar2
  double* red = yb + NUP;                   // [64 W] block maxima
  // problem
  const double* A = a.d.A + D.oA;
  const double* B = a.d.B + D.oB;
  const double* Q = a.d.Q + D.oQ;
  const double* R = a.d.R + D.oR;
  const double* Sm = a.d.S ? a.d.S + D.oS : nullptr;
  const double* q = a.d.q + D.oq;
  const double* r = a.d.r + D.or_;
  const double* f = a.d.f ? a.d.f + D.of : nullptr;
  const double* x0 = a.d.x0 + D.ox0;
  const bool adj = a.rhs == RHS_ADJOINT;
  const double* gx = adj ? a.gx + D.ox : nullptr;
  const double* gu = adj ? a.gu + D.ou : nullptr;
  double *X, *U, *LM;
  if (a.out_is_zb) {
    X = a.x + D.oZB;
    U = X + (int64_t)N * nx;
    LM = U + (int64_t)N * nu;
  } else {
    X = a.x + D.ox;
    U = a.u + D.ou;
    LM = a.lam + D.olam;
  }
  const TF* Fi = (const TF*)a.F + D.oF;
  const int64_t fs = stage_factor_elems(nx, nu);
  const double* rb0 = a.V + D.oV;
  const double* p0 = rb0 + (int64_t)N * nu;
  double* rb2 = a.V2 + D.oV2;
  double* p2 = rb2 + (int64_t)N * nu;
  double* flam = rb2 + v2_flam(N, nx, nu);
  double* rhu = rb2 + v2_rhou(N, nx, nu);   // correction right-hand side r = -rho_u
  double* rhx = rb2 + v2_rhox(N, nx, nu);   // correction right-hand side q = -rho_x (k = 1..N)
  // right-hand side of the system being solved: (r, q, f, x_init), adjoint (-gu, -gx, 0, 0)
  auto rhs_r = [&](int k, int i) { return adj ? -gu[(int64_t)k * nu + i] : r[(int64_t)k * nu + i]; };
  auto rhs_q = [&](int k, int i) { return adj ? -gx[(int64_t)(k - 1) * nx + i] : q[(int64_t)k * nx + i]; };
  auto rhs_f = [&](int k, int i) { return (!adj && f) ? f[(int64_t)k * nx + i] : 0.0; };
  auto rhs_x0 = [&](int i) { return adj ? 0.0 : x0[i]; };

  // zero padding of every LDS vector
  for (int i = tid; i < 14 * NXP + 8 * NUP; i += nt) xc[i] = 0.0;
  __syncthreads();

  // ---- forward rollout (mode 0: z = result, mode 1: z += correction) with the residual of the
  // updated iterate: correction right-hand sides for a following backward pass, returns rel_res.
  auto forward = [&](int mode, const double* rbv, const double* pvv) -> double {
    double mr = 0.0, mb = 0.0;
    for (int i = tid; i < nx; i += nt) {
      xc[i] = mode == 0 ? rhs_x0(i) : 0.0;
      xt[i] = rhs_x0(i);
    }
    __syncthreads();
    for (int k = 0; k < N; ++k) {
      const Lanes L = lanes_now();
      const TF* blk = Fi + (int64_t)k * fs;
      const TF* blk1 = Fi + (int64_t)(k + 1) * fs;
      const double* Ak = A + (int64_t)k * nx * nx;
      const double* Bk = B + (int64_t)k * nx * nu;
      // stage data into registers (the residual's Q, R, S too) and the triangles into LDS
      Frag<S::RXU, 1, S::UW> fLS, fB;
      Frag<S::RXX, S::XC, S::XW> fA;
      Frag<S::RUU, 1, S::UW> fR;
      Frag<S::RUX, S::XC, S::XW> fS;
      frag_load(fLS, blk + off_LS(nx, nu), nx, nu, nu, L, W);
      frag_load(fA, Ak, nx, nx, nx, L, W);
      frag_load(fB, Bk, nx, nu, nu, L, W);
      frag_load(fR, R + (int64_t)k * nu * nu, nu, nu, nu, L, W);
      if (Sm) frag_load(fS, Sm + (int64_t)k * nu * nx, nu, nx, nx, L, W);
      tri_to_lds(blk, nu, LR);
      tri_to_lds(blk1 + off_LQ(nx, nu), nx, LQ);
      for (int j = tid; j < nu; j += nt) {
        dr[j] = (double)blk[off_dR(nx, nu) + j];
        us[j] = rbv[(int64_t)k * nu + j];
      }
      // s = rbar_k + (L^S_k)^T x_k
      {
        double acc[1] = {0.0};
        frag_cols(fLS, xc, nx, acc, L, W);
        colsum_publish<1, S::UW>(acc, pu, NUP, L);
      }
      __syncthreads();
      for (int j = tid; j < nu; j += nt) us[j] += colsum_total(pu, NUP, W, j);
      __syncthreads();
      // u_k = -(L^R_k)^{-T} s
      lr_solve<true>(LR, dr, nu, us, uu);
      __syncthreads();
      for (int j = tid; j < nu; j += nt) {
        const double du = -uu[j];
        uu[j] = du;
        const double tot = mode == 0 ? du : U[(int64_t)k * nu + j] + du;
        ut[j] = tot;
        U[(int64_t)k * nu + j] = tot;
      }
      for (int i = tid; i < nx; i += nt) xn[i] = mode == 0 ? rhs_f(k, i) : flam[(int64_t)k * nx + i];
      __syncthreads();
      // x_{k+1} = A x_k + B u_k + f_k (chain); A x_k + B u_k of the total iterate (residual)
      frag_rows(fA, xc, nx, L, W, [&](int i, double s) { xn[i] += s; });
      if (mode != 0) frag_rows(fA, xt, nx, L, W, [&](int i, double s) { al[i] = s; });
      if (k == 0) frag_rows(fA, xt, nx, L, W, [&](int i, double s) { a0[i] = s; });
      __syncthreads();
      frag_rows(fB, uu, nx, L, W, [&](int i, double s) { xn[i] += s; });
      __syncthreads();
      if (mode != 0) frag_rows(fB, ut, nx, L, W, [&](int i, double s) { al[i] += s; });
      for (int i = tid; i < nx; i += nt) {
        const double tot = mode == 0 ? xn[i] : X[(int64_t)k * nx + i] + xn[i];
        xt1[i] = tot;
        X[(int64_t)k * nx + i] = tot;
      }
      __syncthreads();
      // lam_k = L^Q_{k+1} (L^Q_{k+1})^T x_{k+1} + p_{k+1}
      for (int j = tid; j < nx; j += nt) {
        double s = 0.0;
        for (int i = j; i < nx; ++i) s = fma(LQ[tri(i) + j], xn[i], s);
        ct[j] = s;
      }
      __syncthreads();
      {
        // row sums over the triangle with groups of XW lanes per row
        const int g = S::XW, sub = L.lane % g, per = nt / g;
        for (int i0 = 0; i0 < nx; i0 += per) {
          const int i = i0 + tid / g;
          double s = 0.0;
          if (i < nx)
            for (int j = sub; j <= i; j += g) s = fma(LQ[tri(i) + j], ct[j], s);
          s = xor_sum(s, 1, g);
          if (sub == 0 && i < nx) {
            const double l = pvv[(int64_t)(k + 1) * nx + i] + s;
            const double tot = mode == 0 ? l : LM[(int64_t)k * nx + i] + l;
            lt[i] = tot;
            LM[(int64_t)k * nx + i] = tot;
          }
        }
      }
      __syncthreads();
      // residual rows of stage k (total iterate)
      {
        double cx[S::XC];
#pragma unroll
        for (int c = 0; c < S::XC; ++c) cx[c] = 0.0;
        double cu[1] = {0.0};
        frag_cols(fA, lt, nx, cx, L, W);      // A^T lam_k
        frag_cols(fB, lt, nx, cu, L, W);      // B^T lam_k
        if (k > 0) {
          double hq[S::XC];
#pragma unroll
          for (int c = 0; c < S::XC; ++c) hq[c] = 0.0;
          // Q_k x_k (rows, into xs) and Q_k^T x_k (columns), streamed
          stream_sq<S::RXX, S::XC, S::XW>(Q + (int64_t)k * nx * nx, nx, xt, hq, L, W,
                                          [&](int i, double v) { xs[i] = v; });
#pragma unroll
          for (int c = 0; c < S::XC; ++c) cx[c] = fma(0.5, hq[c], cx[c]);
        }
        double hr[1] = {0.0};
        frag_cols(fR, ut, nu, hr, L, W);      // R^T u_k
        cu[0] = fma(0.5, hr[0], cu[0]);
        if (Sm) frag_cols(fS, ut, nu, cx, L, W);  // S^T u_k
        colsum_publish<S::XC, S::XW>(cx, px, NXP, L);
        colsum_publish<1, S::UW>(cu, pu, NUP, L);
      }
      __syncthreads();
      for (int i = tid; i < nx; i += nt) ax[i] = colsum_total(px, NXP, W, i) + (k > 0 ? 0.5 * xs[i] : 0.0);
      for (int j = tid; j < nu; j += nt) au[j] = colsum_total(pu, NUP, W, j);
      __syncthreads();
      frag_rows(fR, ut, nu, L, W, [&](int i, double s) { au[i] = fma(0.5, s, au[i]); });
      __syncthreads();
      if (Sm) frag_rows(fS, xt, nu, L, W, [&](int i, double s) { au[i] += s; if (k == 0) s0[i] = s; });
      __syncthreads();
      for (int j = tid; j < nu; j += nt) {
        const double ri = rhs_r(k, j);
        const double rho = -ri - au[j];
        mr = fmax(mr, fabs(rho));
        mb = fmax(mb, fabs(ri + (k == 0 && Sm ? s0[j] : 0.0)));
        rhu[(int64_t)k * nu + j] = -rho;
      }
      for (int i = tid; i < nx; i += nt) {
        const double fi = rhs_f(k, i);
        const double axu = mode == 0 ? xn[i] - (mode == 0 ? rhs_f(k, i) : 0.0) : al[i];
        const double rho = -fi - (axu - xt1[i]);
        mr = fmax(mr, fabs(rho));
        mb = fmax(mb, fabs(fi + (k == 0 ? a0[i] : 0.0)));
        flam[(int64_t)k * nx + i] = -rho;
        if (k > 0) {
          const double qi = rhs_q(k, i);
          const double rho2 = -qi - (ax[i] - ltm[i]);
          mr = fmax(mr, fabs(rho2));
          mb = fmax(mb, fabs(qi));
          rhx[(int64_t)k * nx + i] = -rho2;
        }
      }
      __syncthreads();
      for (int i = tid; i < nx; i += nt) {
        xc[i] = xn[i];
        xt[i] = xt1[i];
        ltm[i] = lt[i];
      }
      __syncthreads();
    }
    // stage N rows: rho_x,N = -q_N - (Q_N,sym x_N - lam_{N-1})
    {
      const Lanes L = lanes_now();
      double cx[S::XC];
#pragma unroll
      for (int c = 0; c < S::XC; ++c) cx[c] = 0.0;
      stream_sq<S::RXX, S::XC, S::XW>(Q + (int64_t)N * nx * nx, nx, xt, cx, L, W, [&](int i, double v) { xs[i] = v; });
      colsum_publish<S::XC, S::XW>(cx, px, NXP, L);
      __syncthreads();
      for (int i = tid; i < nx; i += nt) ax[i] = 0.5 * (colsum_total(px, NXP, W, i) + xs[i]);
      __syncthreads();
      for (int i = tid; i < nx; i += nt) {
        const double qi = rhs_q(N, i);
        const double rho = -qi - (ax[i] - ltm[i]);
        mr = fmax(mr, fabs(rho));
        mb = fmax(mb, fabs(qi));
        rhx[(int64_t)N * nx + i] = -rho;
      }
    }
    // block maxima
    red[tid] = mr;
    __syncthreads();
    for (int s2 = nt / 2; s2 > 0; s2 >>= 1) {
      if (tid < s2) red[tid] = fmax(red[tid], red[tid + s2]);
      __syncthreads();
    }
    mr = red[0];
    __syncthreads();
    red[tid] = mb;
    __syncthreads();
    for (int s2 = nt / 2; s2 > 0; s2 >>= 1) {
      if (tid < s2) red[tid] = fmax(red[tid], red[tid + s2]);
      __syncthreads();
    }
    mb = red[0];
    __syncthreads();
    return mb > 0.0 ? mr / mb : mr;
  };

  // ---- backward sweep of the stored correction right-hand side (r, q, f) = (rhu, rhx, flam),
  // x_init = 0: rbar2_k = (L^R_k)^{-1}(r_k + B_k^T w), p2_k = q_k + A_k^T w - L^S_k rbar2_k,
  // w = L^Q_{k+1} (L^Q_{k+1})^T f_k + p2_{k+1}, p2_N = q_N.
  auto backward = [&]() {
    for (int i = tid; i < nx; i += nt) {
      const double v = rhx[(int64_t)N * nx + i];
      pn[i] = v;
      p2[(int64_t)N * nx + i] = v;
    }
    __syncthreads();
    for (int k = N - 1; k >= 0; --k) {
      const Lanes L = lanes_now();
      const TF* blk = Fi + (int64_t)k * fs;
      const TF* blk1 = Fi + (int64_t)(k + 1) * fs;
      Frag<S::RXU, 1, S::UW> fLS, fB;
      Frag<S::RXX, S::XC, S::XW> fA;
      frag_load(fB, B + (int64_t)k * nx * nu, nx, nu, nu, L, W);
      frag_load(fA, A + (int64_t)k * nx * nx, nx, nx, nx, L, W);
      frag_load(fLS, blk + off_LS(nx, nu), nx, nu, nu, L, W);
      tri_to_lds(blk1 + off_LQ(nx, nu), nx, LQ);
      tri_to_lds(blk, nu, LR);
      for (int i = tid; i < nx; i += nt) fl[i] = flam[(int64_t)k * nx + i];
      for (int j = tid; j < nu; j += nt) {
        dr[j] = (double)blk[off_dR(nx, nu) + j];
        rv[j] = rhu[(int64_t)k * nu + j];
      }
      __syncthreads();
      // w = L^Q (L^Q^T f) + p2_{k+1}
      for (int j = tid; j < nx; j += nt) {
        double s = 0.0;
        for (int i = j; i < nx; ++i) s = fma(LQ[tri(i) + j], fl[i], s);
        xs[j] = s;
      }
      __syncthreads();
      {
        const int g = S::XW, sub = L.lane % g, per = nt / g;
        for (int i0 = 0; i0 < nx; i0 += per) {
          const int i = i0 + tid / g;
          double s = 0.0;
          if (i < nx)
            for (int j = sub; j <= i; j += g) s = fma(LQ[tri(i) + j], xs[j], s);
          s = xor_sum(s, 1, g);
          if (sub == 0 && i < nx) ct[i] = pn[i] + s;
        }
      }
      __syncthreads();
      // (rhat, qhat) = (r, q) + [B A]^T w
      {
        double cx[S::XC];
#pragma unroll
        for (int c = 0; c < S::XC; ++c) cx[c] = 0.0;
        double cu[1] = {0.0};
        frag_cols(fA, ct, nx, cx, L, W);
        frag_cols(fB, ct, nx, cu, L, W);
        colsum_publish<S::XC, S::XW>(cx, px, NXP, L);
        colsum_publish<1, S::UW>(cu, pu, NUP, L);
      }
      __syncthreads();
      for (int j = tid; j < nu; j += nt) us[j] = rv[j] + colsum_total(pu, NUP, W, j);
      for (int i = tid; i < nx; i += nt) qv[i] = (k > 0 ? rhx[(int64_t)k * nx + i] : 0.0) + colsum_total(px, NXP, W, i);
      __syncthreads();
      // rbar2 = (L^R)^{-1} rhat
      lr_solve<false>(LR, dr, nu, us, yb);
      __syncthreads();
      for (int j = tid; j < nu; j += nt) rb2[(int64_t)k * nu + j] = yb[j];
      // p2_k = qhat - L^S rbar2
      if (k > 0) {
        frag_rows(fLS, yb, nx, L, W, [&](int i, double s) {
          const double v = qv[i] - s;
          pn[i] = v;
          p2[(int64_t)k * nx + i] = v;
        });
      }
      __syncthreads();
    }
  };

  double rel;
  int it = 0;
  if (!adj) {
    rel = forward(0, rb0, p0);
  } else {
    // zero iterate: the correction right-hand side is the system's own (r, q, f) = (-gu, -gx, 0)
    for (int k = 0; k < N; ++k) {
      for (int j = tid; j < nu; j += nt) {
        rhu[(int64_t)k * nu + j] = rhs_r(k, j);
        U[(int64_t)k * nu + j] = 0.0;
      }
      for (int i = tid; i < nx; i += nt) {
        flam[(int64_t)k * nx + i] = 0.0;
        X[(int64_t)k * nx + i] = 0.0;
        LM[(int64_t)k * nx + i] = 0.0;
        rhx[(int64_t)(k + 1) * nx + i] = rhs_q(k + 1, i);
      }
    }
    __syncthreads();
    backward();
    rel = forward(1, rb2, p2);
  }
  const bool want = a.check || a.max_it > 0;
  while (want && rel > a.tol && it < a.max_it) {
    backward();
    rel = forward(1, rb2, p2);
    ++it;
  }
  if (tid == 0) {
    if (a.rel_res) a.rel_res[b] = rel;
    if (a.iters) a.iters[b] = it;
    if (a.info) {
      const int cur = a.info[b];
      if (cur <= 0) {
        int code = 0;
        if (!isfinite(rel)) code = LQ_INFO_NONFINITE;
        else if (a.max_it > 0 && rel > a.tol) code = LQ_INFO_NOT_CONVERGED;
        else if (cur == LQ_INFO_NONFINITE) code = cur;
        a.info[b] = code;
      }
    }
  }
  __syncthreads();
}

template <int W, int NXP, int NUP, typename TF>
__global__ void __launch_bounds__(64 * W) k_solve_tile(SolveArgs a, const int32_t* __restrict__ order,
                                                       int32_t* counter) {
  extern __shared__ double sm_ts[];
  each_instance(a.batch, order, counter, [&](int b) { tsolve_one<W, NXP, NUP, TF>(a, b, sm_ts); });
}

__global__ void k_reset_counter_ts(int32_t* c) {
  if (threadIdx.x == 0) c[0] = 0;
}

// Wavefronts per workgroup for the padded state size.
constexpr int ts_waves(int NXP) { return NXP <= 32 ? 2 : NXP <= 64 ? 4 : 8; }

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
  return hipFuncSetAttribute(ts_kernel(NXP, NUP, mode == LQ_F64), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)tsolve_lds_bytes(NXP, NUP));
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
