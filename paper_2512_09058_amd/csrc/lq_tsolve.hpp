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
#pragma once
#include <math.h>

#include <type_traits>

#include "lq_internal.hpp"
#include "lq_tile_factor.hpp"

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

// LDS of the kernel for the padded sizes (doubles): vectors that live across stages, then the
// per-stage staging area (triangles, column partials, block maxima).  The checkpointed kernels
// overlay the staging area with the factor-sweep scratch of the segment recomputation.
__host__ __device__ constexpr int tsolve_vec_doubles(int NXP, int NUP) { return 14 * NXP + 8 * NUP; }
__host__ __device__ constexpr int tsolve_stage_doubles(int W, int NXP, int NUP) {
  return NXP * (NXP + 1) / 2 + NUP * (NUP + 1) / 2 + W * (NXP + NUP) + 2 * W;
}
__host__ __device__ constexpr int tsolve_lds_doubles(int W, int NXP, int NUP) {
  return tsolve_vec_doubles(NXP, NUP) + tsolve_stage_doubles(W, NXP, NUP);
}

// Solve of instance b.  TMAX > 0 (checkpointed plans, a.ckpt = s > 0): the factor region holds
// blocks of stages 0, s, 2s, ... and N plus a segment buffer; the blocks of a segment [k0, k1) are
// recomputed into the buffer from the stored L^Q_k1 (tile factor sweep, TMAX = W wavefronts, TP
// the product type the factors were made with) when a pass first reaches it.
template <int W, int NXP, int NUP, typename TF, int TMAX = 0, typename TP = TF>
__device__ __forceinline__ void tsolve_one(const SolveArgs& a, int b, double* sm) {
  typedef TS<W, NXP, NUP> S;
  static_assert(TMAX == 0 || TMAX == W, "the recomputation uses the solve's wavefronts");
  const Desc D = a.desc[b];
  const int N = D.N, nx = D.nx, nu = D.nu, tid = threadIdx.x, nt = blockDim.x;
  Lanes L;
  L.w = __builtin_amdgcn_readfirstlane(tid >> 6);
  L.lane = tid & 63;
  // LDS: vectors
  double* xc = sm;                          // chain state x_k (correction in mode 1)
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
  // LDS: per-stage staging
  double* stg = sm + tsolve_vec_doubles(NXP, NUP);
  double* LQ = stg;                         // packed L^Q_{k+1}
  double* LR = LQ + NXP * (NXP + 1) / 2;    // packed L^R_k
  double* px = LR + NUP * (NUP + 1) / 2;    // column partials, nx-wide  [W][NXP]
  double* pu = px + W * NXP;                //                   nu-wide  [W][NUP]
  double* red = pu + W * NUP;               // [2 W] wavefront maxima
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
  // factor block of stage k: stored, or (checkpoints) in the segment buffer / a checkpoint slot
  const int sc = TMAX > 0 ? a.ckpt : 0;
  int seg0 = -1;  // first stage of the segment held by the buffer
  auto blk_of = [&](int k) -> const TF* {
    if (sc == 0) return Fi + (int64_t)k * fs;
    if (k >= seg0 && k < seg0 + sc && k < N) return Fi + (ckpt_slots(N, sc) + (k - seg0)) * fs;
    return Fi + ckpt_slot(k, N, sc) * fs;
  };
  // make the segment of stage k (< N) resident
  auto ensure = [&](int k) {
    if constexpr (TMAX > 0) {
      if (sc == 0 || k / sc * sc == seg0) return;
      __shared__ int s_rinfo;
      const int k0 = k / sc * sc, k1 = min(k0 + sc, N);
      TF* seg = (TF*)a.F + D.oF + ckpt_slots(N, sc) * fs;
      auto dst = [&](int kk) -> TF* { return kk >= k0 && kk < k1 ? seg + (int64_t)(kk - k0) * fs : nullptr; };
      const TF* from = k1 < N ? Fi + ckpt_slot(k1, N, sc) * fs : nullptr;
      __syncthreads();
      factor_tile_range<TMAX, TF, TP>(D, a.d, k0, k1, dst, from, nullptr, (unsigned char*)stg, s_rinfo);
      seg0 = k0;
    }
  };
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
      ensure(k);
      const Lanes L = lanes_now();
      const TF* blk = blk_of(k);
      const TF* blk1 = blk_of(k + 1);
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
        mr = nan_max(mr, fabs(rho));
        mb = nan_max(mb, fabs(ri + (k == 0 && Sm ? s0[j] : 0.0)));
        rhu[(int64_t)k * nu + j] = -rho;
      }
      for (int i = tid; i < nx; i += nt) {
        const double fi = rhs_f(k, i);
        const double axu = mode == 0 ? xn[i] - (mode == 0 ? rhs_f(k, i) : 0.0) : al[i];
        const double rho = -fi - (axu - xt1[i]);
        mr = nan_max(mr, fabs(rho));
        mb = nan_max(mb, fabs(fi + (k == 0 ? a0[i] : 0.0)));
        flam[(int64_t)k * nx + i] = -rho;
        if (k > 0) {
          const double qi = rhs_q(k, i);
          const double rho2 = -qi - (ax[i] - ltm[i]);
          mr = nan_max(mr, fabs(rho2));
          mb = nan_max(mb, fabs(qi));
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
        mr = nan_max(mr, fabs(rho));
        mb = nan_max(mb, fabs(qi));
        rhx[(int64_t)N * nx + i] = -rho;
      }
    }
    // workgroup maxima: within each wavefront, then over the W wavefront values
    for (int o = 1; o < 64; o <<= 1) {
      mr = nan_max(mr, __shfl_xor(mr, o));
      mb = nan_max(mb, __shfl_xor(mb, o));
    }
    if (L.lane == 0) {
      red[L.w] = mr;
      red[W + L.w] = mb;
    }
    __syncthreads();
    mr = red[0];
    mb = red[W];
    for (int v = 1; v < W; ++v) {
      mr = nan_max(mr, red[v]);
      mb = nan_max(mb, red[W + v]);
    }
    __syncthreads();
    return rel_of(mr, mb);
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
      ensure(k);
      const Lanes L = lanes_now();
      const TF* blk = blk_of(k);
      const TF* blk1 = blk_of(k + 1);
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

  if (adj) {
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
  }
  // pass sequence, with one call site per pass (the passes are inlined): primal F0 (B F1)*,
  // adjoint B F1 (B F1)*; it counts the corrections after the first forward pass
  const bool want = a.check || a.max_it > 0;
  double rel;
  int it = -1;
  for (;;) {
    const bool first = it < 0;
    if (!first || adj) backward();
    const bool f0 = first && !adj;
    rel = forward(f0 ? 0 : 1, f0 ? rb0 : rb2, f0 ? p0 : p2);
    ++it;
    if (!(want && rel > a.tol && it < a.max_it)) break;
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

}  // namespace
}  // namespace lq
