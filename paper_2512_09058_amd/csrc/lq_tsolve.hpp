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
template <bool ORD, int R, int C, int CW, typename T>
__device__ __forceinline__ void frag_load(Frag<R, C, CW>& f, const T* __restrict__ M, int nr, int nc, int ld,
                                          const Lanes& L, int W) {
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int r = frag_row<R, C, CW>(L, W, t);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = frag_col<CW>(L, c);
      const double e = (double)M[(uint32_t)((r < nr ? r : nr - 1) * ld + (j < nc ? j : nc - 1))];
      f.v[t][c] = keep_if<ORD>(r < nr && j < nc, e);
    }
  }
}

// Lane reductions without LDS-unit shuffles: DPP moves inside rows of 16 lanes (quad swaps, then
// the half-row and row mirrors, which pair each lane with one holding the other half's partial
// sum), then the row-pair and half-wave swaps of v_permlane16/32_swap.  lane_sum<F, T> sums over
// the lanes that differ only in the index bits from F up to T (F, T powers of two; the mirror
// steps need F = 1 when T > 4).  Every lane ends with the same value (each step adds its own
// partial and its partner's, a commutative pair).  Called with all 64 lanes active.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  return __longlong_as_double(__builtin_amdgcn_update_dpp(0LL, __double_as_longlong(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ double swap_sum16(double v) {
  const unsigned lo = (unsigned)__double_as_longlong(v), hi = (unsigned)(__double_as_longlong(v) >> 32);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
__device__ __forceinline__ double swap_sum32(double v) {
  const unsigned lo = (unsigned)__double_as_longlong(v), hi = (unsigned)(__double_as_longlong(v) >> 32);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
template <int F, int T>
__device__ __forceinline__ double lane_sum(double v) {
  static_assert(F == 1 || F >= 16 || T <= 4, "mirror steps need the lower lanes reduced");
  if constexpr (F <= 1 && T > 1) v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  if constexpr (F <= 2 && T > 2) v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  if constexpr (F <= 4 && T > 4) v += dpp_mov<0x141>(v);  // row_half_mirror
  if constexpr (F <= 8 && T > 8) v += dpp_mov<0x140>(v);  // row_mirror
  if constexpr (F <= 16 && T > 16) v = swap_sum16(v);
  if constexpr (F <= 32 && T > 32) v = swap_sum32(v);
  return v;
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
    p = lane_sum<1, CW>(p);
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
      const double e = M[(uint32_t)(rc * nr + (j < nr ? j : nr - 1))];
      v[c] = keep_if<true>(r < nr && j < nr, e);  // (used at nx = 128 only)
      p = fma(v[c], x[j], p);
    }
    p = lane_sum<1, CW>(p);
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
    const double s = lane_sum<CW, 64>(acc[c]);
    if (L.lane < CW) part[L.w * pst + frag_col<CW>(L, c)] = s;
  }
}
__device__ __forceinline__ double colsum_total(const double* part, int pst, int W, int col) {
  double s = 0.0;
  for (int w = 0; w < W; ++w) s += part[w * pst + col];
  return s;
}

// Packed lower triangle (rows [0, n), row i holds i + 1 entries) into LDS as float64 by NT
// threads, CH loads per thread in flight per chunk (all issued before the first store).
template <int NT, int CH, typename T>
__device__ __forceinline__ void tri_to_lds(const T* __restrict__ P, int n, double* dst) {
  const int tot = n * (n + 1) / 2;
  for (int e0 = 0; e0 < tot; e0 += CH * NT) {
    double v[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int e = e0 + (int)threadIdx.x + c * NT;
      v[c] = (double)P[(uint32_t)(e < tot ? e : tot - 1)];
    }
    // every lane stores (the ones past the end again the last entry, with its value), so that the
    // loads are not sunk into a conditional store, where each would wait for itself
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int e = e0 + (int)threadIdx.x + c * NT;
      dst[e < tot ? e : tot - 1] = v[c];
    }
  }
}
// Loads per thread per chunk for a padded triangle of order NP (at most 8).
__host__ __device__ constexpr int tri_chunk(int NP, int NT) {
  return (NP * (NP + 1) / 2 + NT - 1) / NT < 8 ? (NP * (NP + 1) / 2 + NT - 1) / NT : 8;
}
// A packed lower triangle of order n as a dense fragment (zero above the diagonal and outside).
template <bool ORD, int R, int C, int CW, typename T>
__device__ __forceinline__ void frag_load_tri(Frag<R, C, CW>& f, const T* __restrict__ P, int n, const Lanes& L,
                                              int W) {
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int r = frag_row<R, C, CW>(L, W, t);
    const int rc = r < n ? r : n - 1;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = frag_col<CW>(L, c);
      const double e = (double)P[(uint32_t)(rc * (rc + 1) / 2 + (j <= rc ? j : rc))];
      f.v[t][c] = keep_if<ORD>(r < n && j <= r, e);
    }
  }
}
__device__ __forceinline__ int tri(int i) { return i * (i + 1) / 2; }

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, l), hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __hiloint2double(hi, lo);
}

// Triangular solves with L^R (packed in LDS, reciprocal diagonal dr zero-padded to NUP):
// wavefront 0, lane j keeps entry j.  TRANS: y = (L^R)^{-T} t, else y = (L^R)^{-1} t.  Unrolled
// over the padded order, so the LDS reads of L^R do not wait on the substitution chain; steps
// beyond nu leave zeros (their entries of t and dr are zero).
template <bool TRANS, int NUP>
__device__ __forceinline__ void lr_solve(const double* LR, const double* dr, int nu, const double* t, double* y) {
  if (threadIdx.x >= 64) return;
  const int j = threadIdx.x;
  double a = j < nu ? t[j] : 0.0;
  const int last = tri(nu) - 1;
#pragma unroll
  for (int st = 0; st < NUP; ++st) {
    const int i = TRANS ? NUP - 1 - st : st;
    const bool use = TRANS ? j < i : (j > i && j < nu);
    const int e = TRANS ? tri(i) + j : tri(j) + i;
    const double l = LR[e < last ? e : last];
    const double yi = readlane_d(a, i) * dr[i];
    if (j == 0) y[i] = yi;
    if (use && i < nu) a = fma(-l, yi, a);
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
__host__ __device__ constexpr int tsolve_vec_doubles(int NXP, int NUP) { return 14 * NXP + 7 * NUP; }
__host__ __device__ constexpr int tsolve_stage_doubles(int W, int NXP, int NUP) {
  return (NXP <= 64 ? 0 : NXP * (NXP + 1) / 2) + NUP * (NUP + 1) / 2 + W * (NXP + NUP) + 2 * W;
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
  // loads masked with the ordered keep_if where registers are short (see keep_if)
  constexpr bool ORD = TMAX > 0 || NXP > 64;
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
  double* yb = dr + NUP;                    // rbar2
  // L^Q_{k+1} as a register fragment up to NXP = 64 (beyond, through LDS)
  constexpr bool LQREG = NXP <= 64;
  // LDS: per-stage staging
  double* stg = sm + tsolve_vec_doubles(NXP, NUP);
  double* LQ = stg;                         // packed L^Q_{k+1} (NXP > 64)
  double* LR = LQ + (LQREG ? 0 : NXP * (NXP + 1) / 2);  // packed L^R_k
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
      factor_tile_range<TMAX, TF, TP, true>(D, a.d, k0, k1, dst, from, nullptr, (unsigned char*)stg, s_rinfo);
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
  // (the stage loops read them unconditionally from clamped indices, sign and presence at use)
  const double* r_src = adj ? gu : r;
  const double* q_src = adj ? gx - nx : q;  // row k of the adjoint's q is gx row k - 1
  const double* f_src = (!adj && f) ? f : q;
  const double rhs_sign = adj ? -1.0 : 1.0;
  const bool has_f = !adj && f;
  auto rhs_r = [&](int k, int i) { return adj ? -gu[(int64_t)k * nu + i] : r[(int64_t)k * nu + i]; };
  auto rhs_q = [&](int k, int i) { return adj ? -gx[(int64_t)(k - 1) * nx + i] : q[(int64_t)k * nx + i]; };
  auto rhs_f = [&](int k, int i) { return (!adj && f) ? f[(int64_t)k * nx + i] : 0.0; };
  auto rhs_x0 = [&](int i) { return adj ? 0.0 : x0[i]; };

  // products with the packed triangle LQ in LDS (the path beyond NXP = 64), groups of XW lanes
  // per column / row: out[j] = sum_{i >= j} LQ[i][j] x[i], then emit(i, sum_{j <= i} LQ[i][j] y[j])
  auto tri_cols_lds = [&](const double* T, const double* x, int n, double* out, const Lanes& L) {
    const int g = S::XW, sub = L.lane % g, per = nt / g;
    for (int j0 = 0; j0 < n; j0 += per) {
      const int j = j0 + tid / g;
      double v = 0.0;
      if (j < n)
        for (int i = j + sub; i < n; i += g) v = fma(T[tri(i) + j], x[i], v);
      v = lane_sum<1, S::XW>(v);
      if (sub == 0 && j < n) out[j] = v;
    }
  };
  auto tri_rows_lds = [&](const double* T, const double* y, int n, const Lanes& L, auto&& emit) {
    const int g = S::XW, sub = L.lane % g, per = nt / g;
    for (int i0 = 0; i0 < n; i0 += per) {
      const int i = i0 + tid / g;
      double v = 0.0;
      if (i < n)
        for (int j = sub; j <= i; j += g) v = fma(T[tri(i) + j], y[j], v);
      v = lane_sum<1, S::XW>(v);
      if (sub == 0 && i < n) emit(i, v);
    }
  };

  // zero padding of every LDS vector
  for (int i = tid; i < tsolve_vec_doubles(NXP, NUP); i += nt) xc[i] = 0.0;
  __syncthreads();

  // Every global read of a stage is issued at the stage's start, before its first barrier, and
  // consumed later, so that a stage waits for one memory round trip instead of one per use
  // (barriers do not wait for outstanding global loads).  Thread t holds entry t of the stage's
  // vectors (nt >= NXP >= nx, nu).
  const bool rx = tid < nx, ru = tid < nu;

  // ---- forward rollout (mode 0: z = result, mode 1: z += correction) with, when `res`, the
  // residual of the updated iterate: correction right-hand sides for a following backward pass,
  // returns rel_res (NaN without `res`, which only a first pass with no refinement and no
  // certificate asked for takes).
  auto forward = [&](int mode, const double* rbv, const double* pvv, bool res) -> double {
    double mr = 0.0, mb = 0.0;
    if (rx) {
      xc[tid] = mode == 0 ? rhs_x0(tid) : 0.0;
      xt[tid] = rhs_x0(tid);
    }
    __syncthreads();
    for (int k = 0; k < N; ++k) {
      ensure(k);
      const Lanes L = lanes_now();
      const TF* blk = blk_of(k);
      const TF* blk1 = blk_of(k + 1);
      const double* Ak = A + (int64_t)k * nx * nx;
      const double* Bk = B + (int64_t)k * nx * nu;
      const double* Qk = Q + (int64_t)k * nx * nx;
      // ---- reads of the stage: Q_k first (its products with the known x_k come first), then the
      // vectors, the other stage matrices into registers and the triangles into LDS
      Frag<(NXP <= 64 ? S::RXX : 1), S::XC, S::XW> fQ;
      if constexpr (NXP <= 64) {
        if (res && k > 0) frag_load<ORD>(fQ, Qk, nx, nx, nx, L, W);
      }
      // vectors: unconditional loads from clamped indices (entries past nx / nu are never used)
      const int iu = ru ? tid : nu - 1, ix = rx ? tid : nx - 1;
      const double v_rb = rbv[(int64_t)k * nu + iu];
      const double v_dr = (double)blk[off_dR(nx, nu) + iu];
      const double v_U0 = U[(int64_t)k * nu + iu];
      const double v_r = rhs_sign * r_src[(int64_t)k * nu + iu];
      const double v_f = keep_if<ORD>(has_f, f_src[(int64_t)k * nx + ix]);
      const double v_fl0 = flam[(int64_t)k * nx + ix];
      const double v_X0 = X[(int64_t)k * nx + ix];
      const double v_LM0 = LM[(int64_t)k * nx + ix];
      const double v_p = pvv[(int64_t)(k + 1) * nx + ix];
      const double v_q = rhs_sign * q_src[(int64_t)(k > 0 ? k : 1) * nx + ix];
      Frag<S::RXU, 1, S::UW> fLS, fB;
      Frag<S::RXX, S::XC, S::XW> fA;
      Frag<S::RUU, 1, S::UW> fR;
      Frag<S::RUX, S::XC, S::XW> fS;
      frag_load<ORD>(fLS, blk + off_LS(nx, nu), nx, nu, nu, L, W);
      frag_load<ORD>(fA, Ak, nx, nx, nx, L, W);
      frag_load<ORD>(fB, Bk, nx, nu, nu, L, W);
      if (res) frag_load<ORD>(fR, R + (int64_t)k * nu * nu, nu, nu, nu, L, W);
      if (res && Sm) frag_load<ORD>(fS, Sm + (int64_t)k * nu * nx, nu, nx, nx, L, W);
      tri_to_lds<S::NT, tri_chunk(NUP, S::NT)>(blk, nu, LR);
      if constexpr (!LQREG) tri_to_lds<S::NT, tri_chunk(NXP, S::NT)>(blk1 + off_LQ(nx, nu), nx, LQ);
      // Q_k x_k (rows, into xs) and Q_k^T x_k (columns, hq) of the total iterate, k >= 1
      double hq[S::XC];
#pragma unroll
      for (int c = 0; c < S::XC; ++c) hq[c] = 0.0;
      if (res && k > 0) {
        if constexpr (NXP <= 64) {
          frag_rows(fQ, xt, nx, L, W, [&](int i, double v) { xs[i] = v; });
          frag_cols(fQ, xt, nx, hq, L, W);
        } else {
          stream_sq<S::RXX, S::XC, S::XW>(Qk, nx, xt, hq, L, W, [&](int i, double v) { xs[i] = v; });
        }
      }
      if (ru) {
        dr[tid] = v_dr;
        us[tid] = v_rb;
      }
      // s = rbar_k + (L^S_k)^T x_k
      {
        double acc[1] = {0.0};
        frag_cols(fLS, xc, nx, acc, L, W);
        colsum_publish<1, S::UW>(acc, pu, NUP, L);
      }
      // L^Q_{k+1} into registers (L^S_k is dead; the load completes behind the x-chain)
      Frag<(LQREG ? S::RXX : 1), S::XC, S::XW> fLQ;
      if constexpr (LQREG) frag_load_tri<ORD>(fLQ, blk1 + off_LQ(nx, nu), nx, L, W);
      __syncthreads();
      if (ru) us[tid] += colsum_total(pu, NUP, W, tid);
      __syncthreads();
      // u_k = -(L^R_k)^{-T} s
      lr_solve<true, NUP>(LR, dr, nu, us, uu);
      __syncthreads();
      if (ru) {
        const double du = -uu[tid];
        uu[tid] = du;
        const double tot = mode == 0 ? du : v_U0 + du;
        ut[tid] = tot;
        U[(int64_t)k * nu + tid] = tot;
      }
      if (rx) xn[tid] = mode == 0 ? v_f : v_fl0;
      __syncthreads();
      // x_{k+1} = A x_k + B u_k + f_k (chain); A x_k + B u_k of the total iterate (residual)
      frag_rows(fA, xc, nx, L, W, [&](int i, double v) { xn[i] += v; });
      if (mode != 0) frag_rows(fA, xt, nx, L, W, [&](int i, double v) { al[i] = v; });
      if (res && k == 0) frag_rows(fA, xt, nx, L, W, [&](int i, double v) { a0[i] = v; });
      __syncthreads();
      frag_rows(fB, uu, nx, L, W, [&](int i, double v) { xn[i] += v; });
      __syncthreads();
      if (mode != 0) frag_rows(fB, ut, nx, L, W, [&](int i, double v) { al[i] += v; });
      if (rx) {
        const double tot = mode == 0 ? xn[tid] : v_X0 + xn[tid];
        xt1[tid] = tot;
        X[(int64_t)k * nx + tid] = tot;
      }
      __syncthreads();
      // lam_k = L^Q_{k+1} (L^Q_{k+1})^T x_{k+1} + p_{k+1}
      if constexpr (LQREG) {
        {
          double cq[S::XC];
#pragma unroll
          for (int c = 0; c < S::XC; ++c) cq[c] = 0.0;
          frag_cols(fLQ, xn, nx, cq, L, W);
          colsum_publish<S::XC, S::XW>(cq, px, NXP, L);
        }
        __syncthreads();
        if (rx) ct[tid] = colsum_total(px, NXP, W, tid);
        __syncthreads();
        frag_rows(fLQ, ct, nx, L, W, [&](int i, double v) { lt[i] = v; });
      } else {
        tri_cols_lds(LQ, xn, nx, ct, L);
        __syncthreads();
        tri_rows_lds(LQ, ct, nx, L, [&](int i, double v) { lt[i] = v; });
      }
      __syncthreads();
      if (rx) {
        const double l = v_p + lt[tid];
        const double tot = mode == 0 ? l : v_LM0 + l;
        lt[tid] = tot;
        LM[(int64_t)k * nx + tid] = tot;
      }
      __syncthreads();
      // residual rows of stage k (total iterate)
      if (res) {
        {
          double cx[S::XC];
#pragma unroll
          for (int c = 0; c < S::XC; ++c) cx[c] = 0.0;
          double cu[1] = {0.0};
          frag_cols(fA, lt, nx, cx, L, W);      // A^T lam_k
          frag_cols(fB, lt, nx, cu, L, W);      // B^T lam_k
          if (k > 0) {
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
        if (rx) ax[tid] = colsum_total(px, NXP, W, tid) + (k > 0 ? 0.5 * xs[tid] : 0.0);
        if (ru) au[tid] = colsum_total(pu, NUP, W, tid);
        __syncthreads();
        frag_rows(fR, ut, nu, L, W, [&](int i, double v) { au[i] = fma(0.5, v, au[i]); });
        __syncthreads();
        if (Sm) frag_rows(fS, xt, nu, L, W, [&](int i, double v) { au[i] += v; if (k == 0) s0[i] = v; });
        __syncthreads();
        if (ru) {
          const double rho = -v_r - au[tid];
          mr = nan_max(mr, fabs(rho));
          mb = nan_max(mb, fabs(v_r + (k == 0 && Sm ? s0[tid] : 0.0)));
          rhu[(int64_t)k * nu + tid] = -rho;
        }
        if (rx) {
          const double axu = mode == 0 ? xn[tid] - v_f : al[tid];
          const double rho = -v_f - (axu - xt1[tid]);
          mr = nan_max(mr, fabs(rho));
          mb = nan_max(mb, fabs(v_f + (k == 0 ? a0[tid] : 0.0)));
          flam[(int64_t)k * nx + tid] = -rho;
          if (k > 0) {
            const double rho2 = -v_q - (ax[tid] - ltm[tid]);
            mr = nan_max(mr, fabs(rho2));
            mb = nan_max(mb, fabs(v_q));
            rhx[(int64_t)k * nx + tid] = -rho2;
          }
        }
      }
      __syncthreads();
      if (rx) {
        xc[tid] = xn[tid];
        xt[tid] = xt1[tid];
        ltm[tid] = lt[tid];
      }
      __syncthreads();
    }
    if (!res) return (double)NAN;
    // stage N rows: rho_x,N = -q_N - (Q_N,sym x_N - lam_{N-1})
    {
      const Lanes L = lanes_now();
      double cx[S::XC];
#pragma unroll
      for (int c = 0; c < S::XC; ++c) cx[c] = 0.0;
      stream_sq<S::RXX, S::XC, S::XW>(Q + (int64_t)N * nx * nx, nx, xt, cx, L, W, [&](int i, double v) { xs[i] = v; });
      colsum_publish<S::XC, S::XW>(cx, px, NXP, L);
      __syncthreads();
      if (rx) ax[tid] = 0.5 * (colsum_total(px, NXP, W, tid) + xs[tid]);
      __syncthreads();
      if (rx) {
        const double qi = rhs_q(N, tid);
        const double rho = -qi - (ax[tid] - ltm[tid]);
        mr = nan_max(mr, fabs(rho));
        mb = nan_max(mb, fabs(qi));
        rhx[(int64_t)N * nx + tid] = -rho;
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
  // w = L^Q_{k+1} (L^Q_{k+1})^T f_k + p2_{k+1}, p2_N = q_N.  Reads issued at the stage start.
  auto backward = [&]() {
    if (rx) {
      const double v = rhx[(int64_t)N * nx + tid];
      pn[tid] = v;
      p2[(int64_t)N * nx + tid] = v;
    }
    __syncthreads();
    for (int k = N - 1; k >= 0; --k) {
      ensure(k);
      const Lanes L = lanes_now();
      const TF* blk = blk_of(k);
      const TF* blk1 = blk_of(k + 1);
      const int iu = ru ? tid : nu - 1, ix = rx ? tid : nx - 1;
      const double v_fl = flam[(int64_t)k * nx + ix];
      const double v_q = keep_if<ORD>(k > 0, rhx[(int64_t)k * nx + ix]);
      const double v_dr = (double)blk[off_dR(nx, nu) + iu];
      const double v_rv = rhu[(int64_t)k * nu + iu];
      Frag<S::RXU, 1, S::UW> fLS, fB;
      Frag<S::RXX, S::XC, S::XW> fA;
      frag_load<ORD>(fB, B + (int64_t)k * nx * nu, nx, nu, nu, L, W);
      frag_load<ORD>(fA, A + (int64_t)k * nx * nx, nx, nx, nx, L, W);
      frag_load<ORD>(fLS, blk + off_LS(nx, nu), nx, nu, nu, L, W);
      Frag<(LQREG ? S::RXX : 1), S::XC, S::XW> fLQ;
      if constexpr (LQREG) frag_load_tri<ORD>(fLQ, blk1 + off_LQ(nx, nu), nx, L, W);
      else tri_to_lds<S::NT, tri_chunk(NXP, S::NT)>(blk1 + off_LQ(nx, nu), nx, LQ);
      tri_to_lds<S::NT, tri_chunk(NUP, S::NT)>(blk, nu, LR);
      if (rx) fl[tid] = v_fl;
      if (ru) dr[tid] = v_dr;
      __syncthreads();
      // w = L^Q (L^Q^T f) + p2_{k+1}
      if constexpr (LQREG) {
        {
          double cq[S::XC];
#pragma unroll
          for (int c = 0; c < S::XC; ++c) cq[c] = 0.0;
          frag_cols(fLQ, fl, nx, cq, L, W);
          colsum_publish<S::XC, S::XW>(cq, px, NXP, L);
        }
        __syncthreads();
        if (rx) xs[tid] = colsum_total(px, NXP, W, tid);
        __syncthreads();
        frag_rows(fLQ, xs, nx, L, W, [&](int i, double v) { ct[i] = pn[i] + v; });
      } else {
        tri_cols_lds(LQ, fl, nx, xs, L);
        __syncthreads();
        tri_rows_lds(LQ, xs, nx, L, [&](int i, double v) { ct[i] = pn[i] + v; });
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
      if (ru) us[tid] = v_rv + colsum_total(pu, NUP, W, tid);
      if (rx) qv[tid] = v_q + colsum_total(px, NXP, W, tid);
      __syncthreads();
      // rbar2 = (L^R)^{-1} rhat
      lr_solve<false, NUP>(LR, dr, nu, us, yb);
      __syncthreads();
      if (ru) rb2[(int64_t)k * nu + tid] = yb[tid];
      // p2_k = qhat - L^S rbar2
      if (k > 0) {
        frag_rows(fLS, yb, nx, L, W, [&](int i, double v) {
          const double pk = qv[i] - v;
          pn[i] = pk;
          p2[(int64_t)k * nx + i] = pk;
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
    rel = forward(f0 ? 0 : 1, f0 ? rb0 : rb2, f0 ? p0 : p2, want || !f0);
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
        if (want && !isfinite(rel)) code = LQ_INFO_NONFINITE;
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
