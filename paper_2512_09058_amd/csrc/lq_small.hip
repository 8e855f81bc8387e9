// Size-specialised kernels for uniform batches with nx + nu <= 16.
//
// Mapping: 16 lanes per instance, four instances per 64-wide wavefront.  Lane i of an
// instance owns row i of the stage matrix Hhat_k = [[R,S],[S^T,Q]] + V V^T (rows 0..nu-1 are
// the inputs, rows nu..nu+nx-1 the states) and, after the stage Cholesky, row i of its factor
// [[L^R, 0],[L^S, L^Q]].  What an instance carries from stage to stage (rows of L^Q_{k+1},
// p_{k+1}; in the solve, x_k and lam_{k-1}) stays in registers.  Cross-row operands are
// broadcast inside the 16-lane row with 64-bit DPP row_newbcast moves (VALU, no LDS).
//
// With one wavefront per SIMD (4096 instances = 1024 wavefronts), latency is hidden by
// instruction-level parallelism only, so all global loads use per-lane clamped addresses
// (no branches around them) and the loads of stage k-1 are issued before stage k is computed.
//
// Factor sweep per stage (backward in time), c_i = column i of [B_k A_k] in lane i:
//   V[i][j]    = sum_{m>=j} c_i[m] L^Q_{k+1}[m][j]       (trmm: broadcast rows of L^Q)
//   Hhat[i][j] = H[i][j] + sum_m V[i][m] V[j][m]          (syrk: broadcast rows of V)
//   chol(Hhat)                                            (potrf, float64, right-looking)
// plus the right-hand-side sweep rbar_k = (L^R_k)^{-1}(r_k + B_k^T w),
// p_k = q_k + A_k^T w - L^S_k rbar_k, w = L^Q_{k+1} L^Q_{k+1}^T f_k + p_{k+1}.
//
// Solve: one forward pass computes the rollout and, in the same pass, the float64 KKT
// residual of the new iterate (eq. opt-cond-ocp-eq); each refinement iteration is a backward
// correction sweep over the stored residual followed by another forward+residual pass.
//
// Factor blocks use the generic workspace layout, so the generic solve and adjoint kernels
// consume these factors unchanged.
#include <math.h>

#include "lq_internal.hpp"

namespace lq {
namespace {

__device__ __forceinline__ double rsqrt_f64(double a) {
  double y = __builtin_amdgcn_rsq(a);
  const double h = 0.5 * a;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// Broadcast lane k of each 16-lane row to the whole row (k is a constant after unrolling).
__device__ __forceinline__ double bc(double v, int k) {
  long x = __double_as_longlong(v);
  switch (k) {
#define BC(K) \
  case K:     \
    x = __builtin_amdgcn_update_dpp((long)0, x, 0x150 + K, 0xF, 0xF, true); \
    break;
    BC(0) BC(1) BC(2) BC(3) BC(4) BC(5) BC(6) BC(7) BC(8) BC(9) BC(10) BC(11) BC(12) BC(13) BC(14) BC(15)
#undef BC
  }
  return __longlong_as_double(x);
}
__device__ __forceinline__ float bc(float v, int k) {
  int x = __float_as_int(v);
  switch (k) {
#define BC(K) \
  case K:     \
    x = __builtin_amdgcn_update_dpp(0, x, 0x150 + K, 0xF, 0xF, true); \
    break;
    BC(0) BC(1) BC(2) BC(3) BC(4) BC(5) BC(6) BC(7) BC(8) BC(9) BC(10) BC(11) BC(12) BC(13) BC(14) BC(15)
#undef BC
  }
  return __int_as_float(x);
}

// 32-bit DPP lane permutations for the row reduction (quad_perm [1,0,3,2], [2,3,0,1],
// row_ror 4, row_ror 8).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double rowmax(double v) {
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x124>(v));
  v = fmax(v, dpp_d<0x128>(v));
  return v;
}

// Right-looking Cholesky of the row-distributed tile (lane i holds row i in h), pivot
// columns 0..NCOL-1.  Returns 0, 1 (a pivot was not positive) or 2 (non-finite pivot); bad
// pivots are replaced by 1 so the sweep continues without NaNs.
template <int NUX, int NCOL>
__device__ __forceinline__ int potrf_rows(double (&h)[NUX], double& mydinv, int i) {
  int bad = 0;
#pragma unroll
  for (int j = 0; j < NCOL; ++j) {
    double dj = bc(h[j], j);
    const bool fin = isfinite(dj);
    const bool ok = fin && dj > 0.0;
    bad = (bad == 0 && !ok) ? (fin ? 1 : 2) : bad;
    dj = ok ? dj : 1.0;
    const double inv = rsqrt_f64(dj);
    h[j] = (i == j) ? dj * inv : h[j] * inv;
    mydinv = (i == j) ? inv : mydinv;
#pragma unroll
    for (int kk = j + 1; kk < NCOL; ++kk) h[kk] = fma(-h[j], bc(h[j], kk), h[kk]);
  }
  return bad;
}

template <typename T>
__device__ __forceinline__ double rnd(double v) {
  return (double)(T)v;
}

template <int NX, int NU>
struct Shape {
  static constexpr int NUX = NX + NU;
  static constexpr int64_t FS = (int64_t)NU * (NU + 1) / 2 + NU + NX * NU + NX * (NX + 1) / 2 + NX;
  static constexpr int ODR = NU * (NU + 1) / 2, OLS = ODR + NU, OLQ = OLS + NX * NU,
                       ODQ = OLQ + NX * (NX + 1) / 2;
};

// Lane identity shared by the kernels.
struct Lane {
  int i, ic, mi;   // row in the instance, clamped input row, clamped state row
  bool isu, inst, valid;
  int b;
  int64_t bb;      // clamped instance index (a valid one, for loads)
};

template <int NX, int NU>
__device__ __forceinline__ Lane lane_id(int batch) {
  constexpr int NUX = NX + NU;
  Lane L;
  const int l = threadIdx.x & 63;
  L.i = l & 15;
  L.b = blockIdx.x * 4 + (l >> 4);
  L.inst = L.b < batch;
  L.valid = L.inst && L.i < NUX;
  L.bb = L.inst ? L.b : 0;
  L.isu = L.i < NU;
  L.ic = L.isu ? L.i : 0;
  L.mi = (!L.isu && L.i < NUX) ? L.i - NU : 0;
  return L;
}

// ------------------------------------------------------------------------------------------
// Factor sweep

template <int NX, int NU>
struct FStage {
  double c[NX];          // column i of [B_k A_k]
  double h[NX + NU];     // lower part of row i of [[R,S],[S^T,Q]] (symmetrised)
  double rq;             // r_k[i] (input lanes) or q_k[m] (state lanes)
  double fk[NX];         // f_k (all lanes)
};

template <int NX, int NU, bool HS, bool HF>
__device__ __forceinline__ void load_fstage(FStage<NX, NU>& st, const Lane& L, int k, const lq_data& d,
                                            int N) {
  constexpr int NUX = NX + NU;
  const int64_t bb = L.bb;
  const double* Ak = d.A + (bb * N + k) * NX * NX;
  const double* Bk = d.B + (bb * N + k) * NX * NU;
  const double* Rk = d.R + (bb * N + k) * NU * NU;
  const double* Qk = d.Q + (bb * (N + 1) + k) * NX * NX;
  const double* Sk = HS ? d.S + (bb * N + k) * NU * NX : Rk;
  const double* cp = L.isu ? Bk + L.ic : Ak + L.mi;
  const int cs = L.isu ? NU : NX;
#pragma unroll
  for (int m = 0; m < NX; ++m) st.c[m] = cp[m * cs];
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    const double a1 = L.isu ? Rk[L.ic * NU + j] : (HS ? Sk[j * NX + L.mi] : 0.0);
    const double a2 = Rk[j * NU + L.ic];
    st.h[j] = L.isu ? (j <= L.ic ? 0.5 * (a1 + a2) : 0.0) : a1;
  }
#pragma unroll
  for (int j = 0; j < NX; ++j) {
    const double a1 = Qk[L.mi * NX + j], a2 = Qk[j * NX + L.mi];
    st.h[NU + j] = (!L.isu && j <= L.mi) ? 0.5 * (a1 + a2) : 0.0;
  }
  const double rv = d.r[(bb * N + k) * NU + L.ic];
  const double qv = d.q[(bb * (N + 1) + k) * NX + L.mi];
  st.rq = L.isu ? rv : (k > 0 ? qv : 0.0);
#pragma unroll
  for (int m = 0; m < NX; ++m) st.fk[m] = HF ? d.f[(bb * N + k) * NX + m] : 0.0;
  (void)NUX;
}

template <int NX, int NU, typename TF, typename TP, bool HS, bool HF>
__global__ void __launch_bounds__(64) k_factor_small(int batch, int N, lq_data d, TF* __restrict__ F,
                                                     double* __restrict__ Vws, int32_t* __restrict__ info) {
  using SH = Shape<NX, NU>;
  constexpr int NUX = SH::NUX;
  constexpr int64_t FS = SH::FS;
  static_assert(NUX <= 16, "tile exceeds a 16-lane row");
  const Lane L = lane_id<NX, NU>(batch);
  const int i = L.i, ic = L.ic, mi = L.mi;
  const bool isu = L.isu, valid = L.valid;

  TF* Fi = F + L.bb * (N + 1) * FS;
  double* rbar = Vws + L.bb * ((int64_t)N * NU + (int64_t)(N + 1) * NX);
  double* pv = rbar + (int64_t)N * NU;

  double h[NUX];
  double lq[NX];
  double mydinv = 1.0, pn = 0.0;
  int code = 0;

  // ---- stage N: factor blockdiag(I, sym Q_N) -> blockdiag(I, L^Q_N)
  {
    const double* QN = d.Q + (L.bb * (N + 1) + N) * NX * NX;
#pragma unroll
    for (int j = 0; j < NUX; ++j) {
      double v;
      if (j < NU) {
        v = (i == j) ? 1.0 : 0.0;
      } else {
        const double a1 = QN[mi * NX + (j - NU)], a2 = QN[(j - NU) * NX + mi];
        v = (!isu && (j - NU) <= mi) ? 0.5 * (a1 + a2) : 0.0;
      }
      h[j] = v;
    }
    pn = d.q[(L.bb * (N + 1) + N) * NX + mi];
    const int bad = potrf_rows<NUX, NUX>(h, mydinv, i);
    if (bad) code = bad == 2 ? LQ_INFO_NONFINITE : N + 1;
#pragma unroll
    for (int j = 0; j < NUX; ++j) h[j] = rnd<TF>(h[j]);
    mydinv = rnd<TF>(mydinv);
    TF* FN = Fi + (int64_t)N * FS;
    if (valid && !isu) {
#pragma unroll
      for (int j = 0; j < NX; ++j)
        if (j <= mi) FN[SH::OLQ + mi * (mi + 1) / 2 + j] = (TF)h[NU + j];
      FN[SH::ODQ + mi] = (TF)mydinv;
      pv[(int64_t)N * NX + mi] = pn;
    }
#pragma unroll
    for (int j = 0; j < NX; ++j) lq[j] = (j <= mi) ? h[NU + j] : 0.0;
  }

  FStage<NX, NU> cur, nxt;
  load_fstage<NX, NU, HS, HF>(cur, L, N - 1, d, N);
  for (int k = N - 1; k >= 0; --k) {
    if (k > 0) load_fstage<NX, NU, HS, HF>(nxt, L, k - 1, d, N);
#pragma unroll
    for (int j = 0; j < NUX; ++j) h[j] = cur.h[j];
    double tq = cur.rq;
    // trmm V = C^T L^Q_{k+1}; t1 = L^Q_{k+1}^T f_k
    TP v[NX];
    double t1[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      v[j] = 0;
      t1[j] = 0.0;
    }
#pragma unroll
    for (int m = 0; m < NX; ++m) {
#pragma unroll
      for (int j = 0; j <= m; ++j) {
        if (sizeof(TP) == 4) {
          const float Lf = bc((float)lq[j], NU + m);
          v[j] += (TP)cur.c[m] * (TP)Lf;
          if (HF) t1[j] = fma((double)Lf, cur.fk[m], t1[j]);
        } else {
          const double Ld = bc(lq[j], NU + m);
          v[j] += (TP)cur.c[m] * (TP)Ld;
          if (HF) t1[j] = fma(Ld, cur.fk[m], t1[j]);
        }
      }
    }
    // w = L^Q_{k+1} t1 + p_{k+1} (state lanes), then (rhat, qhat) = (r, q) + C^T w
    double wv = pn;
    if (HF) {
#pragma unroll
      for (int j = 0; j < NX; ++j) wv = fma(lq[j], t1[j], wv);
    }
#pragma unroll
    for (int m = 0; m < NX; ++m) tq = fma(cur.c[m], bc(wv, NU + m), tq);
    // syrk Hhat = H + V V^T
#pragma unroll
    for (int j = 0; j < NUX; ++j) {
      TP acc = 0;
#pragma unroll
      for (int m = 0; m < NX; ++m) acc += v[m] * bc(v[m], j);
      h[j] += (double)acc;
    }
    // potrf (float64); at k = 0 only the nu input columns
    int bad;
    if (k > 0) bad = potrf_rows<NUX, NUX>(h, mydinv, i);
    else bad = potrf_rows<NUX, NU>(h, mydinv, i);
    if (bad && code == 0) code = bad == 2 ? LQ_INFO_NONFINITE : k + 1;
#pragma unroll
    for (int j = 0; j < NUX; ++j) h[j] = rnd<TF>(h[j]);
    mydinv = rnd<TF>(mydinv);
    // rbar = L^R^{-1} rhat and p_k = qhat - L^S rbar in one column sweep
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      const double rb = bc(tq * mydinv, j);
      tq = (i > j) ? fma(-h[j], rb, tq) : tq;
    }
    // stores
    TF* Fk = Fi + (int64_t)k * FS;
    if (valid) {
      if (isu) {
#pragma unroll
        for (int j = 0; j < NU; ++j)
          if (j <= ic) Fk[ic * (ic + 1) / 2 + j] = (TF)h[j];
        Fk[SH::ODR + ic] = (TF)mydinv;
        rbar[(int64_t)k * NU + ic] = tq * mydinv;
      } else {
#pragma unroll
        for (int j = 0; j < NU; ++j) Fk[SH::OLS + mi * NU + j] = (TF)h[j];
        if (k > 0) {
#pragma unroll
          for (int j = 0; j < NX; ++j)
            if (j <= mi) Fk[SH::OLQ + mi * (mi + 1) / 2 + j] = (TF)h[NU + j];
          Fk[SH::ODQ + mi] = (TF)mydinv;
          pv[(int64_t)k * NX + mi] = tq;
        }
      }
    }
    pn = tq;
#pragma unroll
    for (int j = 0; j < NX; ++j) lq[j] = (j <= mi) ? h[NU + j] : 0.0;
    if (k > 0) cur = nxt;
  }
  if (L.inst && i == 0) info[L.b] = code;
}

// ------------------------------------------------------------------------------------------
// Solve.  Lane roles: lane j < nu carries u_j; lane nu + m carries x_m and lam_m.

template <int NX, int NU, typename TF, bool HS, bool HF>
struct SolveCtx {
  using SH = Shape<NX, NU>;
  Lane L;
  int N;
  const TF* F;             // this instance's factor blocks
  lq_data d;
  const double *rb0, *p0;  // factor-time sweep vectors
  double *rb2, *p2, *flam, *rhou, *rhox;
  double *x, *u, *lam;
  __device__ double LRv(int k, int row, int col) const { return (double)F[k * SH::FS + row * (row + 1) / 2 + col]; }
  __device__ double LSv(int k, int row, int col) const { return (double)F[k * SH::FS + SH::OLS + row * NU + col]; }
  __device__ double LQv(int k, int row, int col) const {
    return (double)F[k * SH::FS + SH::OLQ + row * (row + 1) / 2 + col];
  }
  __device__ double dRv(int k, int row) const { return (double)F[k * SH::FS + SH::ODR + row]; }
};

// Forward-pass operands of stage k, loaded ahead of time.
template <int NX, int NU>
struct FwdStage {
  double g[NX];    // input lanes: column ic of L^S_k;  state lanes: row mi of A_k
  double e[NU];    // input lanes: L^R_k[j][ic] (j > ic used);  state lanes: row mi of B_k
  double s0;       // input lanes: rbar_k[ic];  state lanes: f_k[mi] (or flam_k[mi])
  double s1;       // input lanes: 1 / L^R_k[ic][ic];  state lanes: p_{k+1}[mi]
  double zu, zx, zl;  // old iterate (correction passes): u_k[ic], x_{k+1}[mi], lam_k[mi]
};

// State lanes: column / row mi of L^Q_{k+1} (rows >= mi, cols <= mi used); loaded at the top
// of stage k, consumed after the rollout step.
template <int NX>
struct LqRowCol {
  double lc[NX], lr[NX];
};

template <int NX, int NU, typename TF, bool HS, bool HF>
__device__ __forceinline__ void load_fwd(FwdStage<NX, NU>& st, const SolveCtx<NX, NU, TF, HS, HF>& s, int k,
                                         int mode) {
  const Lane& L = s.L;
  const int N = s.N;
  const int64_t bb = L.bb;
  const double* Ak = s.d.A + (bb * N + k) * NX * NX;
  const double* Bk = s.d.B + (bb * N + k) * NX * NU;
  using SH = Shape<NX, NU>;
  // input lanes: column ic of L^S_k (stride nu) and L^R_k[j][ic] at j(j+1)/2 + ic (inside the
  // packed L^R block for every j < nu); state lanes: rows mi of A_k and B_k
  const TF* fb = s.F + (int64_t)k * SH::FS;
  const TF* gsp = fb + SH::OLS + L.ic;
  const TF* erp = fb + L.ic;
  const double* ap = Ak + L.mi * NX;
  const double* bp = Bk + L.mi * NU;
#pragma unroll
  for (int m = 0; m < NX; ++m) {
    const double gs = (double)gsp[m * NU];
    st.g[m] = L.isu ? gs : ap[m];
  }
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    const double er = (double)erp[j * (j + 1) / 2];
    st.e[j] = L.isu ? er : bp[j];
  }
  const double* rbv = mode == 0 ? s.rb0 : s.rb2;
  const double* pvv = mode == 0 ? s.p0 : s.p2;
  double fv;
  if (mode == 0) fv = HF ? s.d.f[(bb * N + k) * NX + L.mi] : 0.0;
  else fv = s.flam[(int64_t)k * NX + L.mi];
  st.s0 = L.isu ? rbv[(int64_t)k * NU + L.ic] : fv;
  st.s1 = L.isu ? s.dRv(k, L.ic) : pvv[(int64_t)(k + 1) * NX + L.mi];
  if (mode == 1) {
    st.zu = s.u[(int64_t)k * NU + L.ic];
    st.zx = s.x[(int64_t)k * NX + L.mi];
    st.zl = s.lam[(int64_t)k * NX + L.mi];
  } else {
    st.zu = st.zx = st.zl = 0.0;
  }
}

// Column mi of the packed lower L^Q at rows m >= mi sits at m(m+1)/2 + mi, row mi at
// mi(mi+1)/2 + j: one per-lane base plus compile-time offsets.  Masked entries read other
// elements of the same packed block (all offsets stay below nx(nx+1)/2).
template <int NX, int NU, typename TF, bool HS, bool HF>
__device__ __forceinline__ void load_lq(LqRowCol<NX>& st, const SolveCtx<NX, NU, TF, HS, HF>& s, int k) {
  using SH = Shape<NX, NU>;
  const int mi = s.L.mi;
  const TF* blk = s.F + (int64_t)k * SH::FS + SH::OLQ;
  const TF* pc = blk + mi;
  const TF* pr = blk + mi * (mi + 1) / 2;
#pragma unroll
  for (int m = 0; m < NX; ++m) {
    st.lc[m] = (double)pc[m * (m + 1) / 2];
    st.lr[m] = (double)pr[m];
  }
}

// Residual operands of stage k.
template <int NX, int NU>
struct ResStage {
  double g1[NX];   // input lanes: row ic of S_k;  state lanes: row mi of sym(Q_k)
  double g2[NX];   // input lanes: column ic of B_k;  state lanes: column mi of A_k
  double e[NU];    // input lanes: row ic of sym(R_k);  state lanes: column mi of S_k
  double rq;       // r_k[ic] or q_k[mi]
  double fo;       // f_k[mi] (original right-hand side)
};

template <int NX, int NU, typename TF, bool HS, bool HF>
__device__ __forceinline__ void load_res(ResStage<NX, NU>& st, const SolveCtx<NX, NU, TF, HS, HF>& s, int k) {
  const Lane& L = s.L;
  const int N = s.N;
  const int64_t bb = L.bb;
  const double* Ak = s.d.A + (bb * N + k) * NX * NX;
  const double* Bk = s.d.B + (bb * N + k) * NX * NU;
  const double* Rk = s.d.R + (bb * N + k) * NU * NU;
  const double* Qk = s.d.Q + (bb * (N + 1) + k) * NX * NX;
  const double* Sk = HS ? s.d.S + (bb * N + k) * NU * NX : Rk;
#pragma unroll
  for (int m = 0; m < NX; ++m) {
    const double q1 = Qk[L.mi * NX + m], q2 = Qk[m * NX + L.mi];
    const double sr = HS ? Sk[L.ic * NX + m] : 0.0;
    st.g1[m] = L.isu ? sr : 0.5 * (q1 + q2);
    st.g2[m] = L.isu ? Bk[m * NU + L.ic] : Ak[m * NX + L.mi];
  }
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    const double r1 = Rk[L.ic * NU + j], r2 = Rk[j * NU + L.ic];
    const double sc = HS ? Sk[j * NX + L.mi] : 0.0;
    st.e[j] = L.isu ? 0.5 * (r1 + r2) : sc;
  }
  const double rv = s.d.r[(bb * N + k) * NU + L.ic];
  const double qv = s.d.q[(bb * (N + 1) + k) * NX + L.mi];
  st.rq = L.isu ? rv : qv;
  st.fo = HF ? s.d.f[(bb * N + k) * NX + L.mi] : 0.0;
}

// One forward pass.  mode 0: z = solution (x_0 = x_init, f = f_k, sweep vectors of lq_factor);
// mode 1: z += correction (dx_0 = 0, f = flam, sweep vectors rbar2/p2).  With `res`, computes
// the KKT residual of the updated iterate on the fly (and stores it when `store`); returns
// rel_res (uniform over the instance's 16 lanes), or 0 without `res`.
template <int NX, int NU, typename TF, bool HS, bool HF>
__device__ double fwd_res(const SolveCtx<NX, NU, TF, HS, HF>& s, int mode, bool res, bool store) {
  constexpr int NUX = NX + NU;
  const Lane& L = s.L;
  const int N = s.N, i = L.i, mi = L.mi, ic = L.ic;
  const bool isu = L.isu, xl = L.valid && !L.isu, ul = L.valid && L.isu;
  const double x0v = s.d.x0[L.bb * NX + mi];
  double xc = (mode == 0 && !isu) ? x0v : 0.0;  // recursion state (x_k or dx_k)
  double xk = isu ? 0.0 : x0v;                   // updated iterate x_k (x_0 = x_init)
  double lkm = 0.0;                              // updated lam_{k-1}
  double mr = 0.0, mb = 0.0;
  FwdStage<NX, NU> cur, nxt;
  load_fwd<NX, NU, TF, HS, HF>(cur, s, 0, mode);
  for (int k = 0; k < N; ++k) {
    if (k + 1 < N) load_fwd<NX, NU, TF, HS, HF>(nxt, s, k + 1, mode);
    LqRowCol<NX> lq;
    load_lq<NX, NU, TF, HS, HF>(lq, s, k + 1);
    ResStage<NX, NU> rs;
    if (res) load_res<NX, NU, TF, HS, HF>(rs, s, k);
    // t = rbar + L^S^T x on input lanes
    double t = cur.s0, t_b = 0.0;
#pragma unroll
    for (int m = 0; m < NX; ++m) {
      const double xb = bc(xc, NU + m);
      if (m & 1) t_b = fma(cur.g[m], xb, t_b);
      else t = fma(cur.g[m], xb, t);
    }
    t += t_b;
    // u' = L^R^{-T} t, u = -u'
    double uu = 0.0;
#pragma unroll
    for (int j = NU - 1; j >= 0; --j) {
      const double uj = bc(t * cur.s1, j);
      uu = (i == j) ? uj : uu;
      t = (i < j) ? fma(-cur.e[j], uj, t) : t;
    }
    const double du = -uu;
    // x_{k+1} = A x + B u + f on state lanes
    double xn = cur.s0, xn_b = 0.0;
#pragma unroll
    for (int n = 0; n < NX; ++n) {
      const double xb = bc(xc, NU + n);
      if (n & 1) xn_b = fma(cur.g[n], xb, xn_b);
      else xn = fma(cur.g[n], xb, xn);
    }
#pragma unroll
    for (int j = 0; j < NU; ++j) xn = fma(cur.e[j], bc(du, j), xn);
    xn += xn_b;
    // lam = L^Q_{k+1} (L^Q_{k+1}^T x_{k+1}) + p_{k+1}
    double t2 = 0.0;
#pragma unroll
    for (int m = 0; m < NX; ++m) {
      const double xb = bc(xn, NU + m);
      t2 = (m >= mi) ? fma(lq.lc[m], xb, t2) : t2;
    }
    double lm = cur.s1;
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const double tb = bc(t2, NU + j);
      lm = (j <= mi) ? fma(lq.lr[j], tb, lm) : lm;
    }
    // updated iterate
    const double unew = du + cur.zu;
    const double xnew = xn + cur.zx;
    const double lnew = lm + cur.zl;
    if (ul) s.u[(int64_t)k * NU + ic] = unew;
    if (xl) {
      s.x[(int64_t)k * NX + mi] = xnew;
      s.lam[(int64_t)k * NX + mi] = lnew;
    }
    if (res) {
      // residual rows of stage k at the updated iterate (x_k = xk, u_k, lam_k, x_{k+1}, lam_{k-1})
      double au = 0.0, au2 = 0.0, bu = 0.0;  // R u + S x_k + B^T lam ;  S_0 x_init
      double al = -xnew, bl = 0.0;           // A x_k + B u - x_{k+1} ;  A_0 x_init
      double ax = -lkm, ax2 = 0.0;           // S^T u + Q x_k + A^T lam - lam_{k-1}
#pragma unroll
      for (int n = 0; n < NX; ++n) {
        const double xb = bc(xk, NU + n);
        const double lb = bc(lnew, NU + n);
        if (HS) au = fma(rs.g1[n], xb, au);      // input lanes: S row
        au2 = fma(rs.g2[n], lb, au2);            // input lanes: B column -> B^T lam
        al = fma(cur.g[n], xb, al);              // state lanes: A row
        ax = fma(rs.g1[n], xb, ax);              // state lanes: sym Q row
        ax2 = fma(rs.g2[n], lb, ax2);            // state lanes: A column -> A^T lam
      }
      if (k == 0) {
        bu = HS ? au : 0.0;
        bl = al + xnew;
      }
#pragma unroll
      for (int j = 0; j < NU; ++j) {
        const double ub = bc(unew, j);
        au = fma(rs.e[j], ub, au);               // input lanes: sym R row
        al = fma(cur.e[j], ub, al);              // state lanes: B row
        if (HS) ax = fma(rs.e[j], ub, ax);       // state lanes: S column -> S^T u
      }
      au += au2;
      ax += ax2;
      const double rhou = -rs.rq - au;
      const double rhol = -rs.fo - al;
      const double rhox = -rs.rq - ax;
      if (ul) {
        mr = fmax(mr, fabs(rhou));
        mb = fmax(mb, fabs(rs.rq + bu));
      }
      if (xl) {
        mr = fmax(mr, fabs(rhol));
        mb = fmax(mb, fabs(rs.fo + bl));
        if (k > 0) {
          mr = fmax(mr, fabs(rhox));
          mb = fmax(mb, fabs(rs.rq));
        }
      }
      if (store) {
        if (ul) s.rhou[(int64_t)k * NU + ic] = rhou;
        if (xl) {
          s.flam[(int64_t)k * NX + mi] = -rhol;
          if (k > 0) s.rhox[(int64_t)k * NX + mi] = rhox;
        }
      }
    }
    xc = xn;
    xk = xnew;
    lkm = lnew;
    if (k + 1 < N) cur = nxt;
  }
  if (res) {
    // stage N: Q_N x_N - lam_{N-1} = -q_N
    const int64_t bb = L.bb;
    const double* QN = s.d.Q + (bb * (N + 1) + N) * NX * NX;
    double ax = -lkm;
#pragma unroll
    for (int n = 0; n < NX; ++n) {
      const double xb = bc(xk, NU + n);
      ax = fma(0.5 * (QN[mi * NX + n] + QN[n * NX + mi]), xb, ax);
    }
    const double qv = s.d.q[(bb * (N + 1) + N) * NX + mi];
    const double rhox = -qv - ax;
    if (xl) {
      mr = fmax(mr, fabs(rhox));
      mb = fmax(mb, fabs(qv));
      if (store) s.rhox[(int64_t)N * NX + mi] = rhox;
    }
    mr = rowmax(mr);
    mb = rowmax(mb);
    return mb > 0.0 ? mr / mb : mr;
  }
  (void)NUX;
  return 0.0;
}

// Backward sweep of the correction right-hand side (r, q, f) = (-rho_u, -rho_x, -rho_l),
// x_init = 0, into (rbar2, p2).
template <int NX, int NU>
struct BwdStage {
  double lc[NX], lr[NX];  // state lanes: column / row mi of L^Q_{k+1}
  double cc[NX];          // column i of [B_k A_k]
  double hr[NU];          // input lanes: row ic of L^R_k;  state lanes: row mi of L^S_k
  double dr;              // 1 / L^R_k[ic][ic]
  double rho;             // rho_u,k[ic] or rho_x,k[mi]
  double fl;              // flam_k[mi] = -rho_l,k
};

template <int NX, int NU, typename TF, bool HS, bool HF>
__device__ __forceinline__ void load_bwd(BwdStage<NX, NU>& st, const SolveCtx<NX, NU, TF, HS, HF>& s, int k) {
  const Lane& L = s.L;
  const int N = s.N;
  const int64_t bb = L.bb;
  const double* Ak = s.d.A + (bb * N + k) * NX * NX;
  const double* Bk = s.d.B + (bb * N + k) * NX * NU;
  using SH = Shape<NX, NU>;
  const TF* blk = s.F + (int64_t)(k + 1) * SH::FS + SH::OLQ;
  const TF* pc = blk + L.mi;
  const TF* pr = blk + L.mi * (L.mi + 1) / 2;
  const double* cp = L.isu ? Bk + L.ic : Ak + L.mi;
  const int cs = L.isu ? NU : NX;
#pragma unroll
  for (int m = 0; m < NX; ++m) {
    st.lc[m] = (double)pc[m * (m + 1) / 2];
    st.lr[m] = (double)pr[m];
    st.cc[m] = cp[m * cs];
  }
  // input lanes: row ic of packed L^R (entries j <= ic; j > ic reads stay inside the block);
  // state lanes: row mi of L^S
  const TF* hp = L.isu ? s.F + (int64_t)k * SH::FS + L.ic * (L.ic + 1) / 2
                       : s.F + (int64_t)k * SH::FS + SH::OLS + L.mi * NU;
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    const double v = (double)hp[j];
    st.hr[j] = (L.isu && j > L.ic) ? 0.0 : v;
  }
  st.dr = s.dRv(k, L.ic);
  st.rho = L.isu ? s.rhou[(int64_t)k * NU + L.ic] : s.rhox[(int64_t)k * NX + L.mi];
  st.fl = s.flam[(int64_t)k * NX + L.mi];
}

template <int NX, int NU, typename TF, bool HS, bool HF>
__device__ void bwd_corr(const SolveCtx<NX, NU, TF, HS, HF>& s) {
  const Lane& L = s.L;
  const int N = s.N, i = L.i, mi = L.mi, ic = L.ic;
  const bool isu = L.isu, xl = L.valid && !L.isu, ul = L.valid && L.isu;
  double p2n = -s.rhox[(int64_t)N * NX + mi];
  if (xl) s.p2[(int64_t)N * NX + mi] = p2n;
  BwdStage<NX, NU> cur, nxt;
  load_bwd<NX, NU, TF, HS, HF>(cur, s, N - 1);
  for (int k = N - 1; k >= 0; --k) {
    if (k > 0) load_bwd<NX, NU, TF, HS, HF>(nxt, s, k - 1);
    // t1 = L^Q_{k+1}^T f', w = L^Q_{k+1} t1 + p2_{k+1}
    double t1 = 0.0;
#pragma unroll
    for (int m = 0; m < NX; ++m) {
      const double fb = bc(cur.fl, NU + m);
      t1 = (m >= mi) ? fma(cur.lc[m], fb, t1) : t1;
    }
    double w = p2n;
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const double tb = bc(t1, NU + j);
      w = (j <= mi) ? fma(cur.lr[j], tb, w) : w;
    }
    double tq = (isu || k > 0) ? -cur.rho : 0.0, tq_b = 0.0;
#pragma unroll
    for (int m = 0; m < NX; ++m) {
      const double wb = bc(w, NU + m);
      if (m & 1) tq_b = fma(cur.cc[m], wb, tq_b);
      else tq = fma(cur.cc[m], wb, tq);
    }
    tq += tq_b;
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      const double rb = bc(tq * cur.dr, j);
      tq = (i > j) ? fma(-cur.hr[j], rb, tq) : tq;
    }
    if (ul) s.rb2[(int64_t)k * NU + ic] = tq * cur.dr;
    if (xl && k > 0) s.p2[(int64_t)k * NX + mi] = tq;
    p2n = tq;
    if (k > 0) cur = nxt;
  }
}

template <int NX, int NU, typename TF, bool HS, bool HF>
__global__ void __launch_bounds__(64) k_solve_small(SolveArgs a, int N) {
  using Ctx = SolveCtx<NX, NU, TF, HS, HF>;
  constexpr int64_t FS = Shape<NX, NU>::FS;
  Ctx s;
  s.L = lane_id<NX, NU>(a.batch);
  s.N = N;
  s.d = a.d;
  const int64_t bb = s.L.bb;
  s.F = (const TF*)a.F + bb * (N + 1) * FS;
  const int64_t vst = (int64_t)N * NU + (int64_t)(N + 1) * NX;
  s.rb0 = a.V + bb * vst;
  s.p0 = s.rb0 + (int64_t)N * NU;
  double* v2 = a.V2 + bb * v2_elems(N, NX, NU);
  s.rb2 = v2;
  s.p2 = v2 + v2_p2(N, NX, NU);
  s.flam = v2 + v2_flam(N, NX, NU);
  s.rhou = v2 + v2_rhou(N, NX, NU);
  s.rhox = v2 + v2_rhox(N, NX, NU);
  s.x = a.x + bb * N * NX;
  s.u = a.u + bb * N * NU;
  s.lam = a.lam + bb * N * NX;

  const bool res = a.check || a.max_it > 0;
  int it = 0;
  double rel = 0.0;
  bool act = false;
  if (s.L.inst) {
    rel = fwd_res<NX, NU, TF, HS, HF>(s, 0, res, a.max_it > 0);
    act = a.max_it > 0 && rel > a.tol;
  }
  while (__any(act)) {
    if (act) {
      bwd_corr<NX, NU, TF, HS, HF>(s);
      ++it;
      rel = fwd_res<NX, NU, TF, HS, HF>(s, 1, true, it < a.max_it);
      act = it < a.max_it && rel > a.tol;
    }
  }
  if (s.L.inst && s.L.i == 0) {
    const int b = s.L.b;
    if (a.rel_res) a.rel_res[b] = res ? rel : NAN;
    if (a.iters) a.iters[b] = it;
    if (a.info) {
      const int cur = a.info[b];
      if (cur <= 0) {
        int code = 0;
        if (res && !isfinite(rel)) code = LQ_INFO_NONFINITE;
        else if (res && a.max_it > 0 && rel > a.tol) code = LQ_INFO_NOT_CONVERGED;
        else if (cur == LQ_INFO_NONFINITE) code = cur;
        a.info[b] = code;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Dispatch over the compiled (nx, nu) shapes and the presence of S and f.

template <int NX, int NU, typename TF, typename TP>
hipError_t factor_tf(int batch, int N, const lq_data& d, void* F, double* V, int32_t* info, hipStream_t st) {
  const dim3 grid((batch + 3) / 4), block(64);
  const bool hs = d.S != nullptr, hf = d.f != nullptr;
  if (hs && hf)
    hipLaunchKernelGGL((k_factor_small<NX, NU, TF, TP, true, true>), grid, block, 0, st, batch, N, d, (TF*)F, V, info);
  else if (hs)
    hipLaunchKernelGGL((k_factor_small<NX, NU, TF, TP, true, false>), grid, block, 0, st, batch, N, d, (TF*)F, V, info);
  else if (hf)
    hipLaunchKernelGGL((k_factor_small<NX, NU, TF, TP, false, true>), grid, block, 0, st, batch, N, d, (TF*)F, V, info);
  else
    hipLaunchKernelGGL((k_factor_small<NX, NU, TF, TP, false, false>), grid, block, 0, st, batch, N, d, (TF*)F, V, info);
  return hipGetLastError();
}

template <int NX, int NU, typename TF>
hipError_t solve_tf(int N, const SolveArgs& a, hipStream_t st) {
  const dim3 grid((a.batch + 3) / 4), block(64);
  const bool hs = a.d.S != nullptr, hf = a.d.f != nullptr;
  if (hs && hf) hipLaunchKernelGGL((k_solve_small<NX, NU, TF, true, true>), grid, block, 0, st, a, N);
  else if (hs) hipLaunchKernelGGL((k_solve_small<NX, NU, TF, true, false>), grid, block, 0, st, a, N);
  else if (hf) hipLaunchKernelGGL((k_solve_small<NX, NU, TF, false, true>), grid, block, 0, st, a, N);
  else hipLaunchKernelGGL((k_solve_small<NX, NU, TF, false, false>), grid, block, 0, st, a, N);
  return hipGetLastError();
}

#define LQ_SMALL_SHAPES(X) X(12, 4) X(4, 2) X(8, 4) X(10, 6) X(6, 2)

}  // namespace

bool small_variant_available(lq_mode mode, int nx, int nu) {
  if (mode == LQ_MIXED_BF16) return false;
#define X(a, b) \
  if (nx == a && nu == b) return true;
  LQ_SMALL_SHAPES(X)
#undef X
  return false;
}

hipError_t launch_factor_small(lq_mode mode, int batch, int N, int nx, int nu, const lq_data& d, void* F,
                               double* V, int32_t* info, hipStream_t st) {
#define X(a, b)                                                                      \
  if (nx == a && nu == b)                                                            \
    return mode == LQ_F64 ? factor_tf<a, b, double, double>(batch, N, d, F, V, info, st) \
                          : factor_tf<a, b, float, float>(batch, N, d, F, V, info, st);
  LQ_SMALL_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_solve_small(lq_mode mode, int N, int nx, int nu, const SolveArgs& a, hipStream_t st) {
  if (a.rhs != RHS_PRIMAL) return hipErrorInvalidValue;
#define X(a_, b_) \
  if (nx == a_ && nu == b_) return mode == LQ_F64 ? solve_tf<a_, b_, double>(N, a, st) : solve_tf<a_, b_, float>(N, a, st);
  LQ_SMALL_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace lq
