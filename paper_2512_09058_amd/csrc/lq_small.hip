// Size-specialised kernels for uniform batches with nx + nu <= 16.
//
// Mapping: 16 lanes per instance, four instances per 64-wide wavefront.  Lane i of an
// instance owns row i of the stage matrix Hhat_k = [[R,S],[S^T,Q]] + V V^T (rows 0..nu-1 are
// the inputs, rows nu..nu+nx-1 the states) and, after the stage Cholesky, row i of its factor
// [[L^R, 0],[L^S, L^Q]].  Everything an instance carries from stage to stage (the rows of
// L^Q_{k+1}, p_{k+1}) stays in registers.  Cross-row operands are broadcast inside the
// 16-lane row of the wavefront with DPP row_newbcast (a VALU modifier, no LDS traffic).
//
// Per stage (backward in time), with c_i = column i of [B_k A_k] held by lane i:
//   V[i][j]    = sum_{m>=j} c_i[m] L^Q_{k+1}[m][j]       (trmm: broadcast row m of L^Q)
//   Hhat[i][j] = H[i][j] + sum_m V[i][m] V[j][m]          (syrk: broadcast row j of V)
//   chol(Hhat)                                            (potrf, float64, right-looking)
// and the right-hand-side sweep rbar_k = (L^R_k)^{-1}(r_k + B_k^T w), p_k = q_k + A_k^T w -
// L^S_k rbar_k with w = L^Q_{k+1} L^Q_{k+1}^T f_k + p_{k+1}, done as one column-oriented
// substitution over the first nu columns of the factor.
//
// The factor workspace layout is the generic one (stage blocks of lq_internal.hpp), so the
// generic solve and adjoint kernels consume these factors unchanged.
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

// Broadcast lane k's value to the 16 lanes of its row (DPP row_newbcast; k a compile-time
// constant after unrolling).
__device__ __forceinline__ int bc32(int v, int k) {
  switch (k) {
#define BC(K) \
  case K:     \
    return __builtin_amdgcn_update_dpp(0, v, 0x150 + K, 0xF, 0xF, false);
    BC(0) BC(1) BC(2) BC(3) BC(4) BC(5) BC(6) BC(7) BC(8) BC(9) BC(10) BC(11) BC(12) BC(13) BC(14) BC(15)
#undef BC
  }
  return 0;
}
__device__ __forceinline__ double bc(double v, int k) {
  const int lo = bc32(__double2loint(v), k), hi = bc32(__double2hiint(v), k);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float bc(float v, int k) { return __int_as_float(bc32(__float_as_int(v), k)); }

// max over the 16 lanes of a row (quad_perm [1,0,3,2], [2,3,0,1], row_ror 4, row_ror 8)
__device__ __forceinline__ double dpp_d(double v, int ctrl) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  switch (ctrl) {
    case 0xB1:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false);
      break;
    case 0x4E:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false);
      break;
    case 0x124:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x124, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x124, 0xF, 0xF, false);
      break;
    default:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x128, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x128, 0xF, 0xF, false);
      break;
  }
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double rowmax(double v) {
  v = fmax(v, dpp_d(v, 0xB1));
  v = fmax(v, dpp_d(v, 0x4E));
  v = fmax(v, dpp_d(v, 0x124));
  v = fmax(v, dpp_d(v, 0x128));
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

template <int NX, int NU, typename TF, typename TP>
__global__ void __launch_bounds__(64) k_factor_small(int batch, int N, lq_data d, TF* __restrict__ F,
                                                     double* __restrict__ Vws, int32_t* __restrict__ info) {
  constexpr int NUX = NX + NU;
  static_assert(NUX <= 16, "tile exceeds a 16-lane row");
  constexpr int64_t FS = (int64_t)NU * (NU + 1) / 2 + NU + NX * NU + NX * (NX + 1) / 2 + NX;
  constexpr int OLS = NU * (NU + 1) / 2 + NU, OLQ = OLS + NX * NU, ODQ = OLQ + NX * (NX + 1) / 2;
  const int l = threadIdx.x & 63;
  const int i = l & 15;
  const int b = blockIdx.x * 4 + (l >> 4);
  const bool inst = b < batch;
  const bool valid = inst && i < NUX;
  const int64_t bb = inst ? b : 0;
  const bool isu = i < NU;
  const int ic = isu ? i : 0;                       // clamped input row
  const int mi = (!isu && i < NUX) ? i - NU : 0;    // clamped state row

  TF* Fi = F + bb * (N + 1) * FS;
  double* rbar = Vws + bb * ((int64_t)N * NU + (int64_t)(N + 1) * NX);
  double* pv = rbar + (int64_t)N * NU;
  const double* A = d.A + bb * N * NX * NX;
  const double* Bm = d.B + bb * N * NX * NU;
  const double* Q = d.Q + bb * (N + 1) * NX * NX;
  const double* R = d.R + bb * N * NU * NU;
  const double* S = d.S ? d.S + bb * N * NU * NX : nullptr;
  const double* q = d.q + bb * (N + 1) * NX;
  const double* r = d.r + bb * N * NU;
  const double* f = d.f ? d.f + bb * N * NX : nullptr;

  double h[NUX];
  double lq[NX];
  double mydinv = 1.0, pn = 0.0;
  int code = 0;

  // ---- stage N: factor blockdiag(I, sym Q_N) -> blockdiag(I, L^Q_N)
  {
    const double* QN = Q + (int64_t)N * NX * NX;
#pragma unroll
    for (int j = 0; j < NUX; ++j) {
      double v = 0.0;
      if (j < NU) v = (i == j) ? 1.0 : 0.0;
      else if (valid && !isu && (j - NU) <= mi) v = 0.5 * (QN[mi * NX + (j - NU)] + QN[(j - NU) * NX + mi]);
      h[j] = v;
    }
    const int bad = potrf_rows<NUX, NUX>(h, mydinv, i);
    if (bad) code = bad == 2 ? LQ_INFO_NONFINITE : N + 1;
#pragma unroll
    for (int j = 0; j < NUX; ++j) h[j] = rnd<TF>(h[j]);
    mydinv = rnd<TF>(mydinv);
    TF* FN = Fi + (int64_t)N * FS;
    if (valid && !isu) {
#pragma unroll
      for (int j = 0; j < NX; ++j)
        if (j <= mi) FN[OLQ + mi * (mi + 1) / 2 + j] = (TF)h[NU + j];
      FN[ODQ + mi] = (TF)mydinv;
      pn = q[(int64_t)N * NX + mi];
      pv[(int64_t)N * NX + mi] = pn;
    }
#pragma unroll
    for (int j = 0; j < NX; ++j) lq[j] = (j <= mi) ? h[NU + j] : 0.0;
  }

  for (int k = N - 1; k >= 0; --k) {
    const double* Ak = A + (int64_t)k * NX * NX;
    const double* Bk = Bm + (int64_t)k * NX * NU;
    const double* Rk = R + (int64_t)k * NU * NU;
    const double* Qk = Q + (int64_t)k * NX * NX;
    const double* Sk = S ? S + (int64_t)k * NU * NX : nullptr;
    // column i of C = [B_k A_k]
    double c[NX];
#pragma unroll
    for (int m = 0; m < NX; ++m) c[m] = valid ? (isu ? Bk[m * NU + ic] : Ak[m * NX + mi]) : 0.0;
    // lower part of row i of [[R,S],[S^T,Q]]
#pragma unroll
    for (int j = 0; j < NUX; ++j) {
      double v = 0.0;
      if (valid && j <= i) {
        if (isu) v = 0.5 * (Rk[ic * NU + j] + Rk[j * NU + ic]);
        else if (j < NU) v = Sk ? Sk[j * NX + mi] : 0.0;
        else if (k > 0) v = 0.5 * (Qk[mi * NX + (j - NU)] + Qk[(j - NU) * NX + mi]);
      }
      h[j] = v;
    }
    double tq = valid ? (isu ? r[(int64_t)k * NU + ic] : (k > 0 ? q[(int64_t)k * NX + mi] : 0.0)) : 0.0;

    // trmm V = C^T L^Q_{k+1}, and t1 = L^Q_{k+1}^T f_k for the right-hand side
    TP v[NX];
    double t1[NX];
    double fk[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      v[j] = 0;
      t1[j] = 0.0;
      fk[j] = (f && inst) ? f[(int64_t)k * NX + j] : 0.0;
    }
#pragma unroll
    for (int m = 0; m < NX; ++m) {
#pragma unroll
      for (int j = 0; j <= m; ++j) {
        const double L = bc(lq[j], NU + m);
        v[j] += (TP)c[m] * (TP)L;
        if (f) t1[j] = fma(L, fk[m], t1[j]);
      }
    }
    // w = L^Q_{k+1} t1 + p_{k+1} (state lanes), then (rhat, qhat) = (r, q) + C^T w
    double wv = pn;
    if (f) {
#pragma unroll
      for (int j = 0; j < NX; ++j) wv = fma(lq[j], t1[j], wv);
    }
#pragma unroll
    for (int m = 0; m < NX; ++m) tq = fma(c[m], bc(wv, NU + m), tq);
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
    // store factor rows
    TF* Fk = Fi + (int64_t)k * FS;
    if (valid) {
      if (isu) {
#pragma unroll
        for (int j = 0; j < NU; ++j)
          if (j <= ic) Fk[ic * (ic + 1) / 2 + j] = (TF)h[j];
        Fk[NU * (NU + 1) / 2 + ic] = (TF)mydinv;
      } else {
#pragma unroll
        for (int j = 0; j < NU; ++j) Fk[OLS + mi * NU + j] = (TF)h[j];
        if (k > 0) {
#pragma unroll
          for (int j = 0; j < NX; ++j)
            if (j <= mi) Fk[OLQ + mi * (mi + 1) / 2 + j] = (TF)h[NU + j];
          Fk[ODQ + mi] = (TF)mydinv;
        }
      }
    }
    // rbar = L^R^{-1} rhat and p_k = qhat - L^S rbar in one column sweep
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      const double rb = bc(tq * mydinv, j);
      tq = (i > j) ? fma(-h[j], rb, tq) : tq;
    }
    if (valid) {
      if (isu) rbar[(int64_t)k * NU + ic] = tq * mydinv;
      else if (k > 0) pv[(int64_t)k * NX + mi] = tq;
    }
    pn = tq;
#pragma unroll
    for (int j = 0; j < NX; ++j) lq[j] = (j <= mi) ? h[NU + j] : 0.0;
  }
  if (inst && i == 0) info[b] = code;
}

// ------------------------------------------------------------------------------------------
// Solve: forward rollout, then residual + correction sweep / forward correction until the
// relative KKT residual reaches tol.  Lane roles: lane j < nu carries u_j, lane nu + m
// carries x_m and lam_m.

template <int NX, int NU, typename TF>
struct SmallInst {
  static constexpr int NUX = NX + NU;
  static constexpr int64_t FS = (int64_t)NU * (NU + 1) / 2 + NU + NX * NU + NX * (NX + 1) / 2 + NX;
  static constexpr int ODR = NU * (NU + 1) / 2, OLS = ODR + NU, OLQ = OLS + NX * NU, ODQ = OLQ + NX * (NX + 1) / 2;
  int N, i, ic, mi;
  bool isu, valid;
  const TF* F;
  const double *A, *B, *Q, *R, *S, *q, *r, *f, *x0;
  const double *rb0, *p0;
  double *rb2, *p2, *flam;
  double *x, *u, *lam;
  __device__ double LR(int k, int row, int col) const { return (double)F[k * FS + row * (row + 1) / 2 + col]; }
  __device__ double dR(int k, int row) const { return (double)F[k * FS + ODR + row]; }
  __device__ double LS(int k, int row, int col) const { return (double)F[k * FS + OLS + row * NU + col]; }
  __device__ double LQ(int k, int row, int col) const { return (double)F[k * FS + OLQ + row * (row + 1) / 2 + col]; }
};

// mode 0: z = solution with x_0 = x_init, f = f_k, sweep vectors (rb0, p0);
// mode 1: z += correction with x_0 = 0, f = flam, sweep vectors (rb2, p2).
template <int NX, int NU, typename TF>
__device__ void small_fwd(const SmallInst<NX, NU, TF>& s, int mode) {
  constexpr int NUX = NX + NU;
  const int i = s.i, ic = s.ic, mi = s.mi;
  const bool isu = s.isu, valid = s.valid;
  const bool xl = valid && !isu;
  const double* rbv = mode == 0 ? s.rb0 : s.rb2;
  const double* pvv = mode == 0 ? s.p0 : s.p2;
  double xm = (xl && mode == 0) ? s.x0[mi] : 0.0;
  for (int k = 0; k < s.N; ++k) {
    // t_j = rbar_j + (L^S^T x)_j on input lanes
    double t = (valid && isu) ? rbv[(int64_t)k * NU + ic] : 0.0;
#pragma unroll
    for (int m = 0; m < NX; ++m) {
      const double xb = bc(xm, NU + m);
      if (valid && isu) t = fma(s.LS(k, m, ic), xb, t);
    }
    // u' = L^R^{-T} t (back substitution, column oriented), u = -u'
    const double dRi = (valid && isu) ? s.dR(k, ic) : 0.0;
    double uu = 0.0;
#pragma unroll
    for (int j = NU - 1; j >= 0; --j) {
      const double uj = bc(t * dRi, j);
      uu = (i == j) ? uj : uu;
      if (valid && i < j) t = fma(-s.LR(k, j, ic), uj, t);
    }
    const double uval = -uu;
    // x_{k+1} = A x + B u + f
    const double* Ak = s.A + (int64_t)k * NX * NX;
    const double* Bk = s.B + (int64_t)k * NX * NU;
    double xn = 0.0;
    if (xl) xn = mode == 0 ? (s.f ? s.f[(int64_t)k * NX + mi] : 0.0) : s.flam[(int64_t)k * NX + mi];
#pragma unroll
    for (int n = 0; n < NX; ++n) {
      const double xb = bc(xm, NU + n);
      if (xl) xn = fma(Ak[mi * NX + n], xb, xn);
    }
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      const double ub = bc(uval, j);
      if (xl) xn = fma(Bk[mi * NU + j], ub, xn);
    }
    // lam = L^Q_{k+1} (L^Q_{k+1}^T x_{k+1}) + p_{k+1}
    double t2 = 0.0;
#pragma unroll
    for (int m = 0; m < NX; ++m) {
      const double xb = bc(xn, NU + m);
      if (xl && m >= mi) t2 = fma(s.LQ(k + 1, m, mi), xb, t2);
    }
    double lm = xl ? pvv[(int64_t)(k + 1) * NX + mi] : 0.0;
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const double tb = bc(t2, NU + j);
      if (xl && j <= mi) lm = fma(s.LQ(k + 1, mi, j), tb, lm);
    }
    if (valid) {
      if (isu) {
        double* up = s.u + (int64_t)k * NU + ic;
        *up = mode == 0 ? uval : *up + uval;
      } else {
        double* xp = s.x + (int64_t)k * NX + mi;
        double* lp = s.lam + (int64_t)k * NX + mi;
        if (mode == 0) { *xp = xn; *lp = lm; }
        else { *xp += xn; *lp += lm; }
      }
    }
    xm = xn;
    (void)NUX;
  }
}

// Residual of the iterate (returns rel_res, uniform over the instance's lanes); with `sweep`,
// also the backward sweep of the correction right-hand side (rbar2, p2) and flam = -rho_l.
template <int NX, int NU, typename TF>
__device__ double small_resid(const SmallInst<NX, NU, TF>& s, bool sweep) {
  const int i = s.i, ic = s.ic, mi = s.mi, N = s.N;
  const bool isu = s.isu, valid = s.valid;
  const bool xl = valid && !isu;
  double mr = 0.0, mb = 0.0;
  // stage N
  double p2n = 0.0;
  {
    const double* QN = s.Q + (int64_t)N * NX * NX;
    const double xNm = xl ? s.x[(int64_t)(N - 1) * NX + mi] : 0.0;
    double acc = xl ? -s.lam[(int64_t)(N - 1) * NX + mi] : 0.0;
#pragma unroll
    for (int n = 0; n < NX; ++n) {
      const double xb = bc(xNm, NU + n);
      if (xl) acc = fma(0.5 * (QN[mi * NX + n] + QN[n * NX + mi]), xb, acc);
    }
    if (xl) {
      const double qi = s.q[(int64_t)N * NX + mi];
      const double rho = -qi - acc;
      mr = fabs(rho);
      mb = fabs(qi);
      p2n = -rho;
      if (sweep) s.p2[(int64_t)N * NX + mi] = p2n;
    }
  }
  for (int k = N - 1; k >= 0; --k) {
    const double* Ak = s.A + (int64_t)k * NX * NX;
    const double* Bk = s.B + (int64_t)k * NX * NU;
    const double* Rk = s.R + (int64_t)k * NU * NU;
    const double* Qk = s.Q + (int64_t)k * NX * NX;
    const double* Sk = s.S ? s.S + (int64_t)k * NU * NX : nullptr;
    const double xk = xl ? (k > 0 ? s.x[(int64_t)(k - 1) * NX + mi] : s.x0[mi]) : 0.0;
    const double xk1 = xl ? s.x[(int64_t)k * NX + mi] : 0.0;
    const double uk = (valid && isu) ? s.u[(int64_t)k * NU + ic] : 0.0;
    const double lk = xl ? s.lam[(int64_t)k * NX + mi] : 0.0;
    const double lkm = (xl && k > 0) ? s.lam[(int64_t)(k - 1) * NX + mi] : 0.0;
    double au = 0.0, bu = 0.0;    // input row: (R u + S x + B^T lam), and S_0 x_init for ||b||
    double al = -xk1, bl = 0.0;   // state row, dynamics: (A x + B u - x_{k+1}), A_0 x_init
    double ax = -lkm;             // state row, stationarity: (S^T u + Q x + A^T lam - lam_{k-1})
#pragma unroll
    for (int n = 0; n < NX; ++n) {
      const double xb = bc(xk, NU + n);
      const double lb = bc(lk, NU + n);
      if (valid && isu) {
        if (Sk) {
          au = fma(Sk[ic * NX + n], xb, au);
          if (k == 0) bu = fma(Sk[ic * NX + n], xb, bu);
        }
        au = fma(Bk[n * NU + ic], lb, au);
      }
      if (xl) {
        al = fma(Ak[mi * NX + n], xb, al);
        if (k == 0) bl = fma(Ak[mi * NX + n], xb, bl);
        if (k > 0) {
          ax = fma(0.5 * (Qk[mi * NX + n] + Qk[n * NX + mi]), xb, ax);
          ax = fma(Ak[n * NX + mi], lb, ax);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      const double ub = bc(uk, j);
      if (valid && isu) au = fma(0.5 * (Rk[ic * NU + j] + Rk[j * NU + ic]), ub, au);
      if (xl) {
        al = fma(Bk[mi * NU + j], ub, al);
        if (k > 0 && Sk) ax = fma(Sk[j * NX + mi], ub, ax);
      }
    }
    double rhou = 0.0, rhol = 0.0, rhox = 0.0;
    if (valid && isu) {
      const double ri = s.r[(int64_t)k * NU + ic];
      rhou = -ri - au;
      mr = fmax(mr, fabs(rhou));
      mb = fmax(mb, fabs(ri + bu));
    }
    if (xl) {
      const double fi = s.f ? s.f[(int64_t)k * NX + mi] : 0.0;
      rhol = -fi - al;
      mr = fmax(mr, fabs(rhol));
      mb = fmax(mb, fabs(fi + bl));
      if (k > 0) {
        const double qi = s.q[(int64_t)k * NX + mi];
        rhox = -qi - ax;
        mr = fmax(mr, fabs(rhox));
        mb = fmax(mb, fabs(qi));
      }
    }
    if (sweep) {
      // correction right-hand side (r, q, f) = (-rho_u, -rho_x, -rho_l), x_init = 0
      const double fl = -rhol;
      if (xl) s.flam[(int64_t)k * NX + mi] = fl;
      double t1 = 0.0;
#pragma unroll
      for (int m = 0; m < NX; ++m) {
        const double fb = bc(fl, NU + m);
        if (xl && m >= mi) t1 = fma(s.LQ(k + 1, m, mi), fb, t1);
      }
      double w = p2n;
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        const double tb = bc(t1, NU + j);
        if (xl && j <= mi) w = fma(s.LQ(k + 1, mi, j), tb, w);
      }
      double tq = isu ? -rhou : (k > 0 ? -rhox : 0.0);
#pragma unroll
      for (int m = 0; m < NX; ++m) {
        const double wb = bc(w, NU + m);
        if (valid) tq = fma(isu ? Bk[m * NU + ic] : Ak[m * NX + mi], wb, tq);
      }
      // factor row i of stage k: L^R row (input lanes) or L^S row (state lanes)
      double hr[NU];
#pragma unroll
      for (int j = 0; j < NU; ++j) {
        double v = 0.0;
        if (valid) {
          if (isu) v = (j <= ic) ? s.LR(k, ic, j) : 0.0;
          else v = s.LS(k, mi, j);
        }
        hr[j] = v;
      }
      const double dRi = (valid && isu) ? s.dR(k, ic) : 0.0;
#pragma unroll
      for (int j = 0; j < NU; ++j) {
        const double rb = bc(tq * dRi, j);
        tq = (i > j) ? fma(-hr[j], rb, tq) : tq;
      }
      if (valid) {
        if (isu) s.rb2[(int64_t)k * NU + ic] = tq * dRi;
        else if (k > 0) s.p2[(int64_t)k * NX + mi] = tq;
      }
      p2n = tq;
    }
  }
  mr = rowmax(mr);
  mb = rowmax(mb);
  return mb > 0.0 ? mr / mb : mr;
}

template <int NX, int NU, typename TF>
__global__ void __launch_bounds__(64) k_solve_small(SolveArgs a, int N) {
  constexpr int NUX = NX + NU;
  const int l = threadIdx.x & 63;
  const int i = l & 15;
  const int b = blockIdx.x * 4 + (l >> 4);
  const bool inst = b < a.batch;
  const int64_t bb = inst ? b : 0;
  SmallInst<NX, NU, TF> s;
  s.N = N;
  s.i = i;
  s.isu = i < NU;
  s.valid = inst && i < NUX;
  s.ic = s.isu ? i : 0;
  s.mi = (!s.isu && i < NUX) ? i - NU : 0;
  constexpr int64_t FS = SmallInst<NX, NU, TF>::FS;
  s.F = (const TF*)a.F + bb * (N + 1) * FS;
  s.A = a.d.A + bb * N * NX * NX;
  s.B = a.d.B + bb * N * NX * NU;
  s.Q = a.d.Q + bb * (N + 1) * NX * NX;
  s.R = a.d.R + bb * N * NU * NU;
  s.S = a.d.S ? a.d.S + bb * N * NU * NX : nullptr;
  s.q = a.d.q + bb * (N + 1) * NX;
  s.r = a.d.r + bb * N * NU;
  s.f = a.d.f ? a.d.f + bb * N * NX : nullptr;
  s.x0 = a.d.x0 + bb * NX;
  const int64_t vstride = (int64_t)N * NU + (int64_t)(N + 1) * NX;
  s.rb0 = a.V + bb * vstride;
  s.p0 = s.rb0 + (int64_t)N * NU;
  s.rb2 = a.V2 + bb * (vstride + (int64_t)N * NX);
  s.p2 = s.rb2 + (int64_t)N * NU;
  s.flam = s.p2 + (int64_t)(N + 1) * NX;
  s.x = a.x + bb * N * NX;
  s.u = a.u + bb * N * NU;
  s.lam = a.lam + bb * N * NX;

  if (inst) small_fwd<NX, NU, TF>(s, 0);
  int it = 0;
  double rel = 0.0;
  bool have = false;
  bool act = inst && (a.check || a.max_it > 0);
  while (__any(act)) {
    if (act) {
      const bool more = it < a.max_it;
      rel = small_resid<NX, NU, TF>(s, more);
      have = true;
      if (!(rel > a.tol) || !more) {
        act = false;
      } else {
        small_fwd<NX, NU, TF>(s, 1);
        ++it;
      }
    }
  }
  if (inst && i == 0) {
    if (a.rel_res) a.rel_res[b] = have ? rel : NAN;
    if (a.iters) a.iters[b] = it;
    if (a.info) {
      const int cur = a.info[b];
      if (cur <= 0) {
        int code = 0;
        if (have && !isfinite(rel)) code = LQ_INFO_NONFINITE;
        else if (have && a.max_it > 0 && rel > a.tol) code = LQ_INFO_NOT_CONVERGED;
        else if (cur == LQ_INFO_NONFINITE) code = cur;
        a.info[b] = code;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Dispatch table of the compiled (nx, nu) shapes.

template <int NX, int NU>
hipError_t factor_shape(lq_mode mode, int batch, int N, const lq_data& d, void* F, double* V, int32_t* info,
                        hipStream_t st) {
  const dim3 grid((batch + 3) / 4), block(64);
  if (mode == LQ_F64)
    hipLaunchKernelGGL((k_factor_small<NX, NU, double, double>), grid, block, 0, st, batch, N, d, (double*)F, V, info);
  else
    hipLaunchKernelGGL((k_factor_small<NX, NU, float, float>), grid, block, 0, st, batch, N, d, (float*)F, V, info);
  return hipGetLastError();
}

template <int NX, int NU>
hipError_t solve_shape(lq_mode mode, int N, const SolveArgs& a, hipStream_t st) {
  const dim3 grid((a.batch + 3) / 4), block(64);
  if (mode == LQ_F64)
    hipLaunchKernelGGL((k_solve_small<NX, NU, double>), grid, block, 0, st, a, N);
  else
    hipLaunchKernelGGL((k_solve_small<NX, NU, float>), grid, block, 0, st, a, N);
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
#define X(a, b) \
  if (nx == a && nu == b) return factor_shape<a, b>(mode, batch, N, d, F, V, info, st);
  LQ_SMALL_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_solve_small(lq_mode mode, int N, int nx, int nu, const SolveArgs& a, hipStream_t st) {
  if (a.rhs != RHS_PRIMAL) return hipErrorInvalidValue;
#define X(a_, b_) \
  if (nx == a_ && nu == b_) return solve_shape<a_, b_>(mode, N, a, st);
  LQ_SMALL_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace lq
