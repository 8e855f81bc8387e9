// Device code of the matrix-core tile factor sweep, shared by the factor kernel and the
// checkpointed solve kernels (which recompute factor segments with it).
//
// Matrix-core tile kernel of the factor sweep for medium and large stage sizes.
//
// One workgroup per instance (or a persistent grid pulling instances longest first), one
// wavefront per 16-wide tile column of the stage matrix.  The input block and the state block
// are each padded to a multiple of 16 (TU = ceil(nu/16), TX = ceil(nx/16) tiles, T = TU + TX)
// with an identity diagonal and zero coupling, which leaves the factors of the real rows and
// columns unchanged.
//
// Per stage, backward in time (paper, Alg. "factor-block-column-riccati" with one interval):
//   W = V^T = (L^Q_{k+1})^T C,  C = [B_k A_k]                   (trmm, nx x nux)
//   Hhat = [[R,S],[S^T,Q]] + W^T W                              (syrk)
//   chol(Hhat) = [[L^R, 0],[L^S, L^Q]]                           (blocked potrf, float64)
// Matrix-core layout: a 16x16 fragment of a 64-lane wavefront holds element (row(t), c) of the
// tile in slot t of lane 16 g + c, with row(t) = 4t + g for float64 and 4g + t for float32
// products.  That layout is also the B operand of the next product when the contraction index
// of instruction s is row(s), so every product here has the form Y += op(M) X with X a fragment
// in registers and M a tile in LDS.  Wavefront a owns tile column a: its C tiles C(m', a), its
// W tiles W(m, a) and the upper tiles G(b, a) = Hhat(b, a), b <= a.
//   trmm   W(m, a)  = sum_{m' >= m} U^Q(m, m') C(m', a)   with U^Q = (L^Q_{k+1})^T in LDS,
//   syrk   G(b, a) += W(m, b)^T W(m, a), streamed over 16-row slabs m of W through LDS,
//   potrf  per pivot tile j: the owner of column j factors G(j, j) (row per lane, DPP
//          broadcasts, float64) and inverts it; the owners of columns a > j form
//          U(j, a) = L_jj^{-1} G(j, a) = L(a, j)^T on the matrix cores and publish it in LDS;
//          then G(b, a) -= U(j, b)^T U(j, a) for j < b <= a.
// The tiles U(j, a) of the state block are L^Q_k transposed: they stay in LDS as the U^Q operand
// of the next stage.  The right-hand-side sweep (rbar_k, p_k) runs in float64 beside it, as in
// the other factor kernels, and the factor blocks use the shared workspace layout.
//
// Precision: TP is the type of the stage products: float64; float32 (mixed mode: operands the
// float32-rounded L^Q and C, float32 accumulation); or bf16 operands with float32 accumulation
// (rounded from the float32 L^Q, C and W).  The potrf and everything after it is float64 and the
// factors are rounded to TF for storage.
#pragma once
#include <math.h>

#include <type_traits>

#include "lq_internal.hpp"

namespace lq {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Broadcast lane k of each 16-lane row to the whole row (k a constant after unrolling).
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

// Value of lane l (wave-uniform l) for every lane.
__device__ __forceinline__ double lane_bcast(double v, int l) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, l), hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __hiloint2double(hi, lo);
}

// Order the LDS accesses of one wavefront (its DS operations complete in issue order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}

template <typename TP>
struct MM;
template <>
struct MM<double> {
  typedef d4 V;
  static __device__ __forceinline__ int row(int t, int g) { return 4 * t + g; }
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct MM<float> {
  typedef f4 V;
  static __device__ __forceinline__ int row(int t, int g) { return 4 * g + t; }
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// bf16 operands with float32 accumulation: one 16x16x16 instruction per tile product.  Operand
// slot i of lane 16 g + c holds contraction index 4 g + i, so a float32 fragment (row 4g + t in
// slot t) is directly the B operand and the A operand is four consecutive entries of a row.
struct BF16 {};
typedef __bf16 b4 __attribute__((ext_vector_type(4)));
template <>
struct MM<BF16> {
  typedef f4 V;
  static __device__ __forceinline__ int row(int t, int g) { return 4 * g + t; }
};

// Element type of W slabs and of converted C fragments for a product type.
template <typename TP>
struct Elem {
  typedef TP type;
};
template <>
struct Elem<BF16> {
  typedef float type;
};

// Leading dimensions of LDS tiles (padded against bank conflicts; float rows stay 16-byte aligned).
template <typename T>
struct Ld;
template <>
struct Ld<double> {
  static constexpr int v = 17;
};
template <>
struct Ld<float> {
  static constexpr int v = 20;
};

// acc += op(M) X for a 16x16 LDS tile M (leading dimension ld) and a fragment X;
// TR = false: op(M) = M, TR = true: op(M) = M^T.  NEG subtracts.
template <typename TP, bool TR, bool NEG = false, typename TM>
__device__ __forceinline__ typename MM<TP>::V tmm(typename MM<TP>::V acc, const TM* M, int ld,
                                                   const typename MM<TP>::V& X, int g, int c) {
  if constexpr (std::is_same<TP, BF16>::value) {
    b4 av, bv;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float m = (float)(TR ? M[(4 * g + i) * ld + c] : M[c * ld + 4 * g + i]);
      av[i] = (__bf16)(NEG ? -m : m);
      bv[i] = (__bf16)X[i];
    }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kk = MM<TP>::row(s, g);
      TP av = (TP)(TR ? M[kk * ld + c] : M[c * ld + kk]);
      if (NEG) av = -av;
      acc = MM<TP>::mma(av, X[s], acc);
    }
    return acc;
  }
}

// Right-looking Cholesky of a 16x16 tile held one row per lane (lane c of each 16-lane row:
// row c in h).  Returns 0, or for the first failing pivot 1 (finite, not positive) or 2 (not
// finite); failed pivots are replaced by 1, so later pivots of a failed tile are meaningless.  On
// return h[0..c] is row c of L and dinv = 1 / L[c][c].
// Only the first n (wave-uniform) pivots are real: rows and columns n..15 are the identity
// padding with zero coupling, whose factor is the identity.  The pivots run in chunks of four,
// each chunk under a uniform branch, and the chunks past the last real pivot are skipped (within
// a chunk a padding pivot changes nothing but its own diagonal, which stays 1 to rounding).
// Each pivot updates the next pivot's column first and starts its 1/sqrt before its other
// trailing updates, so the next pivot's chain overlaps them.
// 1 / sqrt(d): the hardware estimate y (about 5e-8 relative) with one third-order correction,
// y (1 + e / 2 + 3 e^2 / 8), e = 1 - d y^2 (error O(e^3), so rounding-limited), folded into the
// products that use it; the column is broadcast from before the diagonal lane's select, and the
// failure handling stays off the chain (a second pass, see chol16_pass), which keeps the
// per-pivot dependency chain at about eight instructions.
// SAFE = false: the pivot chain without the failure handling (a pivot that is not positive and
// finite leaves non-finite entries, and the caller factors the tile again with SAFE = true, which
// replaces it by 1); the returned classification is the same in both.
template <bool SAFE>
__device__ __forceinline__ int chol16_pass(double (&h)[16], double& dinv, int c, int n) {
  // the first failing pivot classifies the tile (see the comment above)
  int kind = 0;
  dinv = 1.0;  // rows of skipped padding pivots keep it
  double dj = bc(h[0], 0), y = __builtin_amdgcn_rsq(dj);
#pragma unroll
  for (int j0 = 0; j0 < 16; j0 += 4) {
    if (j0 < n) {
#pragma unroll
      for (int j = j0; j < j0 + 4; ++j) {
        const bool good = dj > 0.0 && dj <= 1.7976931348623157e308;
        kind = kind ? kind : (good ? 0 : (isfinite(dj) ? 1 : 2));
        // x (1 + e p) with e = 1 - dj y^2, p = 1/2 + 3 e / 8, as fma(x e, p, x)
        const double t = dj * y;
        const double e = fma(-t, y, 1.0);
        const double pp = fma(e, 0.375, 0.5);
        const double hy = h[j] * y;
        // column j of L below the pivot (a failed pivot counts as 1: the column is kept)
        double hs = fma(hy * e, pp, hy);
        double dg = fma(t * e, pp, t), di = fma(y * e, pp, y);
        if (SAFE) {
          hs = good ? hs : h[j];
          dg = good ? dg : 1.0;
          di = good ? di : 1.0;
        }
        // look-ahead: the next pivot's column first, and its 1/sqrt estimate, then the other
        // updates, which issue while that estimate is in flight.  The next pivot is lane j+1's
        // updated entry fma(-L[j+1][j], L[j+1][j], h[j+1]), formed on every lane from the two
        // broadcasts (the same operands, so the same value) instead of broadcast after the update.
        if (j + 1 < 16) {
          const double b = bc(hs, j + 1), hold = bc(h[j + 1], j + 1);
          h[j + 1] = fma(-hs, b, h[j + 1]);
          dj = fma(-b, b, hold);
          y = __builtin_amdgcn_rsq(dj);
        }
#pragma unroll
        for (int kk = j + 2; kk < 16; ++kk) h[kk] = fma(-hs, bc(hs, kk), h[kk]);
        h[j] = (c == j) ? dg : hs;
        dinv = (c == j) ? di : dinv;
      }
    }
  }
  return kind;
}

// Columns 4g .. 4g+3 of row c of X = L^{-1} in lane c of 16-lane row g, from L held one row per
// lane (h[k] = L[c][k] for k <= c, as chol16 leaves it) and dinv = 1 / L[c][c]:
//   X[c][q] = dinv delta_cq - sum_{k<c} (dinv L[c][k]) X[k][q],
// with the rows X[k] taken in order k = 0, 1, ... by row broadcasts (row k is final once the steps
// before it are done).  Each lane group forms its own four columns; entries above the diagonal
// are zero and stay zero, so all columns run the same steps.  Registers and DPP only.  With n real
// pivots (the rest identity padding, as in chol16) the steps k >= n - 1 change nothing.
__device__ __forceinline__ void inv16_cols4(double (&x)[4], const double (&h)[16], double dinv, int c, int g, int n) {
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) x[qq] = 4 * g + qq == c ? dinv : 0.0;
  // steps in chunks of four under uniform branches, as in chol16 (extra steps on padding rows are
  // exact no-ops: their multipliers are zero)
#pragma unroll
  for (int k0 = 0; k0 < 15; k0 += 4) {
    if (k0 < n - 1) {
#pragma unroll
      for (int k = k0; k < k0 + 4 && k < 15; ++k) {
        const double mk = k < c ? dinv * h[k] : 0.0;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) x[qq] = fma(-mk, bc(x[qq], k), x[qq]);
      }
    }
  }
}

// Element q = 4 g + qq of a 16-element per-lane row, for the lane's group g.
__device__ __forceinline__ double pick4(const double (&v)[16], int g, int qq) {
  const double a0 = v[qq], a1 = v[4 + qq], a2 = v[8 + qq], a3 = v[12 + qq];
  return g == 0 ? a0 : g == 1 ? a1 : g == 2 ? a2 : a3;
}

// Factor sweep of stages kb-1 down to ka of one instance (TMAX >= T wavefronts own the tile
// columns, any further ones only take part in the cooperative loops and barriers).  kb = N starts
// with chol(Q_N); kb < N starts from the stored L^Q_kb of block `from`.  Stage k's factor block
// goes to dst(k) (nullptr: not stored).  With Vi (only for kb = N, ka = 0) the float64 sweep of
// the right-hand side (rbar, p) runs beside it.  The factor arithmetic does not depend on the range
// or on Vi, so a segment recomputed from its stored right end reproduces the full sweep's blocks
// bit for bit (the U^Q tiles loaded from a stored block equal the ones the sweep leaves in LDS:
// rounded to TF, zero below the diagonal and off the real rows, identity on the padding, whose
// value never reaches a real entry).
template <int TMAX, typename TF, typename TP, bool ORD = false, typename Dst>
__device__ __forceinline__ void factor_tile_range(const Desc& D, const lq_data& d, int ka, int kb, Dst&& dst,
                                                  const TF* __restrict__ from, double* __restrict__ Vi,
                                                  unsigned char* lds, int& s_info) {
  constexpr bool F64 = std::is_same<TP, double>::value;
  constexpr bool EARLY_IN = TMAX <= 5;  // input side of a stage inside its potrf (see input_side)
  typedef typename MM<TP>::V PV;
  typedef typename Elem<TP>::type TE;  // W slabs, converted C fragments
  constexpr int LQ = Ld<TF>::v, LW = Ld<TE>::v, LD = Ld<double>::v;
  const int N = D.N, nx = D.nx, nu = D.nu;
  const int TU = (nu + 15) >> 4, TX = (nx + 15) >> 4, T = TU + TX;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wavefront index (uniform)
  const bool own = w < T;
  const int a = w;
  const TileLds L = tile_lds(TU, TX, F64);
  TF* LQB = (TF*)(lds + L.oLQB);
  double* UP = (double*)(lds + L.oUP);
  double* XP = (double*)(lds + L.oXP);
  TE* WS = (TE*)(lds + L.oWS);
  double* DI = (double*)(lds + L.oDI);
  double* SC = (double*)(lds + L.oSC);
  // per-wavefront relayout tile of the mixed mode, in the slab region (dead at that point)
  double* CV = (double*)(lds + L.oXP) + w * 16 * LD;
  double* pv = (double*)(lds + L.oVec);  // p_{k+1}, then p_k   [16 TX]
  double* wv = pv + 16 * TX;             // w                   [16 TX]
  double* t1 = wv + 16 * TX;             //                     [16 TX]
  double* rq = t1 + 16 * TX;             // (rhat, qhat)        [16 T]
  double* dv = rq + 16 * T;              // 1 / diag of L       [16 T]
  double* rb = dv + 16 * T;              // rbar                [16 TU]
  // U^Q tile (m, m'), m <= m' (state block), row-major; panels U(j, a), a >= j
  auto lqb = [&](int m, int mp) { return LQB + (mp * (mp + 1) / 2 + m) * 16 * LQ; };
  auto upan = [&](int j, int aa) { return UP + (j * T + aa) * 16 * LD; };
  auto xpan = [&](int j, int aa) -> double* {
    if constexpr (F64) return (double*)lqb(j - TU, aa - TU);
    else return XP + ((j & 1) * T + aa) * 16 * LD;
  };
  auto pan = [&](int j, int aa) { return j < TU ? upan(j, aa) : xpan(j, aa); };
  auto wsl = [&](int m, int aa) { return WS + ((m & 1) * T + aa) * 16 * LW; };

  const int oDR = off_dR(nx, nu), oLS = off_LS(nx, nu), oLQ = off_LQ(nx, nu), oDQ = off_dQ(nx, nu);
  const double* Ag = d.A + D.oA;
  const double* Bg = d.B + D.oB;
  const double* Qg = d.Q + D.oQ;
  const double* Rg = d.R + D.oR;
  const double* Sg = d.S ? d.S + D.oS : nullptr;
  const double* qg = d.q + D.oq;
  const double* rg = d.r + D.or_;
  const double* fg = d.f ? d.f + D.of : nullptr;
  const bool rhs = Vi != nullptr;
  double* rbar_g = Vi;
  double* p_g = rhs ? Vi + (int64_t)N * nu : nullptr;

  if (tid == 0) s_info = 0;
  if (rhs) {
    for (int i = tid; i < 16 * TX; i += nt) {
      const double v = i < nx ? qg[(int64_t)N * nx + i] : 0.0;
      pv[i] = v;
      if (i < nx) p_g[(int64_t)N * nx + i] = v;
    }
  }
  if (kb < N) {
    // U^Q tiles of L^Q_kb from the stored packed block: tile (m, m') holds U^Q[j][i] = L^Q[i][j]
    for (int e = tid; e < TX * (TX + 1) / 2 * 256; e += nt) {
      const int tl = e >> 8, j0 = (e >> 4) & 15, i0 = e & 15;
      int mp = 0;
      while ((mp + 1) * (mp + 2) / 2 <= tl) ++mp;
      const int j = 16 * (tl - mp * (mp + 1) / 2) + j0, i = 16 * mp + i0;
      LQB[tl * 16 * LQ + j0 * LQ + i0] = (i < nx && j <= i) ? from[oLQ + i * (i + 1) / 2 + j] : (TF)(i == j ? 1 : 0);
    }
  }
  __syncthreads();

  for (int k = kb == N ? N : kb - 1; k >= ka; --k) {
    // Lane coordinates re-derived per stage from an opaque copy of the thread index: without it
    // the compiler hoists every per-lane address and select of the unrolled tile loops out of the
    // stage loop and runs out of registers.
    int ltid = tid;
    asm volatile("" : "+v"(ltid));
    const int lane = ltid & 63, g = lane >> 4, c = lane & 15;
    const double* Ak = Ag + (int64_t)k * nx * nx;
    const double* Bk = Bg + (int64_t)k * nx * nu;
    const double* Qk = Qg + (int64_t)k * nx * nx;
    const double* Rk = Rg + (int64_t)k * nu * nu;
    const double* Sk = Sg ? Sg + (int64_t)k * nu * nx : nullptr;
    // Symmetric part of [[R,S],[S^T,Q]] (padded) in the float64 fragment layout, tile (bb, aa):
    // at stage N only the state block (Q_N), at stage 0 only the input rows.
    auto load_h = [&](int bb, int aa) -> d4 {
      // branch-free within the wavefront: clamped addresses, out-of-range entries zeroed through
      // an opaque mask (a select on a loaded value compiles to a branch around the load, which
      // waits for it at once), the identity of the padding added
      d4 h = d4{0, 0, 0, 0};
      const bool bu = bb < TU, au = aa < TU;
      const int ib = (bu ? 16 * bb : 16 * (bb - TU)) + g, jb = (au ? 16 * aa : 16 * (aa - TU)) + c;
      if (bu && au) {
        if (k < N) {
          const int jc = min(jb, nu - 1);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int ii = ib + 4 * t, ic = min(ii, nu - 1);
            const bool in = ii < nu && jb < nu;
            h[t] = keep_if<ORD>(in, 0.5 * (Rk[ic * nu + jc] + Rk[jc * nu + ic])) + (!in && ii == jb ? 1.0 : 0.0);
          }
        }
      } else if (bu) {
        if (k < N && Sk) {
          const int jc = min(jb, nx - 1);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int ii = ib + 4 * t, ic = min(ii, nu - 1);
            h[t] = keep_if<ORD>(ii < nu && jb < nx, Sk[ic * nx + jc]);
          }
        }
      } else if (k > 0) {
        const int jc = min(jb, nx - 1);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int ii = ib + 4 * t, ic = min(ii, nx - 1);
          const bool in = ii < nx && jb < nx;
          h[t] = keep_if<ORD>(in, 0.5 * (Qk[ic * nx + jc] + Qk[jc * nx + ic])) + (!in && ii == jb ? 1.0 : 0.0);
        }
      }
      return h;
    };

    d4 G[TMAX];
#pragma unroll
    for (int bb = 0; bb < TMAX; ++bb) G[bb] = d4{0, 0, 0, 0};
    if (k == N) {
      if (own) {
#pragma unroll
        for (int bb = 0; bb < TMAX; ++bb)
          if (bb <= a) G[bb] = load_h(bb, a);
      }
    } else {
      // Up to five tile columns the H tiles are fetched here, so that their reads overlap the
      // trmm below (for more columns the registers they would hold across it are not free).
      constexpr bool EARLY_H = TMAX <= 5;
      if constexpr (EARLY_H) {
        if (own) {
#pragma unroll
          for (int bb = 0; bb < TMAX; ++bb)
            if (bb <= a) G[bb] = load_h(bb, a);
        }
      }
      // ---- w = L^Q_{k+1} (L^Q_{k+1})^T f_k + p_{k+1}
      if (!rhs) {
      } else if (fg) {
        // t1 = (L^Q_{k+1})^T f_k, then w = L^Q_{k+1} t1 + p_{k+1}: every entry is summed by four
        // neighbouring lanes (every fourth term each, so that the serial chains are a quarter as
        // long) and combined by two shuffles; the trip count of the outer loop is uniform
        const double* fk = fg + (int64_t)k * nx;
        const int sl = tid & 3;
        for (int e0 = 0; e0 < 16 * TX; e0 += nt >> 2) {
          const int e = e0 + (tid >> 2);
          double s = 0.0;
          if (e < nx)
            for (int i = e + sl; i < nx; i += 4) s = fma((double)lqb(e >> 4, i >> 4)[(e & 15) * LQ + (i & 15)], fk[i], s);
          s += __shfl_xor(s, 1);
          s += __shfl_xor(s, 2);
          if (sl == 0 && e < nx) t1[e] = s;
        }
        __syncthreads();
        for (int e0 = 0; e0 < 16 * TX; e0 += nt >> 2) {
          const int e = e0 + (tid >> 2);
          double s = 0.0;
          if (e < nx)
            for (int j = sl; j <= e; j += 4) s = fma((double)lqb(j >> 4, e >> 4)[(j & 15) * LQ + (e & 15)], t1[j], s);
          s += __shfl_xor(s, 1);
          s += __shfl_xor(s, 2);
          if (sl == 0 && e < 16 * TX) wv[e] = pv[e] + s;
        }
      } else {
        for (int i = tid; i < 16 * TX; i += nt) wv[i] = pv[i];
      }
      __syncthreads();
      // ---- C tiles of column a (float64 for (rhat, qhat) = (r, q) + C^T w, TP for the trmm)
      // ---- trmm + syrk, streamed over the 16-row slabs m of W.  The fragments C(m', a) are read
      // from global memory two tiles ahead (cache-resident after the first slab); the first slab,
      // which touches every C tile once, also accumulates (C^T w)_a in float64.
      const bool ucol = a < TU;
      const int col = ucol ? 16 * a + c : 16 * (a - TU) + c;
      const int ldc = ucol ? nu : nx;
      const int ncol = ucol ? nu : nx;
      const bool colok = col < ncol;
      const int r0 = MM<TP>::row(0, g);  // row(t, g) = r0 + row(t, 0)
      const double* cb = (ucol ? Bk : Ak) + min(col, ncol - 1);
      // right-hand-side entry of this lane's column (r_k or q_k), read now and used after the
      // trmm; the address is selected, not the value
      const double base_raw = rhs ? *(ucol ? rg + (int64_t)k * nu + min(col, nu - 1)
                                           : qg + (int64_t)k * nx + min(col, nx - 1))
                                  : 0.0;
      // (always issued, with a clamped slab index where the slab lies past the last one: a load
      // under a condition, or a select on its value, makes the wavefront wait for it at once)
      auto load_c = [&](int mp) -> d4 {
        d4 v;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int row = r0 + 16 * mp + MM<TP>::row(t, 0);
          v[t] = keep_if<ORD>(colok && row < nx, cb[min(row, nx - 1) * ldc]);
        }
        return v;
      };
      PV Gs[TMAX];
#pragma unroll
      for (int bb = 0; bb < TMAX; ++bb) Gs[bb] = PV{0, 0, 0, 0};
      double part = 0.0;
      // one slab, with the C fragments of tiles m and m + 1 read by the caller (as a function of
      // its own the slab step compiles to a tighter schedule at ten tile columns: large workload
      // factor 110.7 -> 103.8 ms, measured)
      auto slab = [&](int m, d4 cur, d4 nxt) {
        PV Wf = PV{0, 0, 0, 0};
        if (own) {
          // unrolled, with an exit instead of a guarded body, so that the fragments in flight
          // rotate by renaming: a register copy of a fragment would wait for its load
#pragma unroll
          for (int q = 0; q < TMAX - 1; ++q) {
            const int mp = m + q;
            if (mp >= TX) break;
            const d4 nn = load_c(min(mp + 2, TX - 1));
            if (rhs && m == 0) {
#pragma unroll
              for (int t = 0; t < 4; ++t) part = fma(cur[t], wv[16 * mp + r0 + MM<TP>::row(t, 0)], part);
            }
            PV cx;
#pragma unroll
            for (int t = 0; t < 4; ++t) cx[t] = (TE)cur[t];
            Wf = tmm<TP, false>(Wf, lqb(m, mp), LQ, cx, g, c);
            cur = nxt;
            nxt = nn;
          }
          TE* ws = wsl(m, a);
#pragma unroll
          for (int t = 0; t < 4; ++t) ws[MM<TP>::row(t, g) * LW + c] = Wf[t];
        }
        __syncthreads();
        if (own) {
#pragma unroll
          for (int bb = 0; bb < TMAX; ++bb)
            if (bb <= a && (k > 0 || bb < TU)) Gs[bb] = tmm<TP, true>(Gs[bb], wsl(m, bb), LW, Wf, g, c);
        }
      };
      for (int m = 0; m < TX; ++m) slab(m, load_c(m), load_c(min(m + 1, TX - 1)));
      __syncthreads();
      if (rhs && own) {
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (g == 0) rq[16 * a + c] = keep_if<ORD>(ucol ? col < nu : (k > 0 && col < nx), base_raw) + part;
      }
      // ---- G = [[R,S],[S^T,Q]] + W^T W in float64 (mixed: float32 layout -> float64 layout)
      if (own) {
#pragma unroll
        for (int bb = 0; bb < TMAX; ++bb) {
          if (bb <= a) {
            const d4 h = EARLY_H ? G[bb] : load_h(bb, a);
            if constexpr (F64) {
              G[bb] = h + Gs[bb];
            } else {
#pragma unroll
              for (int t = 0; t < 4; ++t) CV[MM<TP>::row(t, g) * LD + c] = (double)Gs[bb][t];
              wave_sync();
#pragma unroll
              for (int t = 0; t < 4; ++t) G[bb][t] = h[t] + CV[MM<double>::row(t, g) * LD + c];
              wave_sync();
            }
          }
        }
      }
    }

    // ---- the input side of stage k, by wavefront 0 alone once the last input pivot tile is done
    // (up to five tile columns; with more, wavefront 0 alone would take longer than the state
    // pivots' slot and share its SIMD with them: there it runs after the potrf on every wavefront)
    // (L^R_k, L^S_k and their diagonal are final then and no later pivot touches their panels;
    // wavefront 0 has no later pivot work, so this runs beside the state pivots):
    //   rbar_k = (L^R_k)^{-1} rhat,  p_k = qhat - L^S_k rbar_k (rounded factors, float64),
    //   and the L^R_k, 1/diag L^R_k, L^S_k parts of the stage's factor block.
    auto input_side = [&]() {
      if (rhs) {
        // one row per lane, 64 rows per pass
        for (int i0 = 0; i0 < nu; i0 += 64) {
          const int i = i0 + lane;
          double acc = i < nu ? rq[i] : 0.0;
          const double di = i < nu ? (double)(TF)dv[i] : 0.0;
          // contributions of the rows of earlier passes
          for (int jj = 0; jj < i0; ++jj)
            if (i < nu) acc -= (double)(TF)upan(jj >> 4, i >> 4)[(jj & 15) * LD + (i & 15)] * rb[jj];
          // (the coefficient is read on every lane, at a clamped row, and applied through a select:
          // a read under a condition waits for itself at once)
          const int ic = min(i, nu - 1);
          for (int jj = i0; jj < nu && jj < i0 + 64; ++jj) {
            const double y = lane_bcast(acc * di, jj - i0);
            const double lv = (double)(TF)upan(jj >> 4, ic >> 4)[(jj & 15) * LD + (ic & 15)];
            acc = (i > jj && i < nu) ? acc - lv * y : acc;
          }
          if (i < nu) {
            const double v = acc * di;
            rb[i] = v;
            rbar_g[(int64_t)k * nu + i] = v;
          }
          wave_sync();
        }
        if (k > 0) {
          for (int i = lane; i < nx; i += 64) {
            double s = rq[16 * TU + i];
            for (int jj = 0; jj < nu; ++jj)
              s -= (double)(TF)upan(jj >> 4, TU + (i >> 4))[(jj & 15) * LD + (i & 15)] * rb[jj];
            pv[i] = s;
            p_g[(int64_t)k * nx + i] = s;
          }
        }
      }
      TF* Fi = dst(k);
      if (Fi) {
        for (int i = 0; i < nu; ++i)
          for (int jj = lane; jj <= i; jj += 64)
            Fi[i * (i + 1) / 2 + jj] = (TF)upan(jj >> 4, i >> 4)[(jj & 15) * LD + (i & 15)];
        for (int i = lane; i < nu; i += 64) Fi[oDR + i] = (TF)dv[i];
        for (int e = lane; e < nx * nu; e += 64) {
          const int i = e / nu, jj = e - i * nu;
          Fi[oLS + e] = (TF)upan(jj >> 4, TU + (i >> 4))[(jj & 15) * LD + (i & 15)];
        }
      }
    };

    // ---- blocked potrf over the pivot tiles [j0, j1)
    const int j0 = k == N ? TU : 0, j1 = k == 0 ? TU : T;
    for (int j = j0; j < j1; ++j) {
      if (own && a == j) {
        // the diagonal step is the stage's critical path: its wavefront goes first among the
        // wavefronts that share its SIMD (this workgroup's and co-resident ones) until it is done
        __builtin_amdgcn_s_setprio(3);
        // lane coordinates re-derived here so that the diagonal step's per-lane addresses and
        // masks are not kept live across the whole pivot loop
        int dt = tid;
        asm volatile("" : "+v"(dt));
        const int lane = dt & 63, g = lane >> 4, c = lane & 15;
        d4 Gj = G[0];
#pragma unroll
        for (int bb = 1; bb < TMAX; ++bb)
          if (bb == j) Gj = G[bb];
#pragma unroll
        for (int t = 0; t < 4; ++t) SC[MM<double>::row(t, g) * LD + c] = Gj[t];
        wave_sync();
        double dinv = 0.0;
        // real pivots of the tile (the rest is padding)
        const int nreal = __builtin_amdgcn_readfirstlane(min(16, j < TU ? nu - 16 * j : nx - 16 * (j - TU)));
        {
          double h[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) h[q] = SC[c * LD + q];
          int bad = chol16_pass<false>(h, dinv, c, nreal);
          if (__builtin_amdgcn_readfirstlane(bad) != 0) {
            // a pivot failed (the classification is the same on every lane): again from the
            // staged tile, with failed pivots replaced by 1
#pragma unroll
            for (int q = 0; q < 16; ++q) h[q] = SC[c * LD + q];
            bad = chol16_pass<true>(h, dinv, c, nreal);
          }
          if (bad && lane == 0 && s_info == 0) s_info = bad == 2 ? LQ_INFO_NONFINITE : k + 1;
          // U(j, j) = L_jj^T into its panel / the L^Q tiles
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            const int q = 4 * g + qq;
            const double l = q <= c ? pick4(h, g, qq) : 0.0;
            if (j < TU) upan(j, j)[q * LD + c] = l;
            else lqb(j - TU, j - TU)[q * LQ + c] = (TF)l;
          }
          if (g == 0) dv[16 * j + c] = dinv;
          // X = L_jj^{-1}; DI holds X^T row-major (row q = column q of X: DI[q][c] = X[c][q]);
          // the last tile column has no panel to the right of it and needs no inverse (at stage 0
          // the last input tile still has the state columns' panels, L^S_0)
          if (j + 1 < T) {
            double x[4];
            inv16_cols4(x, h, dinv, c, g, nreal);
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) DI[(4 * g + qq) * LD + c] = x[qq];
          }
        }
        // column j is complete: none of its tiles is read again, and redefining them here lets
        // the diagonal step reuse their registers
#pragma unroll
        for (int bb = 0; bb < TMAX; ++bb) G[bb] = d4{0, 0, 0, 0};
        __builtin_amdgcn_s_setprio(0);
      }
      __syncthreads();
      d4 Uf = d4{0, 0, 0, 0};
      if (own && a > j) {
#pragma unroll
        for (int bb = 0; bb < TMAX; ++bb)
          if (bb == j) Uf = tmm<double, true>(Uf, DI, LD, G[bb], g, c);
        double* P = pan(j, a);
#pragma unroll
        for (int t = 0; t < 4; ++t) P[MM<double>::row(t, g) * LD + c] = Uf[t];
        if constexpr (!F64) {
          if (j >= TU) {
            TF* Qt = lqb(j - TU, a - TU);
#pragma unroll
            for (int t = 0; t < 4; ++t) Qt[MM<double>::row(t, g) * LQ + c] = (TF)Uf[t];
          }
        }
      }
      __syncthreads();
      if constexpr (EARLY_IN) {
        if (k < N && j == TU - 1 && w == 0) input_side();
      }
      if (own && a > j) {
#pragma unroll
        for (int bb = 0; bb < TMAX; ++bb)
          if (bb > j && bb <= a && (k > 0 || bb < TU)) G[bb] = tmm<double, true, true>(G[bb], pan(j, bb), LD, Uf, g, c);
      }
    }
    __syncthreads();

    if constexpr (!EARLY_IN) {
      // ---- rbar_k = (L^R_k)^{-1} rhat,  p_k = qhat - L^S_k rbar_k (rounded factors, float64)
      if (rhs && k < N) {
        if (w == 0) {
          // one row per lane, 64 rows per pass
          for (int i0 = 0; i0 < nu; i0 += 64) {
            const int i = i0 + lane;
            double acc = i < nu ? rq[i] : 0.0;
            const double di = i < nu ? (double)(TF)dv[i] : 0.0;
            // contributions of the rows of earlier passes
            for (int jj = 0; jj < i0; ++jj)
              if (i < nu) acc -= (double)(TF)upan(jj >> 4, i >> 4)[(jj & 15) * LD + (i & 15)] * rb[jj];
            // (the coefficient is read on every lane, at a clamped row, and applied through a select:
            // a read under a condition waits for itself at once)
            const int ic = min(i, nu - 1);
            for (int jj = i0; jj < nu && jj < i0 + 64; ++jj) {
              const double y = lane_bcast(acc * di, jj - i0);
              const double lv = (double)(TF)upan(jj >> 4, ic >> 4)[(jj & 15) * LD + (ic & 15)];
              acc = (i > jj && i < nu) ? acc - lv * y : acc;
            }
            if (i < nu) {
              const double v = acc * di;
              rb[i] = v;
              rbar_g[(int64_t)k * nu + i] = v;
            }
            wave_sync();
          }
        }
        __syncthreads();
        if (k > 0) {
          for (int i = tid; i < nx; i += nt) {
            double s = rq[16 * TU + i];
            for (int jj = 0; jj < nu; ++jj)
              s -= (double)(TF)upan(jj >> 4, TU + (i >> 4))[(jj & 15) * LD + (i & 15)] * rb[jj];
            pv[i] = s;
            p_g[(int64_t)k * nx + i] = s;
          }
        }
      }
      // ---- input part of the factor block of stage k (coalesced, from LDS)
      if (TF* Fk = dst(k); Fk && k < N) {
        for (int i = w; i < nu; i += nt >> 6)
          for (int jj = lane; jj <= i; jj += 64)
            Fk[i * (i + 1) / 2 + jj] = (TF)upan(jj >> 4, i >> 4)[(jj & 15) * LD + (i & 15)];
        for (int i = tid; i < nu; i += nt) Fk[oDR + i] = (TF)dv[i];
        for (int e = tid; e < nx * nu; e += nt) {
          const int i = e / nu, jj = e - i * nu;
          Fk[oLS + e] = (TF)upan(jj >> 4, TU + (i >> 4))[(jj & 15) * LD + (i & 15)];
        }
      }
    }
    // ---- factor block of stage k, state part (coalesced, from LDS; the input part went out with
    // the right-hand-side step)
    TF* Fk = dst(k);
    if (Fk && k > 0) {
      for (int i = w; i < nx; i += nt >> 6)
        for (int jj = lane; jj <= i; jj += 64)
          Fk[oLQ + i * (i + 1) / 2 + jj] = lqb(jj >> 4, i >> 4)[(jj & 15) * LQ + (i & 15)];
      for (int i = tid; i < nx; i += nt) Fk[oDQ + i] = (TF)dv[16 * TU + i];
    }
    __syncthreads();
  }
}

}  // namespace
}  // namespace lq
