// Size-specialised kernels for uniform batches with nx + nu <= 16.
//
// Mapping: 16 lanes per instance, four instances per 64-wide wavefront (one wavefront per
// workgroup).  Lane i of an instance owns row i of the stage matrix
// Hhat_k = [[R,S],[S^T,Q]] + V V^T (rows 0..nu-1: inputs, rows nu..nu+nx-1: states) and, after
// the stage Cholesky, row i of its factor [[L^R, 0],[L^S, L^Q]].  What an instance carries from
// stage to stage (rows of L^Q_{k+1}, p_{k+1}; in the solve, x_k and lam_{k-1}) stays in
// registers.  Cross-row operands are broadcast inside the 16-lane row with 64-bit DPP
// row_newbcast moves.
//
// Memory: each stage's matrices of the four instances are fetched with coalesced 16-byte loads
// one stage ahead (they do not depend on the recursion), written to LDS laid out as
// C = [B_k A_k] (nx rows of nu+nx) and H = [[R_k, S_k], [., Q_k]], and read back per lane as
// rows or columns at compile-time offsets.  Factor blocks leave through LDS as coalesced
// 16-byte stores.  (Reading rows per lane straight from global memory touches a different
// cache line per lane and leaves the kernel bound by the vector-memory pipeline.)
//
// Factor sweep per stage (backward in time), c_i = column i of C held by lane i:
//   V[i][j]    = sum_{m>=j} c_i[m] L^Q_{k+1}[m][j]       (trmm: broadcast rows of L^Q)
//   Hhat[i][j] = H[i][j] + sum_m V[i][m] V[j][m]          (syrk: broadcast rows of V)
//   chol(Hhat)                                            (potrf, float64, right-looking)
// plus the right-hand-side sweep rbar_k = (L^R_k)^{-1}(r_k + B_k^T w),
// p_k = q_k + A_k^T w - L^S_k rbar_k, w = L^Q_{k+1} L^Q_{k+1}^T f_k + p_{k+1}.
//
// Solve: one forward pass computes the rollout and, in the same pass, the float64 KKT
// residual of the new iterate (eq. opt-cond-ocp-eq); each refinement iteration is a backward
// correction sweep over the stored residual followed by another forward+residual pass.  The
// four instances of a wavefront share the LDS staging, so they run every pass together; an
// instance that has converged runs it with its stores masked.
//
// Factor blocks use the generic workspace layout, so the generic solve and adjoint kernels
// consume these factors unchanged.
//
// The kernels are templates over the shape; lq_small.hip and lq_small_env.hip instantiate them for
// their lists of (nx, nu) and dispatch to them.
#pragma once
#include <math.h>

#include <type_traits>

#include "lq_internal.hpp"

namespace lq {
namespace {

typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

// 1/sqrt(a): the hardware estimate (about 5e-8 relative) and NR Newton steps (two: 1 ulp; one:
// about 4e-15, enough for factors that are rounded to float32 afterwards).
template <int NR = 2>
__device__ __forceinline__ double rsqrt_f64(double a) {
  double y = __builtin_amdgcn_rsq(a);
  const double h = 0.5 * a;
#pragma unroll
  for (int s = 0; s < NR; ++s) y = y * fma(-h * y, y, 1.5);
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
  v = nan_max(v, dpp_d<0xB1>(v));
  v = nan_max(v, dpp_d<0x4E>(v));
  v = nan_max(v, dpp_d<0x124>(v));
  v = nan_max(v, dpp_d<0x128>(v));
  return v;
}

// Right-looking Cholesky of the row-distributed tile (lane i holds row i in h), pivot
// columns 0..NCOL-1.  Returns 0, 1 (a pivot was not positive) or 2 (a pivot was not finite);
// failed pivots are replaced by 1 so the sweep continues with finite numbers.
template <int NUX, int NCOL, int NR = 2>
__device__ __forceinline__ int potrf_rows(double (&h)[NUX], double& mydinv, int i) {
  // the first failing pivot classifies the stage: finite and not positive (1) or not finite (2);
  // what the replaced pivot does to the later pivots of the stage does not change that
  int kind = 0;
#pragma unroll
  for (int j = 0; j < NCOL; ++j) {
    double dj = bc(h[j], j);
    const bool good = dj > 0.0 && dj <= 1.7976931348623157e308;
    kind = kind ? kind : (good ? 0 : (isfinite(dj) ? 1 : 2));
    dj = good ? dj : 1.0;
    const double inv = rsqrt_f64<NR>(dj);
    h[j] = (i == j) ? dj * inv : h[j] * inv;
    mydinv = (i == j) ? inv : mydinv;
#pragma unroll
    for (int kk = j + 1; kk < NCOL; ++kk) h[kk] = fma(-h[j], bc(h[j], kk), h[kk]);
  }
  return kind;
}

template <typename T>
__device__ __forceinline__ double rnd(double v) {
  return (double)(T)v;
}

template <int NX, int NU>
struct Shape {
  static constexpr int NUX = NX + NU;
  static constexpr int FS = NU * (NU + 1) / 2 + NU + NX * NU + NX * (NX + 1) / 2 + NX;
  static constexpr int ODR = NU * (NU + 1) / 2, OLS = ODR + NU, OLQ = OLS + NX * NU,
                       ODQ = OLQ + NX * (NX + 1) / 2;
  // LDS tiles: rows padded to RSP = nx + nu + 2 elements and instance tiles to a stride that
  // is 8 doubles past a multiple of 32, so that row-wise reads of different lanes and the
  // four instances of a wavefront fall into different LDS banks.
  static constexpr int RSP = NUX + 2;
  static constexpr int LC = (NX * RSP + 31) / 32 * 32 + 8;   // LDS elements of C per instance
  static constexpr int LH = (NUX * RSP + 31) / 32 * 32 + 8;  // LDS elements of H per instance
};

// Lane identity.
struct Lane {
  int lane, g, i, ia, ic, mi;  // lane in wave, instance slot, row, clamped row/input/state index
  bool isu, inst, valid;
  int b0, b;
  int64_t bb;                  // clamped instance index (always a valid instance, for loads)
};

template <int NX, int NU>
__device__ __forceinline__ Lane lane_id(int batch) {
  constexpr int NUX = NX + NU;
  Lane L;
  L.lane = threadIdx.x & 63;
  L.g = L.lane >> 4;
  L.i = L.lane & 15;
  L.ia = L.i < NUX ? L.i : NUX - 1;
  L.b0 = blockIdx.x * 4;
  L.b = L.b0 + L.g;
  L.inst = L.b < batch;
  L.valid = L.inst && L.i < NUX;
  L.bb = L.inst ? L.b : 0;
  L.isu = L.i < NU;
  L.ic = L.isu ? L.i : 0;
  L.mi = (!L.isu && L.i < NUX) ? L.i - NU : 0;
  return L;
}

template <int BYTES>
struct VecT;
template <>
struct VecT<16> {
  using type = u4;
};
template <>
struct VecT<8> {
  using type = u2;
};
template <>
struct VecT<4> {
  using type = unsigned int;
};

// Chunk width (elements) for moving blocks whose element counts / offsets are multiples of it.
template <typename T>
__host__ __device__ constexpr int chunk_w(int a, int b, int c, int d, int e) {
  return (a % (16 / (int)sizeof(T)) == 0 && b % (16 / (int)sizeof(T)) == 0 && c % (16 / (int)sizeof(T)) == 0 &&
          d % (16 / (int)sizeof(T)) == 0 && e % (16 / (int)sizeof(T)) == 0)
             ? 16 / (int)sizeof(T)
             : ((a % (8 / (int)sizeof(T)) == 0 && b % (8 / (int)sizeof(T)) == 0 &&
                 c % (8 / (int)sizeof(T)) == 0 && d % (8 / (int)sizeof(T)) == 0 && e % (8 / (int)sizeof(T)) == 0)
                    ? 8 / (int)sizeof(T)
                    : 1);
}

// One staged segment: per instance and stage a contiguous global block of BLK elements (a
// row-major matrix with rows of RW elements), placed in LDS at instance stride LSTR, row
// stride RS and element offset O0.  The wavefront's four blocks move as 16-byte chunks where
// the shape allows (else 8 or 4 bytes), lane c taking chunks c, c + 64, ...
template <typename T, int BLK, int RW, int RS, int O0, int LSTR>
struct Seg {
  static constexpr int W = chunk_w<T>(BLK, RW, RS, O0, LSTR);
  static constexpr int CPI = BLK / W;
  static constexpr int TOT = 4 * CPI;
  static constexpr int NI = (TOT + 63) / 64;
  using V = typename VecT<W * (int)sizeof(T)>::type;
  V r[NI];

  // base: array base (instance i's block of stage k at i * istr + k * BLK)
  __device__ __forceinline__ void load(const T* base, int64_t istr, const Lane& L, int batch, int k) {
#pragma unroll
    for (int t = 0; t < NI; ++t) {
      int c = L.lane + 64 * t;
      c = c < TOT ? c : TOT - 1;
      const int g = c / CPI, w = c % CPI;
      int inst = L.b0 + g;
      inst = inst < batch ? inst : batch - 1;
      r[t] = *(const V*)(base + (int64_t)inst * istr + (int64_t)k * BLK + w * W);
    }
  }
  __device__ __forceinline__ void store(T* lds, const Lane& L) const {
#pragma unroll
    for (int t = 0; t < NI; ++t) {
      const int c = L.lane + 64 * t;
      if (TOT % 64 == 0 || c < TOT) {
        const int g = c / CPI, e = (c % CPI) * W;
        *(V*)(lds + g * LSTR + (e / RW) * RS + O0 + (e % RW)) = r[t];
      }
    }
  }
};

// Coalesced store of the four instances' blocks of BLK elements from LDS to global memory
// (instance i's block at i * istr + off).  Every lane reads and stores: lanes past the last chunk or
// instance repeat the last valid chunk with its own value, since a read feeding a conditional
// store would be sunk into the condition and wait there.
template <typename T, int BLK>
__device__ __forceinline__ void store_blocks(T* gbase, int64_t istr, int64_t off, const T* lds, const Lane& L,
                                             int batch) {
  constexpr int W = chunk_w<T>(BLK, BLK, BLK, 0, BLK);
  using V = typename VecT<W * (int)sizeof(T)>::type;
  constexpr int CPI = BLK / W, TOT = 4 * CPI, NI = (TOT + 63) / 64;
  const int gmax = min(3, batch - 1 - L.b0);  // last instance slot of the wavefront
#pragma unroll
  for (int t = 0; t < NI; ++t) {
    const int c = min(L.lane + 64 * t, TOT - 1);
    const int g = min(c / CPI, gmax), w = c % CPI;
    *(V*)(gbase + (int64_t)(L.b0 + g) * istr + off + w * W) = *(const V*)(lds + g * BLK + w * W);
  }
}

// The stage data of the four instances of a wavefront, staged through LDS.
template <int NX, int NU, bool HS, bool HF>
struct StageData {
  using SH = Shape<NX, NU>;
  static constexpr int NUX = NX + NU, LC = SH::LC, LH = SH::LH, RSP = SH::RSP;
  Seg<double, NX * NU, NU, RSP, 0, LC> B;               // -> C[:, 0:nu]
  Seg<double, NX * NX, NX, RSP, NU, LC> A;              // -> C[:, nu:]
  Seg<double, NU * NU, NU, RSP, 0, LH> R;               // -> H[0:nu, 0:nu]
  Seg<double, NU * NX, NX, RSP, NU, LH> S;              // -> H[0:nu, nu:]
  Seg<double, NX * NX, NX, RSP, NU * RSP + NU, LH> Q;   // -> H[nu:, nu:]
  Seg<double, NU, NU, NU, 0, NUX> r;                    // -> RQ[0:nu]
  Seg<double, NX, NX, NX, NU, NUX> q;                   // -> RQ[nu:]
  Seg<double, NX, NX, NX, 0, NX> f;                     // -> Fv

  __device__ __forceinline__ void load(const lq_data& d, int N, const Lane& L, int batch, int k, bool withH) {
    B.load(d.B, (int64_t)N * NX * NU, L, batch, k);
    A.load(d.A, (int64_t)N * NX * NX, L, batch, k);
    if (withH) {
      R.load(d.R, (int64_t)N * NU * NU, L, batch, k);
      if (HS) S.load(d.S, (int64_t)N * NU * NX, L, batch, k);
      Q.load(d.Q, (int64_t)(N + 1) * NX * NX, L, batch, k);
      r.load(d.r, (int64_t)N * NU, L, batch, k);
      q.load(d.q, (int64_t)(N + 1) * NX, L, batch, k);
      if (HF) f.load(d.f, (int64_t)N * NX, L, batch, k);
    }
  }
  __device__ __forceinline__ void store(double* sC, double* sH, double* sRQ, double* sFv, const Lane& L,
                                        bool withH) const {
    B.store(sC, L);
    A.store(sC, L);
    if (withH) {
      R.store(sH, L);
      if (HS) S.store(sH, L);
      Q.store(sH, L);
      r.store(sRQ, L);
      q.store(sRQ, L);
      if (HF) f.store(sFv, L);
    }
  }
};

template <int NX, int NU>
__device__ __forceinline__ void zero_S_block(double* sH, const Lane& L) {
  constexpr int LH = Shape<NX, NU>::LH, RSP = Shape<NX, NU>::RSP;
  for (int e = L.lane; e < 4 * NU * NX; e += 64) {
    const int gg = e / (NU * NX), w = e % (NU * NX);
    sH[gg * LH + (w / NX) * RSP + NU + (w % NX)] = 0.0;
  }
}

// ------------------------------------------------------------------------------------------
// Factor sweep

template <int NX, int NU, typename TF, typename TP, bool HS, bool HF>
__global__ void __launch_bounds__(64) k_factor_small(int batch, int N, lq_data d, TF* __restrict__ F,
                                                     double* __restrict__ Vws, int32_t* __restrict__ info) {
  using SH = Shape<NX, NU>;
  constexpr int NUX = SH::NUX, FS = SH::FS, LC = SH::LC, LH = SH::LH;
  static_assert(NUX <= 16, "tile exceeds a 16-lane row");
  __shared__ __attribute__((aligned(16))) double sC[4 * LC];
  __shared__ __attribute__((aligned(16))) double sH[4 * LH];
  __shared__ __attribute__((aligned(16))) double sRQ[4 * NUX];
  __shared__ __attribute__((aligned(16))) double sFv[HF ? 4 * NX : 2];
  __shared__ __attribute__((aligned(16))) TF sOut[4 * FS];

  const Lane L = lane_id<NX, NU>(batch);
  const int i = L.i, ia = L.ia, ic = L.ic, mi = L.mi, g = L.g;
  const bool isu = L.isu, valid = L.valid;
  double* rbar = Vws + L.bb * ((int64_t)N * NU + (int64_t)(N + 1) * NX);
  double* pv = rbar + (int64_t)N * NU;
  if (!HS) zero_S_block<NX, NU>(sH, L);

  StageData<NX, NU, HS, HF> sd;
  sd.load(d, N, L, batch, N - 1, true);

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
    const int bad = potrf_rows<NUX, NUX, sizeof(TF) == 4 ? 1 : 2>(h, mydinv, i);
    if (bad) code = bad == 2 ? LQ_INFO_NONFINITE : N + 1;
#pragma unroll
    for (int j = 0; j < NUX; ++j) h[j] = rnd<TF>(h[j]);
    mydinv = rnd<TF>(mydinv);
    TF* po = sOut + g * FS;
    if (!isu && i < NUX) {
#pragma unroll
      for (int j = 0; j < NX; ++j)
        if (j <= mi) po[SH::OLQ + mi * (mi + 1) / 2 + j] = (TF)h[NU + j];
      po[SH::ODQ + mi] = (TF)mydinv;
      if (valid) pv[(int64_t)N * NX + mi] = pn;
    }
    store_blocks<TF, FS>(F, (int64_t)(N + 1) * FS, (int64_t)N * FS, sOut, L, batch);
#pragma unroll
    for (int j = 0; j < NX; ++j) lq[j] = (j <= mi) ? h[NU + j] : 0.0;
  }

  for (int k = N - 1; k >= 0; --k) {
    sd.store(sC, sH, sRQ, sFv, L, true);
    sd.load(d, N, L, batch, k > 0 ? k - 1 : 0, true);
    // operands of stage k from LDS
    constexpr int RSP = SH::RSP;
    const double* pc = sC + g * LC + ia;          // column ia of C: pc[m * RSP]
    const double* pr = sH + g * LH + ia * RSP;    // row ia of H
    const double* pk = sH + g * LH + ia;          // column ia of H: pk[j * RSP]
    double c[NX];
#pragma unroll
    for (int m = 0; m < NX; ++m) c[m] = pc[m * RSP];
#pragma unroll
    for (int j = 0; j < NUX; ++j) {
      const double col = pk[j * RSP];
      const double rj = pr[j];  // read on every lane: a read under a condition waits at once
      const double sym = 0.5 * (rj + col);
      const double v = (!isu && j < NU) ? col : sym;
      h[j] = j <= i ? v : 0.0;
    }
    const double rqv = sRQ[g * NUX + ia];
    double tq = (isu || k > 0) ? rqv : 0.0;

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
      const double fm = HF ? sFv[g * NX + m] : 0.0;
#pragma unroll
      for (int j = 0; j <= m; ++j) {
        if (sizeof(TP) == 4) {
          const float Lf = bc((float)lq[j], NU + m);
          v[j] += (TP)c[m] * (TP)Lf;
          if (HF) t1[j] = fma((double)Lf, fm, t1[j]);
        } else {
          const double Ld = bc(lq[j], NU + m);
          v[j] += (TP)c[m] * (TP)Ld;
          if (HF) t1[j] = fma(Ld, fm, t1[j]);
        }
      }
    }
    // w = L^Q_{k+1} t1 + p_{k+1} (state lanes), then (rhat, qhat) = (r, q) + C^T w
    double wv = pn;
    if (HF) {
#pragma unroll
      for (int j = 0; j < NX; ++j) wv = fma(lq[j], t1[j], wv);
    }
    {
      double ta[3] = {tq, 0.0, 0.0};
#pragma unroll
      for (int m = 0; m < NX; ++m) ta[m % 3] = fma(c[m], bc(wv, NU + m), ta[m % 3]);
      tq = ta[0] + (ta[1] + ta[2]);
    }
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
    // (the row index through an opaque copy: otherwise the compiler keeps the sixteen lane masks
    // of the unrolled Cholesky live across the stage loop and spills them)
    int io = i;
    asm volatile("" : "+v"(io));
    // (one Newton step for factors stored as float32, two for float64)
    constexpr int NRS = sizeof(TF) == 4 ? 1 : 2;
    if (k > 0) bad = potrf_rows<NUX, NUX, NRS>(h, mydinv, io);
    else bad = potrf_rows<NUX, NU, NRS>(h, mydinv, io);
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
    // factor rows -> LDS block -> coalesced global store
    TF* po = sOut + g * FS;
    if (i < NUX) {
      if (isu) {
#pragma unroll
        for (int j = 0; j < NU; ++j)
          if (j <= ic) po[ic * (ic + 1) / 2 + j] = (TF)h[j];
        po[SH::ODR + ic] = (TF)mydinv;
      } else {
#pragma unroll
        for (int j = 0; j < NU; ++j) po[SH::OLS + mi * NU + j] = (TF)h[j];
#pragma unroll
        for (int j = 0; j < NX; ++j)
          if (j <= mi) po[SH::OLQ + mi * (mi + 1) / 2 + j] = (TF)h[NU + j];
        po[SH::ODQ + mi] = (TF)mydinv;
      }
    }
    store_blocks<TF, FS>(F, (int64_t)(N + 1) * FS, (int64_t)k * FS, sOut, L, batch);
    if (valid) {
      if (isu) rbar[(int64_t)k * NU + ic] = tq * mydinv;
      else if (k > 0) pv[(int64_t)k * NX + mi] = tq;
    }
    pn = tq;
#pragma unroll
    for (int j = 0; j < NX; ++j) lq[j] = (j <= mi) ? h[NU + j] : 0.0;
  }
  if (L.inst && i == 0) info[L.b] = code;
}

// ------------------------------------------------------------------------------------------
// Solve.  Lane roles: lane j < nu carries u_j; lane nu + m carries x_m and lam_m.

template <int NX, int NU, typename TF, bool HS, bool HF>
struct SolveCtx {
  Lane L;
  int N, batch;
  const TF* F;             // factor region base (all instances)
  lq_data d;
  const double *rb0, *p0;  // this instance's factor-time sweep vectors
  double *rb2, *p2, *flam, *rhou, *rhox;
  double *x, *u, *lam;
  TF* sF;                  // LDS: two stage slots x 4 instances x FS
  double *sC, *sH, *sRQ, *sFv;
};

// Per-lane operands of forward stage k (contiguous per instance), loaded a stage ahead.  The
// loads are plain (no arithmetic or selection on the loaded values here): an operation on a
// loaded value placed next to its load makes the wavefront wait for that load at once.
struct FwdVec {
  double rv;          // rbar_k[ic] (used on input lanes)
  double fv;          // f_k[mi] (mode 0) or flam_k[mi] (used on state lanes)
  double s1;          // p_{k+1}[mi]
  double zu, zx, zl;  // old iterate (correction passes): u_k[ic], x_{k+1}[mi], lam_k[mi]
};

template <int NX, int NU, typename TF, bool HS, bool HF>
__device__ __forceinline__ void load_fwdvec(FwdVec& v, const SolveCtx<NX, NU, TF, HS, HF>& s, int k, int mode) {
  const Lane& L = s.L;
  const double* rbv = mode == 0 ? s.rb0 : s.rb2;
  const double* pvv = mode == 0 ? s.p0 : s.p2;
  if (mode == 0) v.fv = HF ? s.d.f[(L.bb * s.N + k) * NX + L.mi] : 0.0;
  else v.fv = s.flam[(int64_t)k * NX + L.mi];
  v.rv = rbv[(int64_t)k * NU + L.ic];
  v.s1 = pvv[(int64_t)(k + 1) * NX + L.mi];
  if (mode == 1) {
    v.zu = s.u[(int64_t)k * NU + L.ic];
    v.zx = s.x[(int64_t)k * NX + L.mi];
    v.zl = s.lam[(int64_t)k * NX + L.mi];
  } else {
    v.zu = v.zx = v.zl = 0.0;
  }
}

// Factor block of one stage for the four instances.
template <int NX, int NU, typename TF>
using FSeg = Seg<TF, Shape<NX, NU>::FS, Shape<NX, NU>::FS, Shape<NX, NU>::FS, 0, Shape<NX, NU>::FS>;

// One forward pass.  mode 0: z = solution (x_0 = x_init, f = f_k, sweep vectors of lq_factor);
// mode 1: z += correction (dx_0 = 0, f = flam, sweep vectors rbar2/p2).  With `res`, computes
// the KKT residual of the updated iterate on the fly (and stores it when `store`); returns
// rel_res (uniform over the instance's 16 lanes), or 0 without `res`.  Lanes of instances with
// act == false store nothing.
template <int NX, int NU, typename TF, bool HS, bool HF>
__device__ double fwd_res(const SolveCtx<NX, NU, TF, HS, HF>& s, int mode, bool res, bool store, bool act) {
  using SH = Shape<NX, NU>;
  constexpr int NUX = SH::NUX, FS = SH::FS, LC = SH::LC, LH = SH::LH;
  const Lane& L = s.L;
  const int N = s.N, batch = s.batch, i = L.i, ia = L.ia, mi = L.mi, ic = L.ic, g = L.g;
  const bool isu = L.isu, xl = act && L.valid && !L.isu, ul = act && L.valid && L.isu;
  const int64_t fistr = (int64_t)(N + 1) * FS;
  const double x0v = s.d.x0[L.bb * NX + mi];
  double xc = (mode == 0 && !isu) ? x0v : 0.0;  // recursion state (x_k or dx_k)
  double xk = isu ? 0.0 : x0v;                   // updated iterate x_k (x_0 = x_init)
  double lkm = 0.0;                              // updated lam_{k-1}
  double mr = 0.0, mb = 0.0;

  // prologue: F_0 in LDS slot 0; stage-0 data and F_1 in flight.  Every stage then runs the same
  // code: no load of the loop sits under a condition (the prefetch index is clamped instead, so
  // the last stage fetches a block again), since a conditional load makes the wavefront wait for
  // every load in flight where the paths join.
  {
    FSeg<NX, NU, TF> f0;
    f0.load(s.F, fistr, L, batch, 0);
    f0.store(s.sF, L);
  }
  FSeg<NX, NU, TF> fn;
  StageData<NX, NU, HS, HF> dn;
  dn.load(s.d, N, L, batch, 0, true);
  fn.load(s.F, fistr, L, batch, 1);
  FwdVec cur, nxt;
  load_fwdvec<NX, NU, TF, HS, HF>(cur, s, 0, mode);

  for (int k = 0; k < N; ++k) {
    // The lane's entries of F_k that start the recursion (in LDS since the previous stage) are
    // read first, in one batch: the empty asm with a memory clobber keeps the compiler from
    // sinking each read to its use, where every read would wait for itself.
    const TF* Fk = s.sF + (k & 1) * 4 * FS + g * FS;  // F_k of this instance
    TF fls[NX], flr[NU];
#pragma unroll
    for (int m = 0; m < NX; ++m) fls[m] = Fk[SH::OLS + m * NU + ic];
#pragma unroll
    for (int j = 0; j < NU; ++j) flr[j] = Fk[j * (j + 1) / 2 + ic];  // L^R[j][ic] for ic < j
    const TF fdr = Fk[SH::ODR + ic];
    asm volatile("" ::: "memory");
    // stage k data and F_{k+1} into LDS (slot (k+1) & 1 held F_{k-1}, no longer needed), then
    // stage k + 1 in flight
    dn.store(s.sC, s.sH, s.sRQ, s.sFv, L, true);
    fn.store(s.sF + ((k + 1) & 1) * 4 * FS, L);
    const int kn = k + 1 < N ? k + 1 : N - 1;
    dn.load(s.d, N, L, batch, kn, true);
    fn.load(s.F, fistr, L, batch, k + 2 <= N ? k + 2 : N);
    load_fwdvec<NX, NU, TF, HS, HF>(nxt, s, kn, mode);
    constexpr int RSP = SH::RSP;
    const TF* Fk1 = s.sF + ((k + 1) & 1) * 4 * FS + g * FS;   // F_{k+1}
    const double* prC = s.sC + g * LC + ia;                    // column ia of C (stride RSP)
    const double* prA = s.sC + g * LC + mi * RSP;              // row mi of C = [B row, A row]

    // t = rbar + L^S^T x on input lanes
    double ta[3] = {cur.rv, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < NX; ++m) {
      const double xb = bc(xc, NU + m);
      ta[m % 3] = fma((double)fls[m], xb, ta[m % 3]);
    }
    double t = ta[0] + (ta[1] + ta[2]);
    // u' = L^R^{-T} t, u = -u'
    const double dRi = (double)fdr;
    double uu = 0.0;
#pragma unroll
    for (int j = NU - 1; j >= 0; --j) {
      const double uj = bc(t * dRi, j);
      uu = (i == j) ? uj : uu;
      const double e = (double)flr[j];  // L^R[j][ic] for ic < j (in-block otherwise)
      t = fma((i < j) ? -e : 0.0, uj, t);
    }
    const double du = -uu;
    // The lane's row of C_k = [B_k A_k] and its L^Q_{k+1} coefficients (column and row mi; the
    // ones outside the triangle stay inside the block and are masked below), read in one batch.
    double pa[NUX];
    TF lqc[NX], lqr[NX];
#pragma unroll
    for (int j = 0; j < NUX; ++j) pa[j] = prA[j];
#pragma unroll
    for (int m = 0; m < NX; ++m) {
      lqc[m] = Fk1[SH::OLQ + mi + m * (m + 1) / 2];
      lqr[m] = Fk1[SH::OLQ + mi * (mi + 1) / 2 + m];
    }
    asm volatile("" ::: "memory");
    // x_{k+1} = A x + B u + f on state lanes
    double xa[3] = {cur.fv, 0.0, 0.0};
#pragma unroll
    for (int n = 0; n < NX; ++n) {
      const double xb = bc(xc, NU + n);
      xa[n % 3] = fma(pa[NU + n], xb, xa[n % 3]);
    }
#pragma unroll
    for (int j = 0; j < NU; ++j) xa[(NX + j) % 3] = fma(pa[j], bc(du, j), xa[(NX + j) % 3]);
    const double xn = xa[0] + (xa[1] + xa[2]);
    // lam = L^Q_{k+1} (L^Q_{k+1}^T x_{k+1}) + p_{k+1}; coefficients masked to the triangle
    double t2a[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < NX; ++m) {
      const double lv = (double)lqc[m];
      const double cm = (m >= mi) ? lv : 0.0;
      t2a[m % 3] = fma(cm, bc(xn, NU + m), t2a[m % 3]);
    }
    const double t2 = t2a[0] + (t2a[1] + t2a[2]);
    double lma[3] = {cur.s1, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const double lv = (double)lqr[j];
      const double cj = (j <= mi) ? lv : 0.0;
      lma[j % 3] = fma(cj, bc(t2, NU + j), lma[j % 3]);
    }
    const double lm = lma[0] + (lma[1] + lma[2]);
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
      // row and column ia of H and column ia of C, read in one batch
      const double* hrp = s.sH + g * LH + ia * RSP;
      const double* hcp = s.sH + g * LH + ia;
      double hr[NUX], hcs[NUX], pcv[NX];
#pragma unroll
      for (int j = 0; j < NUX; ++j) {
        hr[j] = hrp[j];
        hcs[j] = hcp[j * RSP];
      }
#pragma unroll
      for (int n = 0; n < NX; ++n) pcv[n] = prC[n * RSP];
      asm volatile("" ::: "memory");
      // residual rows of stage k at the updated iterate (x_k = xk, u_k, lam_k, x_{k+1}, lam_{k-1})
      double au[2] = {0.0, 0.0};   // input lanes: S x_k ; R u
      double ab[2] = {0.0, 0.0};   // column ia of C times lam: B^T lam (input) / A^T lam (state)
      double al[2] = {-xnew, 0.0}; // state lanes: A x_k - x_{k+1} ; B u
      double ax[2] = {-lkm, 0.0};  // state lanes: Q x_k - lam_{k-1} ; S^T u
#pragma unroll
      for (int n = 0; n < NX; ++n) {
        const double xb = bc(xk, NU + n);
        const double lb = bc(lnew, NU + n);
        const double hrow = hr[NU + n], hcol = hcs[NU + n];
        if (HS) au[0] = fma(hrow, xb, au[0]);
        ab[n & 1] = fma(pcv[n], lb, ab[n & 1]);
        al[0] = fma(pa[NU + n], xb, al[0]);
        ax[0] = fma(0.5 * (hrow + hcol), xb, ax[0]);
      }
      const double bu = (k == 0 && HS) ? au[0] : 0.0;   // S_0 x_init
      const double bl = (k == 0) ? al[0] + xnew : 0.0;  // A_0 x_init
#pragma unroll
      for (int j = 0; j < NU; ++j) {
        const double ub = bc(unew, j);
        const double hrow = hr[j], hcol = hcs[j];
        au[1] = fma(0.5 * (hrow + hcol), ub, au[1]);
        al[1] = fma(pa[j], ub, al[1]);
        if (HS) ax[1] = fma(hcol, ub, ax[1]);
      }
      const double abt = ab[0] + ab[1];
      const double rq = s.sRQ[g * NUX + ia];
      const double fo = HF ? s.sFv[g * NX + mi] : 0.0;
      const double rhou = -rq - ((au[0] + au[1]) + abt);
      const double rhol = -fo - (al[0] + al[1]);
      const double rhox = -rq - ((ax[0] + ax[1]) + abt);
      if (ul) {
        mr = nan_max(mr, fabs(rhou));
        mb = nan_max(mb, fabs(rq + bu));
      }
      if (xl) {
        mr = nan_max(mr, fabs(rhol));
        mb = nan_max(mb, fabs(fo + bl));
        if (k > 0) {
          mr = nan_max(mr, fabs(rhox));
          mb = nan_max(mb, fabs(rq));
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
    cur = nxt;
  }
  if (res) {
    // stage N: Q_N x_N - lam_{N-1} = -q_N
    const int64_t bb = L.bb;
    const double* QN = s.d.Q + (bb * (N + 1) + N) * NX * NX;
    // row and column of Q_N and q_N loaded before any use, so that they arrive together
    double qr[NX], qc[NX];
#pragma unroll
    for (int n = 0; n < NX; ++n) {
      qr[n] = QN[mi * NX + n];
      qc[n] = QN[n * NX + mi];
    }
    const double qv = s.d.q[(bb * (N + 1) + N) * NX + mi];
    double ax = -lkm;
#pragma unroll
    for (int n = 0; n < NX; ++n) {
      const double xb = bc(xk, NU + n);
      ax = fma(0.5 * (qr[n] + qc[n]), xb, ax);
    }
    const double rhox = -qv - ax;
    if (xl) {
      mr = nan_max(mr, fabs(rhox));
      mb = nan_max(mb, fabs(qv));
      if (store) s.rhox[(int64_t)N * NX + mi] = rhox;
    }
    mr = rowmax(mr);
    mb = rowmax(mb);
    return rel_of(mr, mb);
  }
  return 0.0;
}

// Backward sweep of the correction right-hand side (r, q, f) = (-rho_u, -rho_x, -rho_l),
// x_init = 0, into (rbar2, p2).  Lanes of instances with act == false store nothing.
template <int NX, int NU, typename TF, bool HS, bool HF>
__device__ void bwd_corr(const SolveCtx<NX, NU, TF, HS, HF>& s, bool act) {
  using SH = Shape<NX, NU>;
  constexpr int NUX = SH::NUX, FS = SH::FS, LC = SH::LC;
  const Lane& L = s.L;
  const int N = s.N, batch = s.batch, i = L.i, ia = L.ia, mi = L.mi, ic = L.ic, g = L.g;
  const bool isu = L.isu, xl = act && L.valid && !L.isu, ul = act && L.valid && L.isu;
  const int64_t fistr = (int64_t)(N + 1) * FS;
  double p2n = -s.rhox[(int64_t)N * NX + mi];
  if (xl) s.p2[(int64_t)N * NX + mi] = p2n;
  // prologue: F_N in LDS; stages N-1 and N-2 in flight in two register sets, used alternately, so
  // that each stage's data is fetched two stages ahead (a wavefront running alone, as in the
  // refinement tail, would otherwise wait for memory every stage); prefetch indices are clamped
  // and unconditional (see fwd_res)
  {
    FSeg<NX, NU, TF> fa;
    fa.load(s.F, fistr, L, batch, N);
    fa.store(s.sF + (N & 1) * 4 * FS, L);
  }
  // (the lane's residual entry is read through a selected address: selecting between two loaded
  // values would wait for both right after they are issued)
  auto rho_at = [&](int k) { return *(isu ? s.rhou + (int64_t)k * NU + ic : s.rhox + (int64_t)k * NX + mi); };
  FSeg<NX, NU, TF> fnA, fnB;
  StageData<NX, NU, HS, HF> dnA, dnB;
  const int kB = N > 1 ? N - 2 : 0;
  fnA.load(s.F, fistr, L, batch, N - 1);
  dnA.load(s.d, N, L, batch, N - 1, false);
  double rhoA = rho_at(N - 1), flA = s.flam[(int64_t)(N - 1) * NX + mi];
  fnB.load(s.F, fistr, L, batch, kB);
  dnB.load(s.d, N, L, batch, kB, false);
  double rhoB = rho_at(kB), flB = s.flam[(int64_t)kB * NX + mi];
  auto step = [&](int k, FSeg<NX, NU, TF>& fn, StageData<NX, NU, HS, HF>& dn, double& rho_r, double& fl_r) {
    // the lane's L^Q_{k+1} coefficients (in LDS since the previous stage) read first, in one batch
    // (see fwd_res); the ones outside the triangle stay inside the block and are masked below
    const TF* Fk1 = s.sF + ((k + 1) & 1) * 4 * FS + g * FS;
    TF lqc[NX], lqr[NX];
#pragma unroll
    for (int m = 0; m < NX; ++m) {
      lqc[m] = Fk1[SH::OLQ + mi + m * (m + 1) / 2];  // column mi
      lqr[m] = Fk1[SH::OLQ + mi * (mi + 1) / 2 + m];  // row mi
    }
    asm volatile("" ::: "memory");
    // F_k into slot k & 1 (held F_{k+2}, no longer needed), stage-k data into LDS, then stage
    // k - 2 into the same registers
    fn.store(s.sF + (k & 1) * 4 * FS, L);
    dn.store(s.sC, s.sH, s.sRQ, s.sFv, L, false);
    const double rho = rho_r, fl = fl_r;
    const int kp = k > 1 ? k - 2 : 0;
    fn.load(s.F, fistr, L, batch, kp);
    dn.load(s.d, N, L, batch, kp, false);
    rho_r = rho_at(kp);
    fl_r = s.flam[(int64_t)kp * NX + mi];
    constexpr int RSP = SH::RSP;
    const TF* Fk = s.sF + (k & 1) * 4 * FS + g * FS;
    // input lanes: row ic of L^R (packed); state lanes: row mi of L^S (read in one batch)
    const TF* hp = isu ? Fk + ic * (ic + 1) / 2 : Fk + SH::OLS + mi * NU;
    TF hrow[NU];
#pragma unroll
    for (int j = 0; j < NU; ++j) hrow[j] = hp[j];
    const TF fdr = Fk[SH::ODR + ic];
    asm volatile("" ::: "memory");
    // t1 = L^Q_{k+1}^T f', w = L^Q_{k+1} t1 + p2_{k+1} (coefficients masked to the triangle)
    double t1a[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < NX; ++m) {
      const double lv = (double)lqc[m];
      const double cm = (m >= mi) ? lv : 0.0;
      t1a[m % 3] = fma(cm, bc(fl, NU + m), t1a[m % 3]);
    }
    const double t1 = t1a[0] + (t1a[1] + t1a[2]);
    double wa[3] = {p2n, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const double lv = (double)lqr[j];
      const double cj = (j <= mi) ? lv : 0.0;
      wa[j % 3] = fma(cj, bc(t1, NU + j), wa[j % 3]);
    }
    const double w = wa[0] + (wa[1] + wa[2]);
    const double* prC = s.sC + g * LC + ia;
    double tqa[3] = {(isu || k > 0) ? -rho : 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < NX; ++m) tqa[m % 3] = fma(prC[m * RSP], bc(w, NU + m), tqa[m % 3]);
    double tq = tqa[0] + (tqa[1] + tqa[2]);
    const double dr = (double)fdr;
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      const double rb = bc(tq * dr, j);
      const double hv = (double)hrow[j];
      tq = (i > j) ? fma(-hv, rb, tq) : tq;
    }
    if (ul) s.rb2[(int64_t)k * NU + ic] = tq * dr;
    if (xl && k > 0) s.p2[(int64_t)k * NX + mi] = tq;
    p2n = tq;
  };
  for (int k = N - 1; k >= 0; k -= 2) {
    step(k, fnA, dnA, rhoA, flA);
    if (k == 0) break;
    step(k - 1, fnB, dnB, rhoB, flB);
  }
}

template <int NX, int NU, typename TF, bool HS, bool HF>
__global__ void __launch_bounds__(64) k_solve_small(SolveArgs a, int N) {
  using SH = Shape<NX, NU>;
  constexpr int NUX = SH::NUX, FS = SH::FS, LC = SH::LC, LH = SH::LH;
  __shared__ __attribute__((aligned(16))) TF sF[2 * 4 * FS];
  __shared__ __attribute__((aligned(16))) double sC[4 * LC];
  __shared__ __attribute__((aligned(16))) double sH[4 * LH];
  __shared__ __attribute__((aligned(16))) double sRQ[4 * NUX];
  __shared__ __attribute__((aligned(16))) double sFv[HF ? 4 * NX : 2];
  SolveCtx<NX, NU, TF, HS, HF> s;
  s.L = lane_id<NX, NU>(a.batch);
  s.N = N;
  s.batch = a.batch;
  s.d = a.d;
  s.F = (const TF*)a.F;
  s.sF = sF;
  s.sC = sC;
  s.sH = sH;
  s.sRQ = sRQ;
  s.sFv = sFv;
  const int64_t bb = s.L.bb;
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
  if (!HS) zero_S_block<NX, NU>(sH, s.L);

  const bool res = a.check || a.max_it > 0;
  int it = 0;
  double rel = fwd_res<NX, NU, TF, HS, HF>(s, 0, res, a.max_it > 0, s.L.inst);
  bool act = s.L.inst && a.max_it > 0 && rel > a.tol;
  while (__any(act)) {
    bwd_corr<NX, NU, TF, HS, HF>(s, act);
    const double r2 = fwd_res<NX, NU, TF, HS, HF>(s, 1, true, it + 1 < a.max_it, act);
    if (act) {
      ++it;
      rel = r2;
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
  (void)LC;
  (void)LH;
  (void)NUX;
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

// Factor / solve launches of one compiled shape, float64 or mixed mode.
template <int NX, int NU>
hipError_t factor_shape(lq_mode mode, int batch, int N, const lq_data& d, void* F, double* V, int32_t* info,
                        hipStream_t st) {
  return mode == LQ_F64 ? factor_tf<NX, NU, double, double>(batch, N, d, F, V, info, st)
                        : factor_tf<NX, NU, float, float>(batch, N, d, F, V, info, st);
}
template <int NX, int NU>
hipError_t solve_shape(lq_mode mode, int N, const SolveArgs& a, hipStream_t st) {
  return mode == LQ_F64 ? solve_tf<NX, NU, double>(N, a, st) : solve_tf<NX, NU, float>(N, a, st);
}

}  // namespace

// Shapes compiled in lq_small_env.hip (one for every nx + nu = 16 not compiled in lq_small.hip).
int small_env_count();
void small_env_shape(int i, int* nx, int* nu);
hipError_t launch_factor_small_env(lq_mode mode, int batch, int N, int nx, int nu, const lq_data& d, void* F,
                                   double* V, int32_t* info, hipStream_t st);
hipError_t launch_solve_small_env(lq_mode mode, int N, int nx, int nu, const SolveArgs& a, hipStream_t st);

}  // namespace lq
