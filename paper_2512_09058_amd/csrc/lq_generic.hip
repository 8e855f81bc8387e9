// Generic kernels: one workgroup per instance, stage matrices staged in LDS, runtime sizes.
//
// They cover every (N, nx, nu) whose stage tile fits in LDS and every batch shape (uniform
// or ragged, via the per-instance descriptors).  The size-specialised kernels are faster;
// these are the general path and the one the uneven-batch scheduler falls back to.
//
// Factor sweep (paper, Alg. "factor-block-column-riccati" with one interval): per stage,
// backward in time,
//   V_k   = [B_k^T; A_k^T] L^Q_{k+1}                      (trmm)
//   Hhat  = [[R_k, S_k],[S_k^T, Q_k]] + V_k V_k^T          (syrk)
//   chol(Hhat) = [[L^R_k, 0],[L^S_k, L^Q_k]]               (potrf, always float64)
// starting from L^Q_N = chol(Q_N).  At k = 0 only the first nu pivot columns are needed
// (x_0 is fixed), which gives L^R_0 and L^S_0.
//
// Right-hand-side sweeps (the substitution phase of the block factorisation):
//   backward: p_N = q_N;  w = L^Q_{k+1} L^Q_{k+1}^T f_k + p_{k+1};
//             rbar_k = (L^R_k)^{-1} (r_k + B_k^T w);  p_k = q_k + A_k^T w - L^S_k rbar_k
//   forward:  x_0 = x_init;  u_k = -(L^R_k)^{-T} ((L^S_k)^T x_k + rbar_k);
//             x_{k+1} = A_k x_k + B_k u_k + f_k;  lam_k = L^Q_{k+1} L^Q_{k+1}^T x_{k+1} + p_{k+1}
// KKT residual (eq. opt-cond-ocp-eq, x_0 = x_init):
//   rho_u,k = -r_k - (R_k u_k + S_k x_k + B_k^T lam_k)
//   rho_x,k = -q_k - (S_k^T u_k + Q_k x_k + A_k^T lam_k - lam_{k-1})     (1 <= k < N)
//   rho_x,N = -q_N - (Q_N x_N - lam_{N-1})
//   rho_l,k = -f_k - (A_k x_k + B_k u_k - x_{k+1})
// A correction solves K dz = rho, i.e. the sweeps above with (r, q, f, x_init) replaced by
// (-rho_u, -rho_x, -rho_l, 0).  The adjoint system K zbar = (gu, gx, 0) uses (-gu, -gx, 0, 0).
#include <math.h>

#include "lq_internal.hpp"

namespace lq {
hipError_t raise_lds_limit(const void* kernel, size_t lds);  // lq_api.hip

__device__ __forceinline__ double rsqrt_f64(double a) {
  // hardware estimate (~2^-24) and two Newton steps: y <- y (3/2 - a/2 y^2)
  double y = __builtin_amdgcn_rsq(a);
  const double h = 0.5 * a;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

template <typename T>
__device__ __forceinline__ double rnd(double v) {
  return (double)(T)v;
}

// Right-looking Cholesky of the leading n x n block of H (row-major, leading dim ld), for
// pivot columns 0..ncol-1 (trailing update restricted to those columns).  Writes 1/L_jj to
// dinv.  Non-positive pivots are replaced by 1 and reported through *bad (1: not positive
// definite, 2: non-finite), the first time only.
__device__ void potrf_lds(double* H, int ld, int n, int ncol, double* dinv, int* bad) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int j = 0; j < ncol; ++j) {
    __syncthreads();
    double dj = H[j * ld + j];
    const bool fin = isfinite(dj);
    if (!(fin && dj > 0.0)) {
      if (tid == 0 && *bad == 0) *bad = fin ? 1 : 2;
      dj = 1.0;
    }
    const double inv = rsqrt_f64(dj);
    for (int i = j + 1 + tid; i < n; i += nt) H[i * ld + j] *= inv;
    if (tid == 0) {
      H[j * ld + j] = dj * inv;
      dinv[j] = inv;
    }
    __syncthreads();
    const int nr = n - j - 1, nc = ncol - j - 1;
    for (int e = tid; e < nr * nc; e += nt) {
      const int i = j + 1 + e / nc, c = j + 1 + e % nc;
      if (c <= i) H[i * ld + c] -= H[i * ld + j] * H[c * ld + j];
    }
  }
  __syncthreads();
}


// Factor sweep of stages kb-1 down to ka of one instance by the whole workgroup, starting from
// chol(Q_N) if kb = N, else from the stored L^Q_kb block `from`.  Stage k's block goes to
// dst(k) (nullptr: not stored).  With `rhs`, also the backward sweep of (q, r, f) into rbar, p
// and the pivot status into s_info.  Recomputing a range repeats exactly the arithmetic of the
// full sweep, so it reproduces the same factors bit for bit.
template <typename TF, typename TP, typename Dst>
__device__ void factor_range(const Desc& D, const lq_data& d, int ka, int kb, Dst dst, const TF* from,
                             double* __restrict__ rbar, double* __restrict__ pv, bool rhs, double* smem, int& s_bad,
                             int& s_info) {
  const int N = D.N, nx = D.nx, nu = D.nu, nux = nx + nu;
  const int tid = threadIdx.x, nt = blockDim.x;
  double* H = smem;              // nux*nux   (stage tile; also stages C = [B A])
  double* Lq = H + nux * nux;    // nx*nx     L^Q_{k+1}, full square, zero above the diagonal
  double* Vm = Lq + nx * nx;     // nux*nx
  double* pn = Vm + nux * nx;    // nx        p_{k+1}
  double* w = pn + nx;           // nx
  double* tq = w + nx;           // nux       (rhat, qhat)
  double* dinv = tq + nux;       // nux
  double* t1 = dinv + nux;       // nx

  const double* A = d.A + D.oA;
  const double* Bm = d.B + D.oB;
  const double* Q = d.Q + D.oQ;
  const double* R = d.R + D.oR;
  const double* S = d.S ? d.S + D.oS : nullptr;
  const double* q = d.q + D.oq;
  const double* r = d.r + D.or_;
  const double* f = d.f ? d.f + D.of : nullptr;

  if (tid == 0) { s_bad = 0; if (rhs) s_info = 0; }
  if (kb < N) {
    // L^Q_kb from its stored block
    for (int e = tid; e < nx * nx; e += nt) {
      const int i = e / nx, j = e % nx;
      Lq[e] = j <= i ? (double)from[off_LQ(nx, nu) + i * (i + 1) / 2 + j] : 0.0;
    }
    __syncthreads();
  } else {
    // ---- stage N: L^Q_N = chol(sym Q_N), p_N = q_N
    const double* QN = Q + (int64_t)N * nx * nx;
    for (int e = tid; e < nx * nx; e += nt) {
      const int i = e / nx, j = e % nx;
      H[e] = 0.5 * (QN[i * nx + j] + QN[j * nx + i]);
    }
    for (int i = tid; i < nx; i += nt) pn[i] = q[(int64_t)N * nx + i];
    __syncthreads();
    potrf_lds(H, nx, nx, nx, dinv, &s_bad);
    if (tid == 0 && s_bad) { if (rhs) s_info = s_bad == 2 ? LQ_INFO_NONFINITE : N + 1; s_bad = 0; }
    TF* FN = dst(N);
    for (int e = tid; e < nx * nx; e += nt) {
      const int i = e / nx, j = e % nx;
      const double v = j <= i ? rnd<TF>(H[e]) : 0.0;
      Lq[e] = v;
      if (FN && j <= i) FN[off_LQ(nx, nu) + i * (i + 1) / 2 + j] = (TF)v;
    }
    if (FN)
      for (int i = tid; i < nx; i += nt) FN[off_dQ(nx, nu) + i] = (TF)dinv[i];
    if (rhs)
      for (int i = tid; i < nx; i += nt) pv[(int64_t)N * nx + i] = pn[i];
    __syncthreads();
  }

  for (int k = kb - 1; k >= ka; --k) {
    const double* Ak = A + (int64_t)k * nx * nx;
    const double* Bk = Bm + (int64_t)k * nx * nu;
    // C = [B_k A_k] (nx x nux) staged in H with leading dimension nux
    for (int e = tid; e < nx * nux; e += nt) {
      const int m = e / nux, i = e % nux;
      H[e] = i < nu ? Bk[m * nu + i] : Ak[m * nx + (i - nu)];
    }
    // t1 = Lq^T f_k ; then w = Lq t1 + p_{k+1}
    for (int j = tid; j < nx; j += nt) {
      double s = 0.0;
      if (f) {
        const double* fk = f + (int64_t)k * nx;
        for (int m = j; m < nx; ++m) s += Lq[m * nx + j] * fk[m];
      }
      t1[j] = s;
    }
    __syncthreads();
    for (int i = tid; i < nx; i += nt) {
      double s = pn[i];
      if (f)
        for (int j = 0; j <= i; ++j) s += Lq[i * nx + j] * t1[j];
      w[i] = s;
    }
    __syncthreads();
    // (rhat, qhat) = (r_k, q_k) + C^T w ;  V = C^T Lq in the product precision
    for (int i = tid; i < nux; i += nt) {
      double s = i < nu ? r[(int64_t)k * nu + i] : (k > 0 ? q[(int64_t)k * nx + (i - nu)] : 0.0);
      for (int m = 0; m < nx; ++m) s += H[m * nux + i] * w[m];
      tq[i] = s;
    }
    for (int e = tid; e < nux * nx; e += nt) {
      const int i = e / nx, j = e % nx;
      TP s = 0;
      for (int m = j; m < nx; ++m) s += (TP)H[m * nux + i] * (TP)Lq[m * nx + j];
      Vm[e] = (double)s;
    }
    __syncthreads();
    // Hhat = [[R,S],[S^T,Q]] + V V^T (lower triangle; at k = 0 only the first nu columns)
    const int ncol = k > 0 ? nux : nu;
    const double* Rk = R + (int64_t)k * nu * nu;
    const double* Qk = Q + (int64_t)k * nx * nx;
    const double* Sk = S ? S + (int64_t)k * nu * nx : nullptr;
    for (int e = tid; e < nux * nux; e += nt) {
      const int i = e / nux, j = e % nux;
      if (j > i || j >= ncol) continue;
      double h;
      if (i < nu) h = 0.5 * (Rk[i * nu + j] + Rk[j * nu + i]);
      else if (j < nu) h = Sk ? Sk[j * nx + (i - nu)] : 0.0;
      else h = 0.5 * (Qk[(i - nu) * nx + (j - nu)] + Qk[(j - nu) * nx + (i - nu)]);
      TP s = 0;
      for (int m = 0; m < nx; ++m) s += (TP)Vm[i * nx + m] * (TP)Vm[j * nx + m];
      H[e] = h + (double)s;
    }
    __syncthreads();
    potrf_lds(H, nux, nux, ncol, dinv, &s_bad);
    if (tid == 0 && s_bad) {
      if (rhs && s_info == 0) s_info = s_bad == 2 ? LQ_INFO_NONFINITE : k + 1;
      s_bad = 0;
    }
    // round to the storage precision, store, keep L^Q_k for the next stage
    TF* Fk = dst(k);
    for (int e = tid; e < nux * nux; e += nt) {
      const int i = e / nux, j = e % nux;
      if (j > i || j >= ncol) continue;
      const double v = rnd<TF>(H[e]);
      H[e] = v;
      if (!Fk) continue;
      if (i < nu) Fk[i * (i + 1) / 2 + j] = (TF)v;
      else if (j < nu) Fk[off_LS(nx, nu) + (i - nu) * nu + j] = (TF)v;
      else Fk[off_LQ(nx, nu) + (i - nu) * (i - nu + 1) / 2 + (j - nu)] = (TF)v;
    }
    for (int i = tid; i < ncol; i += nt) {
      const double v = rnd<TF>(dinv[i]);
      dinv[i] = v;
      if (!Fk) continue;
      if (i < nu) Fk[off_dR(nx, nu) + i] = (TF)v;
      else Fk[off_dQ(nx, nu) + (i - nu)] = (TF)v;
    }
    __syncthreads();
    // rbar = L^R^{-1} rhat (forward substitution), p_k = qhat - L^S rbar
    if (tid == 0) {
      for (int i = 0; i < nu; ++i) {
        double s = tq[i];
        for (int j = 0; j < i; ++j) s -= H[i * nux + j] * tq[j];
        tq[i] = s * dinv[i];
      }
    }
    __syncthreads();
    if (rhs)
      for (int i = tid; i < nu; i += nt) rbar[(int64_t)k * nu + i] = tq[i];
    if (k > 0) {
      for (int i = tid; i < nx; i += nt) {
        double s = tq[nu + i];
        for (int j = 0; j < nu; ++j) s -= H[(nu + i) * nux + j] * tq[j];
        pn[i] = s;
        if (rhs) pv[(int64_t)k * nx + i] = s;
      }
      for (int e = tid; e < nx * nx; e += nt) {
        const int i = e / nx, j = e % nx;
        Lq[e] = j <= i ? H[(nu + i) * nux + (nu + j)] : 0.0;
      }
    }
    __syncthreads();
  }
}

// Full factor sweep of instance b (lq_factor): every stage block stored, or with a checkpoint
// stride s only the blocks of stages 0, s, 2s, ... and N.
template <typename TF, typename TP>
__device__ void factor_one(const Desc& D, int b, const lq_data& d, TF* __restrict__ F, double* __restrict__ Vws,
                           int32_t* __restrict__ info, int ckpt, double* smem, int& s_bad, int& s_info) {
  const int N = D.N;
  const int64_t fs = stage_factor_elems(D.nx, D.nu);
  TF* Fi = F + D.oF;
  double* rbar = Vws + D.oV;
  double* pv = rbar + (int64_t)N * D.nu;
  auto dst = [&](int k) -> TF* {
    if (ckpt == 0) return Fi + (int64_t)k * fs;
    if (k % ckpt == 0 || k == N) return Fi + ckpt_slot(k, N, ckpt) * fs;
    return nullptr;
  };
  factor_range<TF, TP>(D, d, 0, N, dst, (const TF*)nullptr, rbar, pv, true, smem, s_bad, s_info);
  if (threadIdx.x == 0) info[b] = s_info;
  __syncthreads();
}

// Work distribution shared by the generic kernels: without a counter, workgroup g takes the
// instance order[g] (one workgroup per instance; the order lists instances longest first, so
// the hardware dispatcher starts the long ones first).  With a counter, a persistent grid
// pulls positions from it until the batch is exhausted (every workgroup exits once the counter
// has passed batch).
template <typename F>
__device__ __forceinline__ void for_each_instance(int batch, const int32_t* order, int32_t* counter, F&& body) {
  __shared__ int s_next;
  if (counter == nullptr) {
    const int t = blockIdx.x;
    if (t < batch) body(order ? order[t] : t);
    return;
  }
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(counter, 1);
    __syncthreads();
    const int t = s_next;
    __syncthreads();
    if (t >= batch) break;
    body(order ? order[t] : t);
  }
}

template <int NT, typename TF, typename TP>
__global__ void __launch_bounds__(NT) k_factor_generic(const Desc* __restrict__ desc, int batch, lq_data d,
                                                       TF* __restrict__ F, double* __restrict__ Vws,
                                                       int32_t* __restrict__ info, const int32_t* __restrict__ order,
                                                       int32_t* counter, int ckpt) {
  extern __shared__ double smem[];
  __shared__ int s_bad, s_info;
  for_each_instance(batch, order, counter, [&](int b) {
    const Desc D = desc[b];
    factor_one<TF, TP>(D, b, d, F, Vws, info, ckpt, smem, s_bad, s_info);
  });
}

__global__ void k_reset_counter(int32_t* c) {
  if (threadIdx.x == 0) c[0] = 0;
}

// ------------------------------------------------------------------------------------------
// Solve: forward rollout, then (residual + correction backward sweep, forward correction)
// repeated until rel_res <= tol or max_it corrections.

struct InstView {
  int N, nx, nu;
  const double *A, *B, *Q, *R, *S, *q, *r, *f, *x0;  // problem data (S, f nullable)
  const double *gx, *gu;                              // adjoint right-hand side
  int rhs;
  double *x, *u, *lam;                                // iterate
};

// Right-hand-side accessors: (r_k, q_k, f_k, x_init) of the system being solved.
__device__ __forceinline__ double rhs_r(const InstView& v, int k, int i) {
  return v.rhs == RHS_PRIMAL ? v.r[(int64_t)k * v.nu + i] : -v.gu[(int64_t)k * v.nu + i];
}
__device__ __forceinline__ double rhs_q(const InstView& v, int k, int i) {  // 1 <= k <= N
  return v.rhs == RHS_PRIMAL ? v.q[(int64_t)k * v.nx + i] : -v.gx[(int64_t)(k - 1) * v.nx + i];
}
__device__ __forceinline__ double rhs_f(const InstView& v, int k, int i) {
  return (v.rhs == RHS_PRIMAL && v.f) ? v.f[(int64_t)k * v.nx + i] : 0.0;
}
__device__ __forceinline__ double rhs_x0(const InstView& v, int i) {
  return v.rhs == RHS_PRIMAL ? v.x0[i] : 0.0;
}

// Factor blocks of one instance.  Without checkpoints every stage has its block; with stride
// s > 0 the stages of the current segment [k0, k1) live in the segment buffer and stage k1 (a
// multiple of s, or N) in its checkpoint slot.
template <typename TF>
struct FactView {
  const TF* F;
  int64_t fs;
  int nx, nu;
  int N, s, k0, k1;
  __device__ const TF* blk(int k) const {
    if (s == 0) return F + (int64_t)k * fs;
    if (k >= k0 && k < k1) return F + (ckpt_slots(N, s) + (k - k0)) * fs;
    return F + ckpt_slot(k, N, s) * fs;
  }
  __device__ double LR(int k, int i, int j) const { return (double)blk(k)[i * (i + 1) / 2 + j]; }
  __device__ double dR(int k, int i) const { return (double)blk(k)[off_dR(nx, nu) + i]; }
  __device__ double LS(int k, int i, int j) const { return (double)blk(k)[off_LS(nx, nu) + i * nu + j]; }
  __device__ double LQ(int k, int i, int j) const { return (double)blk(k)[off_LQ(nx, nu) + i * (i + 1) / 2 + j]; }
};

// ---- LDS staging of the stage matrices of the solve sweeps.  A matrix (or a block of its rows)
// is copied into LDS with coalesced loads (consecutive threads read consecutive elements; rows
// padded to m + 1 doubles), then multiplied from there by groups of lanes per row (M x) or per
// column (M^T v), reduced with cross-lane shuffles.  Reading rows or columns per thread straight
// from global memory would touch a different cache line per lane.
struct Stage {
  double* buf;  // LDS staging buffer
  int cap;      // capacity in doubles (>= max(nx, nu) + 1)
};

__device__ __forceinline__ int block_rows(const Stage& s, int m) {
  const int r = s.cap / (m + 1);
  return r < 1 ? 1 : r;
}

// Element e of a block maps to (row, column) = divmod(e, width); the unrolled copies below walk it
// incrementally so that all loads of a batch are issued before the first store.
struct Walk {
  int i, j, di, dj, w;
  __device__ Walk(int e0, int step, int width) : w(width) {
    i = e0 / width;
    j = e0 - i * width;
    di = step / width;
    dj = step - di * width;
  }
  __device__ void next() {
    i += di;
    j += dj;
    if (j >= w) {
      j -= w;
      ++i;
    }
  }
};

constexpr int kStageUnroll = 16;

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  typedef double v __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
};
template <>
struct Vec16<float> {
  typedef float v __attribute__((ext_vector_type(4)));
  static constexpr int n = 4;
};

// rows [r0, r0 + nr) of a row-major matrix with m columns.  A 16-byte aligned source is read in
// 16-byte vectors, kStageUnroll of them in flight per thread before the first LDS store.
template <typename T>
__device__ void stage_dense(const Stage& s, const T* __restrict__ M, int m, int r0, int nr) {
  const int n = nr * m, ld = m + 1, nt = blockDim.x;
  const T* src = M + (int64_t)r0 * m;
  if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
    typedef typename Vec16<T>::v V;
    constexpr int W = Vec16<T>::n;
    const V* vs = reinterpret_cast<const V*>(src);
    const int nv = n / W;  // whole vectors; the tail below
    Walk wk(threadIdx.x * W, nt * W, m);
    for (int base = threadIdx.x; base < nv; base += kStageUnroll * nt) {
      V v[kStageUnroll];
#pragma unroll
      for (int u = 0; u < kStageUnroll; ++u) {
        const int e = base + u * nt;
        v[u] = vs[e < nv ? e : 0];
      }
#pragma unroll
      for (int u = 0; u < kStageUnroll; ++u) {
        if (base + u * nt < nv) {
          int i = wk.i, j = wk.j;
#pragma unroll
          for (int w = 0; w < W; ++w) {
            s.buf[i * ld + j] = (double)v[u][w];
            if (++j == m) {
              j = 0;
              ++i;
            }
          }
        }
        wk.next();
      }
    }
    for (int e = nv * W + threadIdx.x; e < n; e += nt) {
      const int i = e / m;
      s.buf[i * ld + (e - i * m)] = (double)src[e];
    }
    return;
  }
  Walk wk(threadIdx.x, nt, m);
  for (int base = threadIdx.x; base < n; base += kStageUnroll * nt) {
    T v[kStageUnroll];
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      const int e = base + u * nt;
      v[u] = e < n ? src[e] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      if (base + u * nt < n) s.buf[wk.i * ld + wk.j] = (double)v[u];
      wk.next();
    }
  }
}

// rows [r0, r0 + nr) of an n x n lower triangle stored packed by rows, zero above the diagonal
template <typename T>
__device__ void stage_tri(const Stage& s, const T* __restrict__ P, int n, int r0, int nr) {
  const int ld = n + 1, nt = blockDim.x, tot = nr * n;
  Walk wk(threadIdx.x, nt, n);
  for (int base = threadIdx.x; base < tot; base += kStageUnroll * nt) {
    T v[kStageUnroll];
    Walk w2 = wk;
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      const int r = r0 + w2.i;
      v[u] = (base + u * nt < tot && w2.j <= r) ? P[(int64_t)r * (r + 1) / 2 + w2.j] : T(0);
      w2.next();
    }
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      if (base + u * nt < tot) s.buf[wk.i * ld + wk.j] = (double)v[u];
      wk.next();
    }
  }
}

// lanes per dot product of length len (a power of two dividing 64)
__device__ __forceinline__ int dot_lanes(int len) { return len > 64 ? 16 : len > 16 ? 8 : len > 4 ? 4 : 1; }

__device__ __forceinline__ double group_sum(double a, int g) {
  for (int o = g >> 1; o > 0; o >>= 1) a += __shfl_xor(a, o);
  return a;
}

// out(i, sum_j M[i][j] x[j]) for the nr staged rows (m columns)
template <typename F>
__device__ void mv_rows(const Stage& s, int m, int nr, const double* x, F&& out) {
  const int ld = m + 1, g = dot_lanes(m), sub = threadIdx.x & (g - 1), per = blockDim.x / g;
  for (int i0 = 0; i0 < nr; i0 += per) {
    const int i = i0 + threadIdx.x / g;
    double a = 0.0;
    if (i < nr) {
      const double* row = s.buf + i * ld;
      for (int j = sub; j < m; j += g) a = fma(row[j], x[j], a);
    }
    a = group_sum(a, g);
    if (sub == 0 && i < nr) out(i, a);
  }
}

// out(j, sum_i M[i][j] v[i]) over the nr staged rows, for the m columns
template <typename F>
__device__ void mv_cols(const Stage& s, int m, int nr, const double* v, F&& out) {
  const int ld = m + 1, g = dot_lanes(nr), sub = threadIdx.x & (g - 1), per = blockDim.x / g;
  for (int j0 = 0; j0 < m; j0 += per) {
    const int j = j0 + threadIdx.x / g;
    double a = 0.0;
    if (j < m)
      for (int i = sub; i < nr; i += g) a = fma(s.buf[i * ld + j], v[i], a);
    a = group_sum(a, g);
    if (sub == 0 && j < m) out(j, a);
  }
}

// body(r0, nr) on each staged row block of an mr x m matrix, load(r0, nr) staging it
template <typename Ld, typename Body>
__device__ void for_blocks(const Stage& s, int mr, int m, Ld&& load, Body&& body) {
  const int R = block_rows(s, m);
  for (int r0 = 0; r0 < mr; r0 += R) {
    const int nr = mr - r0 < R ? mr - r0 : R;
    __syncthreads();
    load(r0, nr);
    __syncthreads();
    body(r0, nr);
  }
  __syncthreads();
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, l), hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __hiloint2double(hi, lo);
}

// Triangular solves with the staged L^R (nu x nu, leading dimension nu + 1) and its reciprocal
// diagonal dr: y = (L^R)^{-T} t (TRANS) or y = (L^R)^{-1} t.  Wavefront 0; for nu <= 64 lane j
// keeps entry j and step i publishes y_i with a lane read, otherwise the entries stay in LDS.
template <bool TRANS>
__device__ void tri_solve(const Stage& s, int nu, const double* dr, double* t, double* y) {
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x, ld = nu + 1;
  if (nu <= 64) {
    double a = lane < nu ? t[lane] : 0.0;
    for (int st = 0; st < nu; ++st) {
      const int i = TRANS ? nu - 1 - st : st;
      const double yi = readlane_d(a, i) * dr[i];
      if (lane == 0) y[i] = yi;
      const bool upd = TRANS ? lane < i : (lane > i && lane < nu);
      if (upd) a = fma(-(TRANS ? s.buf[i * ld + lane] : s.buf[lane * ld + i]), yi, a);
    }
  } else {
    for (int st = 0; st < nu; ++st) {
      const int i = TRANS ? nu - 1 - st : st;
      __builtin_amdgcn_s_waitcnt(0xc07f);
      __builtin_amdgcn_wave_barrier();
      const double yi = t[i] * dr[i];
      if (lane == 0) y[i] = yi;
      if (TRANS) {
        for (int j = lane; j < i; j += 64) t[j] = fma(-s.buf[i * ld + j], yi, t[j]);
      } else {
        for (int j = i + 1 + lane; j < nu; j += 64) t[j] = fma(-s.buf[j * ld + i], yi, t[j]);
      }
    }
  }
}

// forward sweep; mode 0: z = result (x_0 = x_init, f = f_k);  mode 1: z += result (x_0 = 0,
// f = flam_k from the preceding residual pass)
__device__ void fwd_init(const InstView& v, int mode, double* sm) {
  for (int i = threadIdx.x; i < v.nx; i += blockDim.x) sm[i] = mode == 0 ? rhs_x0(v, i) : 0.0;
  __syncthreads();
}

// stages ka..kb-1 of the forward sweep (state x_ka in sm[0..nx), set by fwd_init or the
// preceding range)
template <typename TF>
__device__ void fwd_sweep(const InstView& v, const FactView<TF>& fv, const double* rbar, const double* pv,
                          const double* flam, int mode, double* sm, const Stage& st, int ka, int kb) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nx = v.nx, nu = v.nu;
  double* xc = sm;        // nx   x_k
  double* xn = xc + nx;   // nx   x_{k+1}
  double* t = xn + nx;    // nu
  double* uu = t + nu;    // nu   u_k
  double* t2 = uu + nu;   // nx
  double* dr = t2 + nx;   // nu   1 / diag L^R_k
  for (int k = ka; k < kb; ++k) {
    const TF* blk = fv.blk(k);
    const TF* blk1 = fv.blk(k + 1);
    for (int j = tid; j < nu; j += nt) {
      t[j] = rbar[(int64_t)k * nu + j];
      dr[j] = (double)blk[off_dR(nx, nu) + j];
    }
    for (int i = tid; i < nx; i += nt) {
      xn[i] = mode == 0 ? rhs_f(v, k, i) : flam[(int64_t)k * nx + i];
      t2[i] = 0.0;
    }
    // t = rbar_k + (L^S_k)^T x_k
    for_blocks(
        st, nx, nu, [&](int r0, int nr) { stage_dense(st, blk + off_LS(nx, nu), nu, r0, nr); },
        [&](int r0, int nr) { mv_cols(st, nu, nr, xc + r0, [&](int j, double a) { t[j] += a; }); });
    // u_k = -(L^R_k)^{-T} t
    for_blocks(
        st, nu, nu, [&](int r0, int nr) { stage_tri(st, blk, nu, r0, nr); },
        [&](int r0, int nr) {
          if (nr == nu) tri_solve<true>(st, nu, dr, t, uu);
        });
    if (block_rows(st, nu) < nu && tid == 0) {  // L^R larger than the staging buffer
      for (int j = nu - 1; j >= 0; --j) {
        double a = t[j];
        for (int i = j + 1; i < nu; ++i) a -= fv.LR(k, i, j) * uu[i];
        uu[j] = a * dr[j];
      }
    }
    __syncthreads();
    for (int j = tid; j < nu; j += nt) uu[j] = -uu[j];
    // x_{k+1} = A_k x_k + B_k u_k + f_k
    const double* Ak = v.A + (int64_t)k * nx * nx;
    const double* Bk = v.B + (int64_t)k * nx * nu;
    for_blocks(
        st, nx, nx, [&](int r0, int nr) { stage_dense(st, Ak, nx, r0, nr); },
        [&](int r0, int nr) { mv_rows(st, nx, nr, xc, [&](int i, double a) { xn[r0 + i] += a; }); });
    for_blocks(
        st, nx, nu, [&](int r0, int nr) { stage_dense(st, Bk, nu, r0, nr); },
        [&](int r0, int nr) { mv_rows(st, nu, nr, uu, [&](int i, double a) { xn[r0 + i] += a; }); });
    // lam_k = L^Q_{k+1} (L^Q_{k+1})^T x_{k+1} + p_{k+1}
    const TF* LQ1 = blk1 + off_LQ(nx, nu);
    const bool one = block_rows(st, nx) >= nx;
    for_blocks(
        st, nx, nx, [&](int r0, int nr) { stage_tri(st, LQ1, nx, r0, nr); },
        [&](int r0, int nr) { mv_cols(st, nx, nr, xn + r0, [&](int j, double a) { t2[j] += a; }); });
    double* lk = v.lam + (int64_t)k * nx;
    double* xk = v.x + (int64_t)k * nx;
    auto emit = [&](int i, double a) {
      const double l = pv[(int64_t)(k + 1) * nx + i] + a;
      if (mode == 0) { lk[i] = l; xk[i] = xn[i]; }
      else { lk[i] += l; xk[i] += xn[i]; }
    };
    if (one) {
      mv_rows(st, nx, nx, t2, emit);
    } else {
      for_blocks(
          st, nx, nx, [&](int r0, int nr) { stage_tri(st, LQ1, nx, r0, nr); },
          [&](int r0, int nr) { mv_rows(st, nx, nr, t2, [&](int i, double a) { emit(r0 + i, a); }); });
    }
    for (int j = tid; j < nu; j += nt) {
      double* uk = v.u + (int64_t)k * nu;
      if (mode == 0) uk[j] = uu[j];
      else uk[j] += uu[j];
    }
    __syncthreads();
    for (int i = tid; i < nx; i += nt) xc[i] = xn[i];
    __syncthreads();
  }
}

__device__ __forceinline__ double block_max(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] = nan_max(red[tid], red[tid + s]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Symmetric-part product: acc += 1/2 (M + M^T) x over the staged rows of an n x n matrix.
__device__ void mv_sym(const Stage& s, int n, int r0, int nr, const double* x, double* acc) {
  mv_rows(s, n, nr, x, [&](int i, double a) { acc[r0 + i] += 0.5 * a; });
  __syncthreads();
  mv_cols(s, n, nr, x + r0, [&](int j, double a) { acc[j] += 0.5 * a; });
}

// Stage N rows of the residual (and p2_N of the correction sweep); mr, mb are per-thread maxima
// of |rho| and |b|, carried over the ranges and reduced at the end.
__device__ void resid_init(const InstView& v, bool sweep, double* p2, double* sm, const Stage& st, double& mr,
                           double& mb) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int N = v.N, nx = v.nx;
  double* pn = sm;        // nx
  double* ax = pn + nx;   // nx
  double* xk = ax + nx;   // nx
  mr = 0.0;
  mb = 0.0;
  const double* xN = v.x + (int64_t)(N - 1) * nx;
  for (int i = tid; i < nx; i += nt) {
    ax[i] = 0.0;
    xk[i] = xN[i];
  }
  const double* QN = v.Q + (int64_t)N * nx * nx;
  for_blocks(
      st, nx, nx, [&](int r0, int nr) { stage_dense(st, QN, nx, r0, nr); },
      [&](int r0, int nr) { mv_sym(st, nx, r0, nr, xk, ax); });
  for (int i = tid; i < nx; i += nt) {
    const double qi = rhs_q(v, N, i);
    const double rho = -qi - (ax[i] - v.lam[(int64_t)(N - 1) * nx + i]);
    mr = nan_max(mr, fabs(rho));
    mb = nan_max(mb, fabs(qi));
    pn[i] = -rho;
    if (sweep) p2[(int64_t)N * nx + i] = -rho;
  }
  __syncthreads();
}

// Residual rows of stages kb-1 down to ka; with `sweep`, the backward sweep of the correction
// right-hand side into (rbar2, p2) and -rho_l into flam.
template <typename TF>
__device__ void resid_bwd(const InstView& v, const FactView<TF>& fv, bool sweep, double* rbar2, double* p2,
                          double* flam, double* sm, const Stage& st, double& mr, double& mb, int ka, int kb) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nx = v.nx, nu = v.nu;
  double* pn = sm;          // nx   p2_{k+1}
  double* au = pn + nx;     // nu   R_sym u + S x_k + B^T lam_k
  double* al = au + nu;     // nx   A x_k + B u
  double* ax = al + nx;     // nx   S^T u + Q_sym x_k + A^T lam_k
  double* a0 = ax + nx;     // nx   A x_k (k = 0: part of b)
  double* s0 = a0 + nx;     // nu   S x_k (k = 0: part of b)
  double* xk = s0 + nu;     // nx
  double* uk = xk + nx;     // nu
  double* lk = uk + nu;     // nx
  double* w = lk + nx;      // nx   correction: -rho_l, then w
  double* t1 = w + nx;      // nx
  double* tq = t1 + nx;     // nux  (rhat, qhat)
  double* dr = tq + nx + nu;  // nu  1 / diag L^R_k
  double* yb = dr + nu;     // nu   rbar2_k
  for (int k = kb - 1; k >= ka; --k) {
    const double* Ak = v.A + (int64_t)k * nx * nx;
    const double* Bk = v.B + (int64_t)k * nx * nu;
    const double* Rk = v.R + (int64_t)k * nu * nu;
    const double* Qk = v.Q + (int64_t)k * nx * nx;
    const double* Sk = v.S ? v.S + (int64_t)k * nu * nx : nullptr;
    for (int i = tid; i < nx; i += nt) {
      xk[i] = k > 0 ? v.x[(int64_t)(k - 1) * nx + i] : rhs_x0(v, i);
      lk[i] = v.lam[(int64_t)k * nx + i];
      al[i] = 0.0;
      ax[i] = 0.0;
      a0[i] = 0.0;
      t1[i] = 0.0;
    }
    for (int j = tid; j < nu; j += nt) {
      uk[j] = v.u[(int64_t)k * nu + j];
      au[j] = 0.0;
      s0[j] = 0.0;
    }
    for_blocks(
        st, nu, nu, [&](int r0, int nr) { stage_dense(st, Rk, nu, r0, nr); },
        [&](int r0, int nr) { mv_sym(st, nu, r0, nr, uk, au); });
    if (Sk)
      for_blocks(
          st, nu, nx, [&](int r0, int nr) { stage_dense(st, Sk, nx, r0, nr); },
          [&](int r0, int nr) {
            mv_rows(st, nx, nr, xk, [&](int i, double a) { au[r0 + i] += a; s0[r0 + i] = a; });
            mv_cols(st, nx, nr, uk + r0, [&](int j, double a) { ax[j] += a; });
          });
    for_blocks(
        st, nx, nu, [&](int r0, int nr) { stage_dense(st, Bk, nu, r0, nr); },
        [&](int r0, int nr) {
          mv_rows(st, nu, nr, uk, [&](int i, double a) { al[r0 + i] += a; });
          mv_cols(st, nu, nr, lk + r0, [&](int j, double a) { au[j] += a; });
        });
    for_blocks(
        st, nx, nx, [&](int r0, int nr) { stage_dense(st, Ak, nx, r0, nr); },
        [&](int r0, int nr) {
          mv_rows(st, nx, nr, xk, [&](int i, double a) { al[r0 + i] += a; a0[r0 + i] = a; });
          mv_cols(st, nx, nr, lk + r0, [&](int j, double a) { ax[j] += a; });
        });
    if (k > 0)
      for_blocks(
          st, nx, nx, [&](int r0, int nr) { stage_dense(st, Qk, nx, r0, nr); },
          [&](int r0, int nr) { mv_sym(st, nx, r0, nr, xk, ax); });
    // residual rows of stage k
    for (int i = tid; i < nu; i += nt) {
      const double ri = rhs_r(v, k, i);
      const double rho = -ri - au[i];
      au[i] = -rho;  // correction right-hand side r = -rho_u
      mr = nan_max(mr, fabs(rho));
      mb = nan_max(mb, fabs(ri + (k == 0 ? s0[i] : 0.0)));
    }
    for (int i = tid; i < nx; i += nt) {
      const double fi = rhs_f(v, k, i);
      const double rho = -fi - (al[i] - v.x[(int64_t)k * nx + i]);
      mr = nan_max(mr, fabs(rho));
      mb = nan_max(mb, fabs(fi + (k == 0 ? a0[i] : 0.0)));
      w[i] = -rho;
      if (k > 0) {
        const double qi = rhs_q(v, k, i);
        const double rho2 = -qi - (ax[i] - v.lam[(int64_t)(k - 1) * nx + i]);
        mr = nan_max(mr, fabs(rho2));
        mb = nan_max(mb, fabs(qi));
        ax[i] = -rho2;  // q = -rho_x
      }
    }
    __syncthreads();
    if (!sweep) continue;
    // correction right-hand side: r = -rho_u (au), q = -rho_x (ax), f = -rho_l (w), x_init = 0
    const TF* blk = fv.blk(k);
    const TF* LQ1 = fv.blk(k + 1) + off_LQ(nx, nu);
    for (int i = tid; i < nx; i += nt) flam[(int64_t)k * nx + i] = w[i];
    for (int j = tid; j < nu; j += nt) dr[j] = (double)blk[off_dR(nx, nu) + j];
    // t1 = (L^Q_{k+1})^T f, then w = L^Q_{k+1} t1 + p2_{k+1}
    for_blocks(
        st, nx, nx, [&](int r0, int nr) { stage_tri(st, LQ1, nx, r0, nr); },
        [&](int r0, int nr) { mv_cols(st, nx, nr, w + r0, [&](int j, double a) { t1[j] += a; }); });
    for_blocks(
        st, nx, nx, [&](int r0, int nr) { stage_tri(st, LQ1, nx, r0, nr); },
        [&](int r0, int nr) { mv_rows(st, nx, nr, t1, [&](int i, double a) { w[r0 + i] = pn[r0 + i] + a; }); });
    // (rhat, qhat) = (r, q) + [B A]^T w
    for (int j = tid; j < nu; j += nt) tq[j] = au[j];
    for (int i = tid; i < nx; i += nt) tq[nu + i] = k > 0 ? ax[i] : 0.0;
    for_blocks(
        st, nx, nu, [&](int r0, int nr) { stage_dense(st, Bk, nu, r0, nr); },
        [&](int r0, int nr) { mv_cols(st, nu, nr, w + r0, [&](int j, double a) { tq[j] += a; }); });
    for_blocks(
        st, nx, nx, [&](int r0, int nr) { stage_dense(st, Ak, nx, r0, nr); },
        [&](int r0, int nr) { mv_cols(st, nx, nr, w + r0, [&](int j, double a) { tq[nu + j] += a; }); });
    // rbar2 = (L^R_k)^{-1} rhat
    for_blocks(
        st, nu, nu, [&](int r0, int nr) { stage_tri(st, blk, nu, r0, nr); },
        [&](int r0, int nr) {
          if (nr == nu) tri_solve<false>(st, nu, dr, tq, yb);
        });
    if (block_rows(st, nu) < nu && tid == 0) {
      for (int i = 0; i < nu; ++i) {
        double a = tq[i];
        for (int j = 0; j < i; ++j) a -= fv.LR(k, i, j) * yb[j];
        yb[i] = a * dr[i];
      }
    }
    __syncthreads();
    for (int j = tid; j < nu; j += nt) rbar2[(int64_t)k * nu + j] = yb[j];
    // p2_k = qhat - L^S_k rbar2
    if (k > 0) {
      for_blocks(
          st, nx, nu, [&](int r0, int nr) { stage_dense(st, blk + off_LS(nx, nu), nu, r0, nr); },
          [&](int r0, int nr) {
            mv_rows(st, nu, nr, yb, [&](int i, double a) {
              const double pk = tq[nu + r0 + i] - a;
              pn[r0 + i] = pk;
              p2[(int64_t)k * nx + r0 + i] = pk;
            });
          });
    }
  }
}

__device__ __forceinline__ double resid_final(double mr, double mb, double* red) {
  mr = block_max(mr, red);
  mb = block_max(mb, red);
  return rel_of(mr, mb);
}

template <typename TF>
__device__ void solve_one(const SolveArgs& a, int b, double* sm, double* red) {
  const Desc D = a.desc[b];
  InstView v;
  v.N = D.N; v.nx = D.nx; v.nu = D.nu;
  v.A = a.d.A + D.oA; v.B = a.d.B + D.oB; v.Q = a.d.Q + D.oQ; v.R = a.d.R + D.oR;
  v.S = a.d.S ? a.d.S + D.oS : nullptr; v.q = a.d.q + D.oq; v.r = a.d.r + D.or_;
  v.f = a.d.f ? a.d.f + D.of : nullptr; v.x0 = a.d.x0 + D.ox0;
  v.rhs = a.rhs;
  v.gx = a.gx ? a.gx + D.ox : nullptr;
  v.gu = a.gu ? a.gu + D.ou : nullptr;
  if (a.out_is_zb) {
    v.x = a.x + D.oZB;
    v.u = a.x + D.oZB + (int64_t)D.N * D.nx;
    v.lam = a.x + D.oZB + (int64_t)D.N * (D.nx + D.nu);
  } else {
    v.x = a.x + D.ox; v.u = a.u + D.ou; v.lam = a.lam + D.olam;
  }
  FactView<TF> fv;
  fv.F = (const TF*)a.F + D.oF;
  fv.fs = stage_factor_elems(D.nx, D.nu);
  fv.nx = D.nx; fv.nu = D.nu;
  fv.N = D.N; fv.s = a.ckpt; fv.k0 = 0; fv.k1 = 0;
  const int N = D.N, nx = D.nx, nu = D.nu;
  const int sc = a.ckpt;
  const double* rb0 = a.V + D.oV;
  const double* p0 = rb0 + (int64_t)N * nu;
  double* rb2 = a.V2 + D.oV2;
  double* p2 = rb2 + (int64_t)N * nu;
  double* flam = p2 + (int64_t)(N + 1) * nx;
  // with checkpoints the factor-sweep scratch comes first in LDS, the solve vectors after it
  double* fsm = sm;
  Stage st;
  st.buf = sc ? sm + a.lds_factor_doubles : sm;
  st.cap = a.stage_doubles;
  double* ssm = st.buf + st.cap;
  __shared__ int s_bad, s_info;
  TF* seg = (TF*)a.F + D.oF + (sc ? ckpt_slots(N, sc) * fv.fs : 0);
  auto recompute = [&](int k0, int k1) {  // factors of stages [k0, k1) into the segment buffer
    fv.k0 = k0;
    fv.k1 = k1;
    auto dst = [&](int k) -> TF* { return (k >= k0 && k < k1) ? seg + (int64_t)(k - k0) * fv.fs : nullptr; };
    const TF* from = (k1 < N) ? (const TF*)a.F + D.oF + ckpt_slot(k1, N, sc) * fv.fs : nullptr;
    factor_range<TF, TF>(D, a.d, k0, k1, dst, from, nullptr, nullptr, false, fsm, s_bad, s_info);
  };
  // forward pass over all stages (segment by segment with checkpoints)
  auto forward = [&](const double* rb, const double* pv, const double* fl, int mode) {
    fwd_init(v, mode, ssm);
    if (!sc) {
      fwd_sweep<TF>(v, fv, rb, pv, fl, mode, ssm, st, 0, N);
      return;
    }
    for (int k0 = 0; k0 < N; k0 += sc) {
      const int k1 = k0 + sc < N ? k0 + sc : N;
      recompute(k0, k1);
      fwd_sweep<TF>(v, fv, rb, pv, fl, mode, ssm, st, k0, k1);
    }
  };
  // residual (+ correction sweep) pass, backward over all stages
  auto residual = [&](bool sweep) -> double {
    double mr, mb;
    resid_init(v, sweep, p2, ssm, st, mr, mb);
    if (!sc) {
      resid_bwd<TF>(v, fv, sweep, rb2, p2, flam, ssm, st, mr, mb, 0, N);
    } else {
      for (int k1 = N; k1 > 0;) {
        const int k0 = ((k1 - 1) / sc) * sc;
        if (sweep) recompute(k0, k1);
        resid_bwd<TF>(v, fv, sweep, rb2, p2, flam, ssm, st, mr, mb, k0, k1);
        k1 = k0;
      }
    }
    return resid_final(mr, mb, red);
  };

  if (a.rhs == RHS_PRIMAL) {
    forward(rb0, p0, nullptr, 0);
  } else {
    // adjoint: backward sweep of (r, q, f) = (-gu, -gx, 0) first (lq_factor did the primal one)
    // The residual pass of the zero iterate gives exactly -rho = the right-hand side, so the
    // iterate is zeroed and one residual/sweep pass plus a forward correction gives zbar.
    for (int k = 0; k < N; ++k) {
      for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        v.x[(int64_t)k * nx + i] = 0.0;
        v.lam[(int64_t)k * nx + i] = 0.0;
      }
      for (int i = threadIdx.x; i < nu; i += blockDim.x) v.u[(int64_t)k * nu + i] = 0.0;
    }
    __syncthreads();
    residual(true);
    forward(rb2, p2, flam, 1);
  }
  int it = 0;
  double rel = 0.0;
  bool have = false;
  if (a.check || a.max_it > 0) {
    for (;;) {
      const bool more = it < a.max_it;
      rel = residual(more);
      have = true;
      if (!(rel > a.tol) || !more) break;  // converged (or NaN handled below) or out of iterations
      forward(rb2, p2, flam, 1);
      ++it;
    }
  }
  if (threadIdx.x == 0) {
    if (a.rel_res) a.rel_res[b] = have ? rel : NAN;
    if (a.iters) a.iters[b] = it;
    if (a.info) {
      int cur = a.info[b];
      if (cur <= 0) {
        int code = 0;
        if (have && !isfinite(rel)) code = LQ_INFO_NONFINITE;
        else if (have && a.max_it > 0 && rel > a.tol) code = LQ_INFO_NOT_CONVERGED;
        else if (cur == LQ_INFO_NONFINITE) code = cur;
        a.info[b] = code;
      }
    }
  }
  __syncthreads();
}

template <int NT, typename TF>
__global__ void __launch_bounds__(NT) k_solve_generic(SolveArgs a, const int32_t* __restrict__ order,
                                                      int32_t* counter) {
  extern __shared__ double sm[];
  __shared__ double red[NT];
  for_each_instance(a.batch, order, counter, [&](int b) { solve_one<TF>(a, b, sm, red); });
}

// Gradient outer products of the adjoint (one workgroup per instance).

__global__ void __launch_bounds__(128) k_grad_generic(GradArgs a) {
  const int b = blockIdx.x;
  if (b >= a.batch) return;
  const Desc D = a.desc[b];
  const int N = D.N, nx = D.nx, nu = D.nu;
  const int tid = threadIdx.x, nt = blockDim.x;
  const double* x = a.x + D.ox;
  const double* u = a.u + D.ou;
  const double* lam = a.lam + D.olam;
  const double* xb = a.ZB + D.oZB;
  const double* ub = xb + (int64_t)N * nx;
  const double* lb = ub + (int64_t)N * nu;
  const double* x0 = a.d.x0 + D.ox0;
#define XS(k, i) ((k) == 0 ? x0[i] : x[(int64_t)((k)-1) * nx + (i)])
#define XB(k, i) ((k) == 0 ? 0.0 : xb[(int64_t)((k)-1) * nx + (i)])
  for (int k = 0; k < N; ++k) {
    double* gA = a.gA + D.oA + (int64_t)k * nx * nx;
    for (int e = tid; e < nx * nx; e += nt) {
      const int i = e / nx, j = e % nx;
      gA[e] = -(lb[(int64_t)k * nx + i] * XS(k, j) + lam[(int64_t)k * nx + i] * XB(k, j));
    }
    double* gB = a.gB + D.oB + (int64_t)k * nx * nu;
    for (int e = tid; e < nx * nu; e += nt) {
      const int i = e / nu, j = e % nu;
      gB[e] = -(lb[(int64_t)k * nx + i] * u[(int64_t)k * nu + j] + lam[(int64_t)k * nx + i] * ub[(int64_t)k * nu + j]);
    }
    double* gR = a.gR + D.oR + (int64_t)k * nu * nu;
    for (int e = tid; e < nu * nu; e += nt) {
      const int i = e / nu, j = e % nu;
      gR[e] = -0.5 * (ub[(int64_t)k * nu + i] * u[(int64_t)k * nu + j] + u[(int64_t)k * nu + i] * ub[(int64_t)k * nu + j]);
    }
    if (a.gS) {
      double* gS = a.gS + D.oS + (int64_t)k * nu * nx;
      for (int e = tid; e < nu * nx; e += nt) {
        const int i = e / nx, j = e % nx;
        gS[e] = -(ub[(int64_t)k * nu + i] * XS(k, j) + u[(int64_t)k * nu + i] * XB(k, j));
      }
    }
    for (int j = tid; j < nu; j += nt) a.gr[D.or_ + (int64_t)k * nu + j] = -ub[(int64_t)k * nu + j];
    if (a.gf)
      for (int i = tid; i < nx; i += nt) a.gf[D.of + (int64_t)k * nx + i] = -lb[(int64_t)k * nx + i];
  }
  for (int k = 0; k <= N; ++k) {
    double* gQ = a.gQ + D.oQ + (int64_t)k * nx * nx;
    for (int e = tid; e < nx * nx; e += nt) {
      const int i = e / nx, j = e % nx;
      gQ[e] = k == 0 ? 0.0 : -0.5 * (XB(k, i) * XS(k, j) + XS(k, i) * XB(k, j));
    }
    for (int i = tid; i < nx; i += nt) a.gq[D.oq + (int64_t)k * nx + i] = k == 0 ? 0.0 : -XB(k, i);
  }
  const double* A0 = a.d.A + D.oA;
  const double* S0 = a.d.S ? a.d.S + D.oS : nullptr;
  for (int j = tid; j < nx; j += nt) {
    double s = 0.0;
    for (int i = 0; i < nx; ++i) s += A0[i * nx + j] * lb[i];
    if (S0)
      for (int i = 0; i < nu; ++i) s += S0[i * nx + j] * ub[i];
    a.gx0[D.ox0 + j] = -s;
  }
#undef XS
#undef XB
}

// ------------------------------------------------------------------------------------------
// Host-side launchers (called from the runtime).

size_t generic_factor_lds(int nx, int nu) {
  const int nux = nx + nu;
  return sizeof(double) * ((size_t)nux * nux + (size_t)nx * nx + (size_t)nux * nx + 3 * nx + 2 * nux);
}
// LDS of the solve: the staging buffer (the largest stage matrix, at most 12288 doubles; larger
// ones go through in row blocks) and the sweep vectors.
size_t generic_stage_doubles(int nx, int nu) {
  const size_t m = nx > nu ? nx : nu;
  const size_t full = m * (m + 1);
  return full < 12288 ? full : (12288 > m + 1 ? 12288 : m + 1);
}
size_t generic_solve_lds(int nx, int nu) { return sizeof(double) * (size_t)(9 * nx + 6 * nu); }

template <int NT>
static hipError_t factor_nt(lq_mode mode, const Desc* desc, int batch, const lq_data& d, void* F, double* V,
                            int32_t* info, size_t lds, const GenericLaunch& c, hipStream_t st) {
  const dim3 grid(c.counter ? c.grid : batch), block(NT);
  if (mode == LQ_F64)
    hipLaunchKernelGGL((k_factor_generic<NT, double, double>), grid, block, lds, st, desc, batch, d, (double*)F, V,
                       info, c.order, c.counter, c.ckpt);
  else
    hipLaunchKernelGGL((k_factor_generic<NT, float, float>), grid, block, lds, st, desc, batch, d, (float*)F, V,
                       info, c.order, c.counter, c.ckpt);
  return hipGetLastError();
}

hipError_t launch_factor_generic(lq_mode mode, const Desc* desc, int batch, const lq_data& d, void* F,
                                 double* V, int32_t* info, size_t lds, const GenericLaunch& c, hipStream_t st) {
  if (c.counter) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, c.counter);
  }
  switch (c.threads) {
    case 64: return factor_nt<64>(mode, desc, batch, d, F, V, info, lds, c, st);
    case 256: return factor_nt<256>(mode, desc, batch, d, F, V, info, lds, c, st);
    case 512: return factor_nt<512>(mode, desc, batch, d, F, V, info, lds, c, st);
    default: return factor_nt<128>(mode, desc, batch, d, F, V, info, lds, c, st);
  }
}

template <int NT>
static hipError_t solve_nt(lq_mode mode, const SolveArgs& a, size_t lds, const GenericLaunch& c, hipStream_t st) {
  const dim3 grid(c.counter ? c.grid : a.batch), block(NT);
  if (mode == LQ_F64)
    hipLaunchKernelGGL((k_solve_generic<NT, double>), grid, block, lds, st, a, c.order, c.counter);
  else
    hipLaunchKernelGGL((k_solve_generic<NT, float>), grid, block, lds, st, a, c.order, c.counter);
  return hipGetLastError();
}

hipError_t launch_solve_generic(lq_mode mode, const SolveArgs& a, size_t lds, const GenericLaunch& c,
                                hipStream_t st) {
  if (c.counter) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, c.counter);
  }
  switch (c.threads) {
    case 64: return solve_nt<64>(mode, a, lds, c, st);
    case 256: return solve_nt<256>(mode, a, lds, c, st);
    case 512: return solve_nt<512>(mode, a, lds, c, st);
    default: return solve_nt<128>(mode, a, lds, c, st);
  }
}

// Raise the dynamic-LDS limit of every generic factor instantiation (done once per plan, not
// inside calls, so the calls stay capturable in a graph).
template <int NT>
static const void* generic_kernel(bool factor, lq_mode mode) {
  if (factor)
    return mode == LQ_F64 ? (const void*)k_factor_generic<NT, double, double> : (const void*)k_factor_generic<NT, float, float>;
  return mode == LQ_F64 ? (const void*)k_solve_generic<NT, double> : (const void*)k_solve_generic<NT, float>;
}

static const void* generic_kernel(int threads, bool factor, lq_mode mode) {
  switch (threads) {
    case 64: return generic_kernel<64>(factor, mode);
    case 256: return generic_kernel<256>(factor, mode);
    case 512: return generic_kernel<512>(factor, mode);
    default: return generic_kernel<128>(factor, mode);
  }
}

// Raise the dynamic-LDS limit of the generic factor (factor = true) or solve instantiations (done
// once per plan, not inside calls, so the calls stay capturable in a graph).
hipError_t prepare_generic(bool factor, size_t lds) {
  hipError_t e = hipSuccess;
  for (int t : {64, 128, 256, 512})
    for (lq_mode m : {LQ_F64, LQ_MIXED_F32}) {
      hipError_t r =
          raise_lds_limit(generic_kernel(t, factor, m), lds);
      if (r != hipSuccess) e = r;
    }
  return e;
}

// Workgroups of the generic kernels that fit on one CU at the given LDS size.
int generic_blocks_per_cu(int threads, size_t lds, bool factor, lq_mode mode) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, generic_kernel(threads, factor, mode), threads, lds) !=
      hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n > 0 ? n : 1;
}

hipError_t launch_grad_generic(const GradArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_generic, dim3(a.batch), dim3(128), 0, st, a);
  return hipGetLastError();
}

}  // namespace lq
