// Shared definitions of the QP kernels (lq_qp.hip) and their driver (lq_api.hip).
#pragma once
#include "lq_internal.hpp"
#include "lqqp.h"

namespace lq {

struct QPArgs {
  const Desc* desc;
  int32_t batch, m;
  lq_data d;                     // the problem (cost and dynamics)
  const double *C, *D, *bl, *bu;  // constraint rows
  double *Qn, *Rn, *Sn, *qn, *rn, *x0n;  // Newton systems (LQ data layout; no f: they have f = 0)
  double *x, *u, *y;             // iterate (output layout), multipliers of the rows
  double *dx, *du, *dlam;        // Newton solution (output layout)
  double *qc, *rc, *fc;          // refinement of a parallel-in-time Newton solve: right-hand side
  double *cdx, *cdu, *cdlam;     //   (data layout) and correction (output layout)
  double *xbar, *ubar;           // proximal centre (output layout)
  double *sig, *w, *gd, *e, *eprev;  // per row
  double *part;                  // per (instance, stage): partial sums
  double *tau;                   // per instance
  int32_t* fl;                   // per instance: flags
  double sigma0, ginv, eps, theta, sigma_up, sigma_max, inner_tol;
  int32_t warm;
  int64_t omats;  // stage-parallel kernels with staged stage matrices: their offset in dynamic LDS (doubles)
  int64_t orbuf;  // rollouts with staged stages: offset of their two LDS slots (doubles; 0: none)
};

// Byte offsets of the QP workspace.
struct QPLayout {
  size_t oQn, oRn, oSn, oqn, orn, ox0n, odx, odu, odlam, oqc, orc, ofc, ocdx, ocdu, ocdlam, oxb, oub, osig, ow,
      ogd, oe, oep, opart, otau, ofl, orel, oinfo, ocnt, total;
};

// totals: elements of Q, R, S, q, r, f, x0, x, u, lam in the plan's layout; sumK = sum (N + 1).
QPLayout qp_layout(const int64_t* totals, int64_t sumK, int batch, int m);
QPArgs qp_args(const Desc* desc, int batch, int m, const lq_data& d, const lq_qp_constraints& c,
               const lq_qp_opts& op, void* ws, const QPLayout& L, double* x, double* u, double* y);
// which: 0 start, 1 Newton systems, 2 direction + search + step + count of inner loops running,
// 3 outer step + count of instances running (the counts go to *out).
hipError_t qp_launch(int which, const QPArgs& a, int maxN, int nxmax, int numax, hipStream_t st, const int32_t* info,
                     int32_t* out);
// One refinement step of a parallel-in-time Newton solve (which 0: the Newton system's KKT residual
// at (dx, du, dlam) as the right-hand side (qc, rc, fc) of a correction system with x_init = 0;
// which 1: (dx, du, dlam) += the correction).  tot: elements of x, u, lam (plan layout).
hipError_t qp_refine(int which, const QPArgs& a, int maxN, int nxmax, int numax, const int64_t* tot, hipStream_t st);
hipError_t qp_finish(const QPArgs& a, double* lam, int32_t* status, int32_t* iters, hipStream_t st);

}  // namespace lq
