/*
 * lqqp.h -- box-constrained LQ optimal-control QPs solved on the GPU by the proximal augmented
 * Lagrangian method whose inner problems are minimised by semismooth Newton steps (the paper's
 * Sec. "Solving problems with inequality constraints": eq. ocp-al, eq. ocp-al-funcs,
 * eq. qpalm-ocp-hessians, eq. newton-sys-with-x0, eq. elim-x0) with the exact line search of
 * Sec. "Parallel exact line search" (eq. psi-prime, the bisection over breakpoints).  The Newton
 * systems have the structure of eq. opt-cond-ocp-eq and are solved by lq_factor / lq_solve.
 *
 * Problem: the LQ problem of `data` (lqkkt.h layout and conventions) plus, per stage j,
 *   bl_j <= C_j x_j + D_j u_j <= bu_j   (j = 0..N-1, x_0 = x_init fixed),   bl_N <= C_N x_N <= bu_N,
 * with m rows per stage (+-inf bounds allowed).  Constraint arrays (DEVICE float64, caller-owned),
 * instance i of the plan at:
 *   C   m * (offset of q_i):              [N_i + 1][m][nx_i]
 *   D   m * (offset of r_i):              [N_i][m][nu_i]
 *   bl, bu, y (multipliers)  m * sum_{l < i} (N_l + 1):  [N_i + 1][m]
 * x, u, lam in the plan's output layout (lqkkt.h).
 *
 * Method (constants in lq_qp_opts; these outer rules follow the QPALM papers the method cites):
 *   start: u = 0 (or the given u when warm), x simulated from x_init, y = 0 (or the given y),
 *   Sigma = sigma0, Gamma = gamma I, proximal centre = the start;
 *   inner: generalised Hessian and gradient of the augmented Lagrangian at the iterate (active rows
 *   (Cx + Du + y / Sigma) outside [bl, bu]), Newton direction by lq_factor + lq_solve, or with
 *   intervals > 1 by the parallel-in-time lq_pit_factor + lq_pit_solve (the iterate satisfies the
 *   dynamics, so the direction's dynamics residual is 0), exact step along it; the
 *   inner loop of an instance ends when its inner stationarity residual ||grad + M^T lam||_inf is at
 *   most inner_tol max(1, ||z||_inf, ||yhat||_inf), when a full step changes no row's activity, or
 *   after max_inner steps; a step is u <- u + tau du with x simulated again from u (x + tau dx in exact
 *   arithmetic; the dynamics stay exact whatever the accuracy of the Newton solve);
 *   outer: y <- yhat, stop when ||Cx + Du - Pi(Cx + Du + y / Sigma)||_inf <= eps and
 *   ||z - zbar||_inf / gamma <= eps, else Sigma_i <- min(sigma_max, sigma_up Sigma_i) on rows whose
 *   violation did not fall below theta times the previous one, centre <- z.
 * Outputs: x, u (the QP solution), lam (multipliers of the dynamics), y (of the bounds: positive at
 * an active upper bound, negative at a lower one), status[batch] (0 converged, 1 max_outer reached,
 * 2 a Newton factorisation failed), iters[batch] (inner steps taken).
 * Requirements: a float64 plan without checkpoints; m <= 256; intervals > 1 needs a uniform plan
 * and 1 < intervals <= N.  The call synchronises with the host
 * once per inner step (the loops end when every instance is done).
 */
#ifndef LQQP_H
#define LQQP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "lqkkt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t m;
  const double* C;
  const double* D;
  const double* bl;
  const double* bu;
} lq_qp_constraints;

typedef struct {
  double sigma0;     /* initial penalty (e.g. 1e2) */
  double gamma;      /* proximal weight: Gamma = gamma I (e.g. 1e7) */
  double eps;        /* outer tolerance (e.g. 1e-9) */
  double theta;      /* penalty rows grow unless their violation fell below theta x previous (0.25) */
  double sigma_up;   /* growth factor (10) */
  double sigma_max;  /* cap (1e9) */
  double inner_tol;  /* inner stationarity tolerance, relative (1e-11) */
  int32_t max_outer; /* e.g. 100 */
  int32_t max_inner; /* per outer iteration, e.g. 50 */
  int32_t warm;      /* 1: start from the u and y passed in */
  int32_t intervals; /* 0 or 1: Newton systems by lq_factor / lq_solve; P > 1: by the parallel-in-time
                        lq_pit_factor / lq_pit_solve with P intervals (uniform plans; lqpit.h) */
} lq_qp_opts;

/* Bytes of the QP workspace (the Newton systems' data, the direction, the rows' state, partial
 * sums, per-instance flags, and with intervals > 1 the parallel-in-time factors; 256-byte aligned,
 * caller-owned) for this plan, m rows per stage and the number of intervals (0 or 1: serial). */
size_t lq_qp_workspace_bytes(const lq_plan* plan, int32_t m, int32_t intervals);

/* Solves every instance's QP.  plan_workspace: lq_plan_workspace_bytes(plan) bytes (the Newton
 * factors of the serial path); qp_workspace: lq_qp_workspace_bytes(plan, m, opts->intervals) bytes.  Returns LQ_OK / LQ_EINVAL /
 * LQ_EUNSUPPORTED / LQ_EHIP; per-instance outcomes in status and iters (device int32[batch]). */
int lq_qp_solve(const lq_plan* plan, const lq_data* data, const lq_qp_constraints* cons, const lq_qp_opts* opts,
                void* plan_workspace, void* qp_workspace, double* x, double* u, double* lam, double* y,
                int32_t* status, int32_t* iters, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LQQP_H */
