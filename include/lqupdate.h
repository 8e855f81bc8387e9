/*
 * lqupdate.h -- factorisation updates of the stored Riccati factors (the paper's Sec.
 * "Factorization updates" and Alg. "fact-mod-riccati-update", one interval) and a new right-hand
 * side for stored factors.
 *
 * Changes of the penalty factors of constraint rows (D_j u_j + C_j x_j) change the stage Hessians
 * by a low-rank term (eq. low-rank-update-Hj):
 *   R_j += D_j^T dSigma_j D_j,   S_j += D_j^T dSigma_j C_j,   Q_j += C_j^T dSigma_j C_j,
 * dSigma_j diagonal (positive entries: rows entering, negative: rows leaving the active set; the
 * modified stage Hessians must stay positive definite).  Instead of a new lq_factor, the stored
 * factors are updated by hyperbolic Householder transformations, stage by stage backward in time.
 *
 * Update rows (lq_update), m rows per stage, DEVICE float64 arrays in the plan's instance order,
 * row-major, owned by the caller:
 *   C     instance i at element m * (offset of q_i) (lq_plan_offsets(plan, LQ_ARR_q)):
 *         [N_i + 1][m][nx_i]  (stages 0..N; stage 0's rows multiply the fixed initial state)
 *   D     instance i at element m * (offset of r_i): [N_i][m][nu_i]  (stages 0..N-1)
 *   dsig  instance i at element m * sum_{l < i} (N_l + 1): [N_i + 1][m]  (0: row unchanged)
 * 0 <= m <= LQ_UPDATE_MAX_ROWS; m = 0 (or upd = NULL) means no rows.
 *
 * Status: return LQ_OK / LQ_EINVAL / LQ_EUNSUPPORTED / LQ_EHIP (lq_last_error() has the message).
 * Calls are asynchronous on `stream`.
 */
#ifndef LQUPDATE_H
#define LQUPDATE_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "lqkkt.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LQ_UPDATE_MAX_ROWS 64
/* info of lq_factor_update: the nonzero rows of the instance exceed lq_update_max_columns(plan);
 * nothing of that instance was changed -- factor it again with lq_factor (the paper's rule:
 * refactor when the rank of the change is large). */
#define LQ_INFO_UPDATE_RANK (-3)

typedef struct {
  int32_t m;
  const double* C;
  const double* D;
  const double* dsig;
} lq_update;

/* Applies the rows to the problem data in place (eq. low-rank-update-Hj): Q, R, S are the device
 * arrays of the plan's packed layout (lqkkt.h), S required.  Q_0 is changed too (it multiplies the
 * fixed x_0 and does not enter the solution). */
int lq_update_data(const lq_plan* plan, const lq_update* upd, double* Q, double* R, double* S,
                   hipStream_t stream);

/* Largest number of nonzero rows per instance (summed over its stages) that lq_factor_update takes
 * for this plan (limited by the LDS that holds Upsilon; 0 if the plan's stages do not fit). */
int32_t lq_update_max_columns(const lq_plan* plan);

/* Updates the factors in `workspace` (written by lq_factor for the data before the change, float64
 * plan without checkpoints) to those of the modified data, by the hyperbolic Householder recursion
 * of Alg. "fact-mod-riccati-update", and recomputes the right-hand-side sweep from `data` (its A, B,
 * q, r, f; pass the modified data, e.g. after lq_update_data).  lq_solve with the modified data then
 * solves the modified problem.  With no rows only the right-hand-side sweep is recomputed: a new
 * right-hand side (q, r, f, x0) for unchanged matrices.  info (device int32[batch]) is written: 0,
 * k + 1 when the updated matrix of stage k is not positive definite, -1 non-finite,
 * LQ_INFO_UPDATE_RANK (instance unchanged). */
int lq_factor_update(const lq_plan* plan, const lq_data* data, const lq_update* upd, void* workspace,
                     int32_t* info, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LQUPDATE_H */
