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
 * 0 <= m <= LQ_UPDATE_MAX_ROWS; m = 0 (or upd = NULL) means no rows.  Plans with update rows need
 * nx <= 128 and at most 65535 instances.
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

/* Bytes of the device workspace lq_factor_update needs beside the plan's workspace when it is given
 * update rows (the state rows Phi_k of every stage, their signs and counts, a status per instance;
 * 256-byte aligned, caller-owned, no contents kept between calls).  0 if the plan cannot update. */
size_t lq_update_workspace_bytes(const lq_plan* plan);

/* Updates the factors in `workspace` (written by lq_factor for the data before the change, float64
 * plan without checkpoints) to those of the modified data, and recomputes the right-hand-side sweep
 * from `data` (its A, B, q, r, f; pass the modified data, e.g. after lq_update_data).  lq_solve with
 * the modified data then solves the modified problem.
 * Method (Alg. "fact-mod-riccati-update", one interval), three passes:
 *   1. per instance, backward in time: hyperbolic Householder transformations of the input pivots
 *      [L^R_k; L^S_k] with Upsilon_k = [B_k^T Phi_{k+1}, D_k^T; A_k^T Phi_{k+1}, C_k^T] (columns scaled
 *      by sqrt|dSigma|, signature sign dSigma), which leave Phi_k, stored in update_workspace;
 *   2. per (instance, stage), all at once: L^Q_k <- factor of L^Q_k L^Q_k^T + Phi_k S_k Phi_k^T;
 *   3. per instance: the right-hand-side sweep from the updated factors.
 * With no rows (upd NULL or m = 0) only pass 3 runs (update_workspace may be NULL): a new right-hand
 * side (q, r, f, x0) for unchanged matrices.  info (device int32[batch]) is written: 0, k + 1 when
 * the updated matrix of stage k is not positive definite (the highest such stage), -1 non-finite,
 * LQ_INFO_UPDATE_RANK (instance unchanged, its sweep too). */
int lq_factor_update(const lq_plan* plan, const lq_data* data, const lq_update* upd, void* workspace,
                     void* update_workspace, int32_t* info, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LQUPDATE_H */
