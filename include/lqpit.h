/*
 * lqpit.h -- parallel-in-time solve of the LQ-OCP KKT system (the paper's Sec. "Cyqlone: parallel
 * factorization and solution of KKT systems with optimal control structure"): the horizon of every
 * instance is split into P intervals that are factored at the same time, coupled through the
 * multipliers of the dynamics at the interval boundaries, whose Schur complement (block-tridiagonal,
 * nx x nx blocks) is factored by cyclic reduction.
 *
 * Problem, data layout and sign convention: as lqkkt.h (eq. ocp-eq, eq. opt-cond-ocp-eq), for a
 * UNIFORM batch (every instance N, nx, nu); data arrays are device float64 in the packed layout of
 * lqkkt.h; S and f may be NULL.  Outputs x (x_1..x_N), u (u_0..u_{N-1}), lam (lam_0..lam_{N-1}) as
 * there.
 *
 * Method (own formulation of the paper's Cyqlone ordering, interval boundaries at
 * s_p = 1 + floor(p N / P), p = 0..P-1):
 *   - stage j (1 <= j < N) holds (u_j, x_j); the wrap stage N holds (u_0, x_N) with cost R_0, Q_N,
 *     no cross term, linear terms r_0 + S_0 x_init and q_N (x_0 = x_init is eliminated);
 *   - interval p holds the stages s_p .. s_{p+1} - 1 (the last interval ends with the wrap stage);
 *     the dynamics between its stages are eliminated by the interval's own Riccati recursion
 *     (Alg. "factor-block-column-riccati"): backward from its last stage, whose stage matrix gets
 *     no cost-to-go term, carrying the coupling (B^, A^) of the interval's outgoing dynamics
 *     constraint, L^B_j = B^_j (L^R_j)^{-T}, A^cl_j = A^_j - L^B_j (L^S_j)^T, (B^, A^)_{j-1} =
 *     A^cl_j (B_{j-1}, A_{j-1}), and at the first stage L^A = A^cl_s (L^Q_s)^{-T};
 *   - boundary multipliers beta_0 = lam_0 (wrap constraint x_1 = B_0 u_0 + f_0 + A_0 x_init) and
 *     beta_p = lam_{s_p - 1} (p >= 1); Schur complement (Sec. "Computation of the Schur complement"):
 *       D_p = (L^Q_{s_p})^{-T} (L^Q_{s_p})^{-1} + M^fwd_{p-1 mod P},  M^fwd = sum_j L^B_j L^B_j^T + L^A L^A^T,
 *       K_p (block row p+1, column p) = -L^A_(p) (L^Q_{s_p})^{-1};
 *     right-hand side: the coupling constraints at each interval's solution with zero boundary
 *     multipliers (free first state x_s = -P_s^{-1} p_s);
 *   - the Schur complement is factored and solved by cyclic reduction (lqblocktri.h), and each
 *     interval is solved again with the boundary multipliers as linear terms.
 *
 * Workspace: lq_pit_workspace_bytes(...) bytes of device memory, 256-byte aligned, caller-owned;
 * lq_pit_factor fills it with the factors (per stage L^R, L^S, L^Q in lqkkt.h's packed stage block,
 * stage j in slot j - 1; per interval L^A, M^fwd, L^Q_s; the cyclic-reduction factors of the
 * Schur complement); lq_pit_solve reads them for any right-hand side (q, r, f, x0 of `data`; the
 * matrices must be those given to lq_pit_factor).
 * Limits: 1 <= P <= N, nx <= 256, nu <= 256, batch <= 65535.
 * Status: return LQ_OK / LQ_EINVAL / LQ_EUNSUPPORTED / LQ_EHIP (lq_last_error() has the message);
 * per instance `info` (device int32[batch]): 0, j (>= 1) when stage j's matrix was not positive
 * definite, N + 1 + p when the Schur complement's block row p was not, -1 non-finite residual.
 * rel_res (device float64[batch], may be NULL) receives ||b - K z||_inf / ||b||_inf of the returned
 * solution (eq. opt-cond-ocp-eq).
 */
#ifndef LQPIT_H
#define LQPIT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "lqkkt.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes of workspace for a uniform batch split into P intervals (0 for invalid sizes). */
size_t lq_pit_workspace_bytes(int32_t batch, int32_t N, int32_t nx, int32_t nu, int32_t P);

/* Factorisation: the interval recursions (one workgroup per instance and interval), the Schur
 * complement blocks and their cyclic-reduction factorisation.  info is written. */
int lq_pit_factor(int32_t batch, int32_t N, int32_t nx, int32_t nu, int32_t P, const lq_data* data,
                  void* workspace, int32_t* info, hipStream_t stream);

/* Solution for the right-hand side in `data` with the factors in `workspace`: interval sweeps with
 * zero boundary multipliers, the Schur right-hand side, its cyclic-reduction solve, interval sweeps
 * with the boundary multipliers, the float64 KKT residual.  info is read (a factor code is kept)
 * and updated. */
int lq_pit_solve(int32_t batch, int32_t N, int32_t nx, int32_t nu, int32_t P, const lq_data* data,
                 void* workspace, double* x, double* u, double* lam, double* rel_res, int32_t* info,
                 hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LQPIT_H */
