/*
 * lqblocktri.h -- batched symmetric positive definite block-tridiagonal solves on gfx950:
 * cyclic reduction (CR), parallel cyclic reduction (PCR) and preconditioned conjugate gradients
 * (PCG), the solvers of the paper's Sec. "Cyclic reduction of block-tridiagonal linear systems"
 * and its appendix "Cyclic reduction and parallel cyclic reduction" (Alg. "cr", Alg. "pcr"; the
 * preconditioners of Sec. "Handling of the final scalar levels").
 *
 * System (eq. block-tri): Nb diagonal blocks M_k (n x n, symmetric positive definite), Nb - 1
 * subdiagonal blocks K_k (block row k + 1, block column k), right-hand side b:
 *   M_k x_k + K_{k-1} x_{k-1} + K_k^T x_{k+1} = b_k.
 * Nb need not be a power of two (neighbours outside 0..Nb-1 are absent; the system is not periodic).
 *
 * Conventions: every array pointer is a DEVICE pointer owned by the caller; float64, row-major:
 *   M [batch][Nb][n][n]   K [batch][Nb-1][n][n] (may be NULL when Nb == 1)
 *   b, x [batch][Nb][n]   info, iters [batch] (int32)   rel_res [batch] (float64).
 * Only the lower triangles of the M_k are read by the factorisations (the matrix-vector products
 * of PCG read M_k whole: pass symmetric blocks).  Limits: n <= 256, batch <= 65535.
 * Workspace: lq_bt_workspace_bytes(batch, Nb, n, method) bytes, 8-byte aligned, caller-owned.
 * Calls are asynchronous on `stream`.  Return values: LQ_OK (0), LQ_EINVAL (-1, missing pointer or
 * non-positive size), LQ_EUNSUPPORTED (-2, sizes above the limits), LQ_EHIP (-3, launch failure);
 * lq_last_error() (lqkkt.h) gives the message.  Numerical outcomes per system in `info`: 0, k + 1
 * when a block eliminated for block row k was not positive definite (its pivot replaced by 1),
 * -2 (PCG stopped at max_it above tol), -1 (PCG residual not finite).
 */
#ifndef LQBLOCKTRI_H
#define LQBLOCKTRI_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { LQ_BT_CR = 0, LQ_BT_PCR = 1, LQ_BT_PCG = 2 } lq_bt_method;

#define LQ_BT_PRECOND_JACOBI 0 /* block-Jacobi: D^{-1}, D = blkdiag(M_k)                              */
#define LQ_BT_PRECOND_STAIR 1  /* symmetric stair: D^{-1} (I - Koff D^{-1}), Koff the off-diagonal part */

/* Bytes of workspace a method needs for this batch (0 for non-positive sizes). */
size_t lq_bt_workspace_bytes(int32_t batch, int32_t Nb, int32_t n, lq_bt_method method);

/* Cyclic-reduction factorisation (Alg. "cr", factor part; Sec. "Cyclic reduction as block
 * Cholesky factorization"): level l = 0, 1, ... eliminates the block rows k with 2-adic valuation
 * l (k = 2^l (2i + 1)), block row 0 last.  The workspace receives, per system, the blocks L_k
 * (diagonal factor), U_k and Y_k (factor blocks in the rows k - 2^l and k + 2^l of column k) of the
 * Cholesky factor of the valuation-ordered matrix, in the layout
 *   [L: batch Nb n n][coupling scratch: batch Nb n n][U: batch Nb n n][Y: batch Nb n n]
 * (block k of system s at offset (s Nb + k) n n of its region; U_0 and Y_k with k + 2^l >= Nb are
 * not written).  info is written. */
int lq_bt_cr_factor(int32_t batch, int32_t Nb, int32_t n, const double* M, const double* K, void* workspace,
                    int32_t* info, hipStream_t stream);

/* Solution with the factors of lq_bt_cr_factor (same workspace): forward substitution level by
 * level, then the eliminated unknowns from the last level back (eq. cr-odd).  b is read, x
 * written (they must differ). */
int lq_bt_cr_solve(int32_t batch, int32_t Nb, int32_t n, const void* workspace, const double* b, double* x,
                   hipStream_t stream);

/* Parallel cyclic reduction (Alg. "pcr"): every level factors every diagonal block and
 * eliminates both neighbours at distance 2^l from every equation, until no coupling is left; then
 * x_k = M_k^{-1} b_k of the decoupled blocks.  info is written. */
int lq_bt_pcr_solve(int32_t batch, int32_t Nb, int32_t n, const double* M, const double* K, const double* b,
                    double* x, void* workspace, int32_t* info, hipStream_t stream);

/* Preconditioned conjugate gradients from x = 0, stopped when ||b - M x||_inf <= tol ||b||_inf or
 * after max_it iterations, with the block-Jacobi or the stair preconditioner (LQ_BT_PRECOND_*).
 * iters and rel_res (may be NULL) receive the iterations and the relative residual of the
 * returned x; info is written. */
int lq_bt_pcg(int32_t batch, int32_t Nb, int32_t n, const double* M, const double* K, const double* b, double* x,
              int32_t precond, double tol, int32_t max_it, void* workspace, int32_t* iters, double* rel_res,
              int32_t* info, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LQBLOCKTRI_H */
