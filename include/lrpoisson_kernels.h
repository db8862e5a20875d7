/*
 * lrpoisson_kernels.h -- the cross approximation's building blocks as entry
 * points of their own, so that each can be checked against reference linear
 * algebra (and reused): the calls below run exactly the kernel sequences a
 * solve runs, on caller data.
 *
 * Conventions: as in lrpoisson.h (float64, column-major, device memory for
 * matrices, ``stream`` a hipStream_t, the call returns after its work
 * completed; LRP_EINVAL for invalid arguments before any device work).
 */
#ifndef LRPOISSON_KERNELS_H
#define LRPOISSON_KERNELS_H

#include "lrpoisson.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Householder TSQR of a tall panel, then maxvol on its orthonormal factor:
 * the orthonormal basis a cross step builds before choosing its pivots
 * (Section 3: QR of the factors; Section 4.2: maximal-volume rows by the
 * maxvol algorithm).
 *  A: n x k (lda >= n, read only), 1 <= k <= LRP_MAX_RANK, k <= n <=
 *     LRP_MAX_N.
 *  Q: n x k (ldq >= n), written: orthonormal columns with A = Q R.
 *  R: k x k (ldr >= k), written: upper triangular (zeros below).
 *  rows: host array of k int32, written: the maxvol rows I of Q, distinct,
 *     in [0, n).  B = Q Q[I,:]^-1 has B[I,:] = identity and
 *     max |B| <= tau up to the float32 rounding of the check that finds
 *     violators (tau > 1; 0 takes the solver's default 1.05).
 *  converged: host int32, written: 1 when a check/swap round found no
 *     entry of B above tau (the rounds continue, up to 67, until one does;
 *     a cross step runs three per sweep and resumes in the next), else 0
 *     (the rows are then the best found so far).
 * A rank-deficient A is allowed (Q stays orthonormal; maxvol then picks
 * rows of a nonsingular Q[I,:] all the same). */
lrp_status lrp_kernel_qr_maxvol(lrp_ctx *ctx, int64_t n, int32_t k, const double *A,
                                int64_t lda, double tau, double *Q, int64_t ldq,
                                double *R, int64_t ldr, int32_t *rows, int32_t *converged,
                                void *stream);

/* The one-sided (Hestenes) Jacobi SVD of the rounding core (Section 3: the
 * SVD of the small core after the QR of the factors):
 *  M: k x k (ldm >= k, read only), 1 <= k <= LRP_MAX_RANK.
 *  W, Z: k x k (leading dimension k), sigma: k, written, with
 *     M = W diag(sigma) Z^T, sigma descending (ties: lower column first),
 *     Z orthogonal, W's columns orthonormal where sigma > 0 and zero where
 *     sigma = 0. */
lrp_status lrp_kernel_core_svd(lrp_ctx *ctx, int32_t k, const double *M, int64_t ldm,
                               double *W, double *sigma, double *Z, void *stream);

/* Rounding of a low-rank product (Section 3's rounding, for the sums of
 * low-rank matrices that the Stokes driver forms; Section 5): X = U V^T with
 * U, V: n x K (ld >= n, read only), 16 <= n <= LRP_MAX_N, K >= 0 (any
 * number of columns), to the relative Frobenius accuracy eps in (0, 1):
 * Ux (n x rmax, ldx >= n, written: carries the scale) and Vx (orthonormal
 * columns) of rank *rank_out.  Randomized range finder: a Gaussian sketch of
 * min(64, n) columns, one power step, TSQR twice and the Jacobi core SVD;
 * LRP_ERANKCAP when the rank exceeds rmax or comes within 8 of the sketch
 * width (*rank_out then holds the rank found; outputs unwritten). */
lrp_status lrp_lowrank_round(lrp_ctx *ctx, int64_t n, int32_t K, const double *U,
                             const double *V, int64_t ld, double eps, double *Ux, double *Vx,
                             int64_t ldx, int32_t rmax, int32_t *rank_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LRPOISSON_KERNELS_H */
