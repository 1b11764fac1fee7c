/*
 * zolo_blocks.h - building blocks of the Zolo-PD library, exported for
 * kernel-level checks and benchmarks.  Same conventions as zolo.h: FP64,
 * column-major, device pointers for matrices, host pointers for scalar arrays,
 * work queued on the handle's stream and complete on return, LAPACK-style
 * negative return for an invalid argument, 4 for a HIP error.
 */
#ifndef ZOLO_BLOCKS_H
#define ZOLO_BLOCKS_H

#include "zolo.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C_b = alpha op(A_b) op(B_b) + beta C_b for b < batch (op = transpose when
 * trans* != 0), on the FP64 matrix cores.  This is the product every BLAS3
 * phase of Zolo-PD uses: the trailing updates and Q formation of the QR-type
 * step (eq. (12)), X^T X and the factors of the Cholesky-type step
 * (Algorithm 1 step 4(d)), and H = Qp^T A (Algorithm 1 step 5).
 * strides are in elements between consecutive matrices of the batch. */
int zolo_dgemm(zolo_handle h, int transa, int transb, int m, int n, int k, double alpha,
               const double* A, int lda, long long strideA, const double* B, int ldb, long long strideB,
               double beta, double* C, int ldc, long long strideC, int batch);

/* Upper Cholesky Z_b = R_b^T R_b, in place, for b < batch (the factorisation
 * of Z_{2j-1} = X^T X + c_{2j-1} I in Algorithm 1 step 4(d), with R the factor
 * the paper calls L).  The strict lower triangle is set to zero.
 * info[b] (host) receives 0 or the 1-based column of the first non-positive
 * pivot; the return value is ZOLO_BREAKDOWN if any info[b] != 0. */
int zolo_dpotrf_batched(zolo_handle h, int n, double* Z, int ldz, long long strideZ, int batch, int* info);

/* Rinv_b = R_b^{-1} for upper-triangular R_b (strict lower part of Rinv
 * zero), for b < batch.  Used to form X (X^T X + c I)^{-1} in eq. (11). */
int zolo_dtrtri_batched(zolo_handle h, int n, const double* R, int ldr, long long strideR,
                        double* Rinv, int ldi, long long strideI, int batch);

/* Structured Householder QR of the stacked [p_b I; Y_b] (n + m rows, n
 * columns), b < batch <= 16, m >= 1, n >= 1 (Section 3.1: each reflector has
 * m + 1 nonzeros, each block of 64 reflectors m + 64 live rows).  The
 * identity block is placed on top; the pair is the paper's
 * [X; sqrt(c_{2j-1}) I] of eq. (12) with rows reordered, which leaves
 * Q_{j1} Q_{j2}^T unchanged.
 * pivots (host, batch entries) are the p_b >= 0.  On entry Y_b (m x n) holds
 * the dense block; D_b (n x n) is overwritten.  On exit, form_q == 0: D_b
 * holds R_b (upper triangular, zero below) and Y_b the Y-part of the
 * Householder vectors; form_q != 0: D_b holds Q_D (n x n, upper triangular)
 * and Y_b holds Q_Y (m x n) with [Q_D; Q_Y] R = [p_b I; Y_b].
 * With p_b = 0 this is a Householder QR of Y_b alone (R in D_b). */
int zolo_structured_qr_batched(zolo_handle h, int m, int n, const double* pivots, double* Y, int ldy,
                               long long strideY, double* D, int ldd, long long strideD, int batch, int form_q);

#ifdef __cplusplus
}
#endif

#endif /* ZOLO_BLOCKS_H */
