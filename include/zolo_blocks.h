/*
 * zolo_blocks.h - building blocks of the Zolo-PD library, exported for
 * kernel-level checks and benchmarks.  Same conventions as zolo.h: FP64
 * (the zolo_s* variants: FP32, the precision of the FP32 steps of the mixed
 * schedule, zolo_opts.precision = 1), column-major, device pointers for
 * matrices, host pointers for scalar arrays, work queued on the handle's
 * stream and complete on return, LAPACK-style negative return for an invalid
 * argument, 4 for a HIP error.
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

/* The same product in FP32 on the FP32 matrix cores (the X^T X, factor and
 * X F products of an FP32 Cholesky-type step of the mixed schedule). */
int zolo_sgemm(zolo_handle h, int transa, int transb, int m, int n, int k, float alpha,
               const float* A, int lda, long long strideA, const float* B, int ldb, long long strideB,
               float beta, float* C, int ldc, long long strideC, int batch);

/* Upper Cholesky Z_b = R_b^T R_b, in place, for b < batch (the factorisation
 * of Z_{2j-1} = X^T X + c_{2j-1} I in Algorithm 1 step 4(d), with R the factor
 * the paper calls L).  The strict lower triangle is set to zero.
 * info[b] (host) receives 0 or the 1-based column of the first non-positive
 * pivot; the return value is ZOLO_BREAKDOWN if any info[b] != 0. */
int zolo_dpotrf_batched(zolo_handle h, int n, double* Z, int ldz, long long strideZ, int batch, int* info);

/* FP32 variant of zolo_dpotrf_batched (same arguments and results). */
int zolo_spotrf_batched(zolo_handle h, int n, float* Z, int ldz, long long strideZ, int batch, int* info);

/* Rinv_b = R_b^{-1} for upper-triangular R_b (strict lower part of Rinv
 * zero), for b < batch.  Used to form X (X^T X + c I)^{-1} in eq. (11). */
int zolo_dtrtri_batched(zolo_handle h, int n, const double* R, int ldr, long long strideR,
                        double* Rinv, int ldi, long long strideI, int batch);

/* FP32 variant of zolo_dtrtri_batched. */
int zolo_strtri_batched(zolo_handle h, int n, const float* R, int ldr, long long strideR,
                        float* Rinv, int ldi, long long strideI, int batch);

/* Structured Householder QR of the stacked [Y_b; p_b I] ((m + n) x n), or a
 * plain Householder QR of Y_b (m x n, m >= n) when pivots is NULL, for
 * b < batch <= 16 (Section 3.1 / eq. (12): with Y = X and p = sqrt(c_{2j-1})
 * this is the factorisation of a QR-type Zolo-PD step; each block of 64
 * reflectors acts on the m + 64 contiguous rows [p0, m + p0 + 64)).
 * M_b = M + b * strideM has leading dimension ldm >= m + n (stacked) or >= m
 * (plain).  On entry rows 0..m-1 of M_b hold Y_b; the call writes p_b I into
 * rows m..m+n-1.  pivots (host, batch entries) must be >= 0.
 * On exit: if R != NULL, R_b = R + b * strideR (n x n, ldr >= n) receives the
 * upper-triangular factor (zeros below); if form_q != 0, M_b holds the thin
 * Q with [Q_1; Q_2] R = M_b (Q_2, the bottom n x n block, is upper
 * triangular), else M_b holds the Householder vectors. */
int zolo_structured_qr_batched(zolo_handle h, int m, int n, const double* pivots, double* M, int ldm,
                               long long strideM, double* R, int ldr, long long strideR, int batch, int form_q);

/* Eigen-decomposition A = Z diag(w) Z^T of a symmetric n x n matrix (lower
 * triangle read; A is not modified), the eigensolver of Zolo-SVD
 * (Algorithm 2: H = V diag(S) V^T): Householder tridiagonalisation, divide
 * and conquer on the tridiagonal matrix, back-transformation.  w (HOST, n
 * entries) receives the eigenvalues in descending order, Z (device, ldz >= n)
 * the matching orthonormal eigenvectors.  Allocates its workspace (about
 * 4 n^2 doubles) for the call.  Returns 0, a negative argument index, 3 if
 * the workspace cannot be allocated or 4 for a HIP error. */
int zolo_dsyevd(zolo_handle h, int n, const double* A, int lda, double* w, double* Z, int ldz);

#ifdef __cplusplus
}
#endif

#endif /* ZOLO_BLOCKS_H */
