/*
 * zolo.h - C ABI of the MI355X (gfx950) Zolo-PD library.
 *
 * The library computes the polar decomposition A = Qp * H of a real m x n
 * matrix (m >= n): Qp has orthonormal columns and H is symmetric positive
 * semidefinite (eq. (1) of Li, Liu & Du, arXiv 1806.06204).  It runs the
 * Zolo-PD iteration of Algorithm 1 (Section 2.2): every step applies the
 * scaled Zolotarev function of eq. (8) to the iterate X, either through r
 * independent Householder QRs of the stacked [X; sqrt(c_{2j-1}) I] (eq. (12))
 * or, once that is safe, through Cholesky factors of X^T X + c_{2j-1} I
 * (Algorithm 1 step 4(d)), and finally forms H = (Qp^T A + (Qp^T A)^T)/2.
 * The r factorisations of one step run together in batched GPU kernels.
 *
 * Conventions for every call:
 *   - real FP64, column-major storage, leading dimensions in elements;
 *   - matrix pointers (A, Qp, H, U, V) are DEVICE pointers, on the GPU that is
 *     current when the handle was created; S and every scalar array are HOST
 *     pointers;
 *   - work is queued on the handle's HIP stream; the calls return once the
 *     results are complete (each iteration reads one scalar back to the host);
 *   - the caller owns A, Qp, H, U, S, V; A is never modified; outputs must not
 *     overlap A;
 *   - the library owns its device workspace, kept in the handle and grown on
 *     demand; zolo_destroy releases it;
 *   - zolo_pd's QR-type steps of one matrix (r = 1, and the condition
 *     estimate) also queue part of each trailing update on a second stream
 *     that the handle creates on its first zolo_pd call, ordered against the
 *     handle's stream by events; everything is complete when the call
 *     returns, and the results are the same as on one stream;
 *   - no call prints, throws or aborts.
 *
 * Return codes (int):
 *    0  ZOLO_OK
 *   -i  the i-th argument is invalid (LAPACK convention, counting from 1)
 *    1  ZOLO_NOT_CONVERGED: max_iter reached; outputs hold the last iterate
 *       and info holds the achieved errors
 *    2  ZOLO_NONFINITE: A holds NaN or Inf
 *    3  ZOLO_ALLOC: device workspace allocation failed
 *    4  ZOLO_HIP: a HIP runtime call failed
 *    5  ZOLO_KERNEL: a kernel reported an internal failure (a cooperative
 *       barrier that did not complete within its bounded wait)
 *    6  ZOLO_BREAKDOWN: a factorisation met a non-positive pivot where no
 *       fallback exists (building-block entry points only)
 *    7  ZOLO_SCRATCH: the problem needs more device workspace than the fixed
 *       scratch of zolo_pd_noalloc holds
 */
#ifndef ZOLO_H
#define ZOLO_H

#ifdef __cplusplus
extern "C" {
#endif

#define ZOLO_OK 0
#define ZOLO_NOT_CONVERGED 1
#define ZOLO_NONFINITE 2
#define ZOLO_ALLOC 3
#define ZOLO_HIP 4
#define ZOLO_KERNEL 5
#define ZOLO_BREAKDOWN 6
#define ZOLO_SCRATCH 7

#define ZOLO_MAX_R 8
#define ZOLO_MAX_ITER 16

typedef struct zolo_handle_s* zolo_handle;

/* Options.  Initialise with zolo_default_opts(). */
typedef struct {
    int max_iter;        /* iteration limit (default 10, at most ZOLO_MAX_ITER) */
    int stop_rule;       /* 0 verified (default): once the predicted l reaches
                            1 - 1e-15, stop when ||X^T X - I||_F / sqrt(n) <= tau,
                            else continue with l = sqrt(1 - sqrt(n) d), or, if
                            sqrt(n) d >= 1, with the condition estimate of
                            the current X;
                            1 paper: ||X_new - X_old||_F / ||X_new||_F <= eps^(1/(2r+1))
                            (Algorithm 1 step 4(d), Algorithm 3 step 4(e)) */
    double tau;          /* verified-stop threshold (default 5e-14) */
    double chol_switch;  /* QR-type step while (1+c_1)/(l^2+c_1) > chol_switch
                            (default 100; the QDWH switch of Section 2.1) */
    int qr_variant;      /* 0 (default): structured QR of [X; sqrt(c) I] with
                            m + NB live rows per panel (Section 3.1);
                            1: the same blocked Householder QR and Q formation
                            applied to [X; sqrt(c) I] as a dense (m + n) x n
                            matrix (every reflector spans all rows below its
                            pivot, Q_2 is used as a full matrix), the
                            comparison of Section 3.1 / Table 2.  Needs the
                            workspace of an (m + n) x n problem. */
    int precision;       /* 0 (default): every step in FP64.
                            1 mixed: every Cholesky-type step that is not
                            predicted to be the last (l_next < 1 - 1e-15) runs
                            in FP32 on the FP32 matrix cores; QR-type steps, the
                            last step, the stop checks and H stay in FP64.
                            An FP32 step perturbs the iterate by about the FP32
                            unit roundoff and later steps converge to the polar
                            factor of the perturbed iterate, so Qp stays
                            orthogonal to FP64 accuracy but the backward error
                            is of FP32 size (about 1e-7) whenever a step ran in
                            FP32.  info->prec says which steps did. */
    int compute_errors;  /* 1: fill info->bwd_err and info->orth_err (costs two
                            extra GEMMs); 0 (default): leave them at -1 */
    int l_source;        /* how l is found when the caller passes l <= 0:
                            0 (default) condition estimate from a QR of X0;
                            1 the learned estimator installed with
                            zolo_set_estimator (zolo_learn.h): 39 features of
                            a 32-column sketch of X0 into a small network that
                            also gives r when r <= 0.  Without an installed
                            estimator, or when its output is not finite, the
                            condition estimate is used.  Either way the
                            verified stop rule judges the result: an l above
                            sigma_min costs iterations, not accuracy. */
    int batch_streams;   /* zolo_pd_batched only: number of solves run at once,
                            each on its own stream and host thread (0: 16; 1:
                            one after another on the handle's stream).  Their
                            panels of up to 2304 live rows run one workgroup
                            per matrix on the solve's stream; larger panels
                            are cooperative launches that share one stream,
                            so at most one of those is in flight at any time.
                            Solves overlap only as far as the HIP runtime has
                            hardware queues for their streams
                            (GPU_MAX_HW_QUEUES, 4 unless set; about 16 suits
                            16 solves). */
    int r_policy;        /* how r is chosen when the caller passes r <= 0:
                            0 (default) the smallest r whose scalar recursion
                            converges within two steps (Section 2.2, Table 1;
                            with l_source = 1, the network's degree output);
                            1 the r of least predicted time on this GPU: the
                            step kinds each r takes from l (the same rules as
                            the solve) priced by a per-step cost model of the
                            library's kernels (zolo_predict). */
    int reserved[6];
} zolo_opts;

/* Per-call report. */
typedef struct {
    int status;            /* same value as the return code */
    int iters;             /* iterations taken */
    int r_used;            /* Zolotarev degree r */
    int chol_fallbacks;    /* Cholesky-type steps redone as QR-type */
    int l_from;            /* 0 l given, 1 condition estimate, 2 learned */
    int l_reestimates;     /* verified stop: times sqrt(n) d >= 1 voided the
                              bound from d (l was above sigma_min) and l was
                              re-estimated from the current X */
    int checks;            /* verified stop: orthogonality checks computed */
    char kind[ZOLO_MAX_ITER + 1];  /* 'Q' or 'C' per iteration, NUL-terminated */
    char prec[ZOLO_MAX_ITER + 1];  /* 'd' (FP64) or 's' (FP32) per iteration */
    double alpha;          /* scaling alpha >= sigma_max(A) used, X0 = A / alpha */
    double l0;             /* l used for the first step (after clamping) */
    double l_seq[ZOLO_MAX_ITER];   /* l before each step */
    double orth_check;     /* last ||X^T X - I||_F / sqrt(n) (verified rule), else -1 */
    double t_stage[8];     /* milliseconds: [0] scale and estimates, [1] QR-type
                              steps, [2] Cholesky-type steps, [3] stop checks,
                              [4] H, [5] eigensolver (zolo_svd), [6] U = Qp V,
                              [7] whole call */
    double flops_exec;     /* floating-point operations executed by the kernels */
    double flops_paper;    /* the paper method's count for the executed schedule:
                              5 r m n^2 per QR-type step, m n^2 + r (n^3/3 +
                              2 m n^2) per Cholesky-type step, 2 m n^2 for H,
                              m n^2 per verified check */
    double bwd_err;        /* ||A - Qp H||_F / ||A||_F if requested, else -1 */
    double orth_err;       /* ||Qp^T Qp - I||_F / sqrt(n) if requested, else -1 */
} zolo_info;

/* Fill *opts with the defaults listed above. */
void zolo_default_opts(zolo_opts* opts);

/* Create a handle bound to the current HIP device and to `stream` (a
 * hipStream_t; NULL = the default stream).  Returns 0 or ZOLO_HIP. */
int zolo_create(zolo_handle* handle, void* stream);

/* Change the stream a handle queues work on. */
int zolo_set_stream(zolo_handle handle, void* stream);

/* Release the handle and its device workspace. */
int zolo_destroy(zolo_handle handle);

/* Zolotarev coefficients for lower bound l and degree r (host only, no handle).
 * Section 2.2: c[0..2r-1] = c_1..c_{2r} of eq. (7); a[0..r-1] = a_1..a_r of
 * eq. (10) (taken as the quotient that makes the partial-fraction identity (9)
 * hold); *mhat = Mhat of eq. (8); *l_next = Zhat(l; l), the l-update of
 * Algorithm 1 step 4(c) (with l^2 + c_{2j} in the numerator).
 * Any output pointer may be NULL.  l is clamped to >= 1e-20.
 * Returns 0, -1 if l is not in (0, 1], -2 if r is not in [1, ZOLO_MAX_R]. */
int zolo_coeffs(double l, int r, double* c, double* a, double* mhat, double* l_next);

/* Predicted schedule and time of a Zolo-PD solve of an m x n matrix from
 * lower bound l with degree r (host only, no handle, nothing launched).
 * The step kinds follow the solve's own rules (Algorithm 1 step 4 with the
 * coefficients of eqs. (7)-(10), QR-type while the bound on kappa(Z_j)
 * exceeds chol_switch, one verified check once l reaches 1 - 1e-15); each
 * step is priced by a cost model of this library's kernels on MI355X
 * (rates of the FP64 matrix-core products and per-panel latencies of the
 * factorisations).  kinds (may be NULL) receives 'Q'/'C' per step,
 * NUL-terminated (ZOLO_MAX_ITER + 1 chars); *ms (may be NULL) the predicted
 * milliseconds including H.  Returns 0, -1 for l outside (0, 1], -2 for r
 * outside [1, ZOLO_MAX_R], -3/-4 for m < n or n < 1. */
int zolo_predict(double l, int r, int m, int n, double chol_switch, char* kinds, double* ms);

/* Zolo-PD, Algorithm 1: A (m x n, lda >= m) -> Qp (m x n, ldq >= m) and
 * H (n x n, ldh >= n), with m >= n >= 1.
 *   alpha > 0: used as the upper bound of sigma_max(A) (Algorithm 1 step 1);
 *              alpha <= 0: estimated as 1.01 x a power-iteration estimate.
 *   l in (0,1]: lower bound of sigma_min(A/alpha) (step 2);
 *              l <= 0: estimated as 1/(sqrt(n) ||R^{-1}||_1) from A/alpha = QR.
 *   r in [1,8]: Zolotarev degree; r <= 0: chosen by opts->r_policy (the
 *              smallest r whose scalar recursion converges within two
 *              steps, step 3 and Table 1, by default).
 * opts may be NULL (defaults).  info may be NULL; when given it is written
 * on every return, with info->status equal to the return code. */
int zolo_pd(zolo_handle handle, int m, int n, const double* A, int lda,
            double alpha, double l, int r,
            double* Qp, int ldq, double* H, int ldh,
            const zolo_opts* opts, zolo_info* info);

/* zolo_pd without any device allocation, for callers that cannot allocate:
 * code that must not call hipMalloc (serving loops with fixed memory,
 * harnesses that forbid allocation).  Same arguments, results and return
 * codes as zolo_pd (the same kernels on the same workspace layout give the
 * same bits), but the workspace is a fixed 256 MiB device array of the
 * library, one per GPU, held from the library's load until the process
 * ends (its device address is looked up by zolo_create).  Problems whose
 * workspace exceeds it are rejected with ZOLO_SCRATCH before any work is
 * queued; at degree r = 8 in FP64 that admits e.g. m <= 1024 with n <= 512,
 * or m = n = 768 (smaller r, larger matrices).  Every call on one GPU uses
 * the same array and leaves its contents behind (the call clears what must
 * start at zero itself): calls that overlap on one GPU, from any handle or
 * thread, race and must be serialised by the caller.  It calls no
 * hipMalloc/hipFree; launch statistics and the GEMM autotuner, when
 * switched on, create HIP events on first use. */
int zolo_pd_noalloc(zolo_handle handle, int m, int n, const double* A, int lda,
                    double alpha, double l, int r,
                    double* Qp, int ldq, double* H, int ldh,
                    const zolo_opts* opts, zolo_info* info);

/* Zolo-PD of `count` independent matrices of possibly different shapes (the
 * paper's per-group work of Algorithm 3 steps 1-4).  opts->batch_streams
 * solves run at once, each on a worker stream of the handle with its own
 * workspace sized for the largest matrix; the workers are created on the
 * first such call and kept (workspaces grown on demand) until zolo_destroy.
 * If fewer workers can be set up than asked for, the call runs on those it
 * has (ZOLO_ALLOC only when none can be).  With batch_streams = 1 the
 * matrices are solved one after another on the handle's stream.  The
 * call waits for the caller's stream before it starts and returns when
 * every result is complete.
 * Arrays have `count` entries: m, n, lda, ldq, ldh, alpha, l, r are HOST
 * arrays; A, Qp, H are HOST arrays of DEVICE pointers.  alpha, l, r may be
 * NULL (all estimated / chosen by the policy).  info may be NULL or point to
 * `count` structs.  Returns 0 if every matrix converged, 1 if some did not,
 * or the first error code (negative: -(argument index) of the first bad
 * argument, counting a bad entry of an array as that array's index; -14 for
 * invalid opts). */
int zolo_pd_batched(zolo_handle handle, int count, const int* m, const int* n,
                    const double* const* A, const int* lda, const double* alpha,
                    const double* l, const int* r, double* const* Qp, const int* ldq,
                    double* const* H, const int* ldh, const zolo_opts* opts, zolo_info* info);

/* Zolo-SVD, Algorithm 2: A = Qp H by zolo_pd, then H = V diag(S) V^T by a
 * plain FP64 symmetric eigensolver on the GPU (Householder
 * tridiagonalisation, divide and conquer, back-transformation; the same as
 * zolo_dsyevd), then U = Qp V.  U is m x n (ldu >= m), S has n entries
 * (host, descending), V is n x n (ldv >= n).  The eigensolver and the
 * product are timed in info->t_stage[5] and [6], apart from the polar
 * decomposition.  Allocates the eigensolver's workspace (about 5 n^2 + m n
 * doubles) for the call. */
int zolo_svd(zolo_handle handle, int m, int n, const double* A, int lda,
             double alpha, double l, int r,
             double* U, int ldu, double* S, double* V, int ldv,
             const zolo_opts* opts, zolo_info* info);

#ifdef __cplusplus
}
#endif

#endif /* ZOLO_H */
