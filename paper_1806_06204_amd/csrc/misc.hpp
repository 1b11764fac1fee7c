// Launchers for the library's helper kernels (misc.hip), Cholesky pieces
// (chol.hip) and the structured QR (qr.hip).
#pragma once

#include "common.hpp"

namespace zolo {

struct ShiftArgs {
    int batch = 0;
    double shift[kMaxInlineAlpha] = {};
};

// --- misc.hip -------------------------------------------------------------
hipError_t scale_copy(int m, int n, const double* A, long long lda, double* X, long long ldx, double s,
                      int* nonfinite_flag, hipStream_t st);
hipError_t broadcast_copy(int m, int n, const double* X, long long ldx, double* Y, long long ldy, long long sy,
                          int batch, hipStream_t st);
hipError_t shift_copy(int n, const double* G, long long ldg, double* Z, long long ldz, long long sz,
                      const ShiftArgs& sh, hipStream_t st);
hipError_t fill_matrix(int m, int n, double* Z, long long ldz, long long sz, int batch, double diag, double off,
                       hipStream_t st);
hipError_t zero_strict_lower(int n, double* Z, long long ldz, long long sz, int batch, hipStream_t st);
// mode 0: S = (C + C^T)/2;  mode 1: S = mirror of the upper triangle of C, plus add_diag * I.
hipError_t symmetrize(int n, const double* C, long long ldc, double* S, long long lds, int mode, double add_diag,
                      hipStream_t st);
// out[0] = ||X - Y||_F^2 (0 if Y null), out[1] = ||X||_F^2.  part: >= 2048 doubles.
hipError_t frob2(int m, int n, const double* X, long long ldx, const double* Y, long long ldy, double* part,
                 double* out, hipStream_t st);
// out[0] = ||G - I||_F^2 from the upper triangle of symmetric G.  part: >= 2048 doubles.
hipError_t orth2(int n, const double* G, long long ldg, double* part, double* out, hipStream_t st);
// v <- A^T A v / ||A^T A v||, *lam = v^T A^T A v (u: m, w: n scratch).
hipError_t power_step(int m, int n, const double* A, long long lda, double* v, double* u, double* w, double* lam,
                      hipStream_t st);
hipError_t fill_vector(int n, double* v, double val, hipStream_t st);
// *out = max_j sum_{i<=j} |R[i][j]|  (colsum: n doubles scratch).
hipError_t norm1_upper(int n, const double* R, long long ldr, double* colsum, double* out, hipStream_t st);

// --- chol.hip -------------------------------------------------------------
// Batched upper Cholesky Z_b = R_b^T R_b in place (strict lower part zeroed).
// info_dev[b] (int, device) receives 0 or the 1-based column of the first
// non-positive pivot.  work: >= batch * 64 * 64 doubles.
hipError_t potrf_batched(int n, double* Z, long long ldz, long long sz, int batch, int* info_dev, double* work,
                         hipStream_t st);
// Batched inverse of upper-triangular R_b into Rinv_b (strict lower part zero).
hipError_t trtri_batched(int n, const double* R, long long ldr, long long sr, double* Rinv, long long ldi,
                         long long si, int batch, double* work, long long work_elems, hipStream_t st);

// --- qr.hip ---------------------------------------------------------------
constexpr int kPanelNB = 64;

struct QrWork {
    double* W = nullptr;          // batch * kPanelNB * n doubles
    double* T = nullptr;          // batch * npanels * kPanelNB * kPanelNB doubles
    double* partials = nullptr;   // batch * 2 * maxG * kPanelNB doubles
    unsigned* counters = nullptr; // batch * npanels
    int* error_flag = nullptr;    // 1 int
    int max_coresident = 0;       // workgroups of the panel kernel that fit at once
};

// Structured Householder QR of the stacked [D_b; Y_b] with D_b = pivot_b * I
// (n x n) on top and Y_b (m x n) below, for b < batch (Section 3.1 / eq. (12)).
// On entry Y_b holds the dense block; D_b must be zero.  On exit Y_b holds
// the lower parts of the Householder vectors (their D-part is the identity),
// D_b holds R (upper triangular) and work.T the block-reflector factors.
// rows_live(p) = m for every panel (live rows m + NB per panel).
hipError_t structured_geqrf(int m, int n, double* Y, long long ldy, long long sy, double* D, long long ldd,
                            long long sd, const double* pivots, int batch, const QrWork& w, hipStream_t st);
// Forms the explicit thin Q = [Q_D; Q_Y] in place of (D_b, Y_b) from the
// output of structured_geqrf (reflectors applied last panel first).  Q_D is
// upper triangular.
hipError_t structured_orgqr(int m, int n, double* Y, long long ldy, long long sy, double* D, long long ldd,
                            long long sd, int batch, const QrWork& w, hipStream_t st);

}  // namespace zolo
