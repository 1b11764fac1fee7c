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
// The next four exist for T = double and T = float.
template <class T>
hipError_t shift_copy(int n, const T* G, long long ldg, T* Z, long long ldz, long long sz, const ShiftArgs& sh,
                      hipStream_t st);
template <class T>
hipError_t fill_matrix(int m, int n, T* Z, long long ldz, long long sz, int batch, double diag, double off,
                       hipStream_t st);
template <class T>
hipError_t zero_strict_lower(int n, T* Z, long long ldz, long long sz, int batch, hipStream_t st);
// mode 0: S = (C + C^T)/2;  mode 1: S = mirror of the upper triangle of C, plus add_diag * I.
template <class T>
hipError_t symmetrize(int n, const T* C, long long ldc, T* S, long long lds, int mode, double add_diag,
                      hipStream_t st);
// Y = s * X, FP64 -> FP32 or FP32 -> FP64 (m x n).
template <class S, class D>
hipError_t convert(int m, int n, const S* X, long long ldx, D* Y, long long ldy, double s, hipStream_t st);
// out[0] = ||X - Y||_F^2 (0 if Y null), out[1] = ||X||_F^2.  part: >= 2048 doubles.
hipError_t frob2(int m, int n, const double* X, long long ldx, const double* Y, long long ldy, double* part,
                 double* out, hipStream_t st);
// out[0] = ||G - I||_F^2 from the upper triangle of symmetric G.  part: >= 2048 doubles.
hipError_t orth2(int n, const double* G, long long ldg, double* part, double* out, hipStream_t st);
// v <- A^T A v / ||A^T A v||, *lam = v^T A^T A v (u: m, w: n scratch).
hipError_t power_step(int m, int n, const double* A, long long lda, double* v, double* u, double* w, double* lam,
                      hipStream_t st);
hipError_t fill_vector(int n, double* v, double val, hipStream_t st);
// p[0..count) = 0 by a kernel (not a memset node, so that it may be captured).
hipError_t zero_ints(int* p, int count, hipStream_t st);
// *out = max_j sum_{i<=j} |R[i][j]|  (colsum: n doubles scratch).
hipError_t norm1_upper(int n, const double* R, long long ldr, double* colsum, double* out, hipStream_t st);

// --- chol.hip -------------------------------------------------------------
// Both exist for T = double and T = float.
// Batched upper Cholesky Z_b = R_b^T R_b in place (strict lower part zeroed).
// info_dev[b] (int, device) receives 0 or the 1-based column of the first
// non-positive pivot.  work: >= batch * 64 * 64 elements.
template <class T>
hipError_t potrf_batched(int n, T* Z, long long ldz, long long sz, int batch, int* info_dev, T* work,
                         hipStream_t st);
// Batched inverse of upper-triangular R_b into Rinv_b (strict lower part zero).
// work: work_elems elements (n^2 batch / 2 + 64^2 batch suffices).
template <class T>
hipError_t trtri_batched(int n, const T* R, long long ldr, long long sr, T* Rinv, long long ldi, long long si,
                         int batch, T* work, long long work_elems, hipStream_t st);

// --- qr.hip ---------------------------------------------------------------
constexpr int kPanelNB = 64;
constexpr int kQrBlock = 2 * kPanelNB;  // two panels: one compact-WY factor Tb
constexpr int kQrSuper = 2 * kQrBlock;  // two blocks share one trailing update (factor Ts)
constexpr size_t kQrSplitElems = (size_t)4 << 20;  // smallest split-K workspace of the QR updates (32 MiB)

struct QrWork {
    double* W = nullptr;          // qr_w_elems(n, batch) doubles
    double* W2 = nullptr;         // qr_w_elems(n, batch) doubles
    double* T = nullptr;          // batch * npanels * kPanelNB^2 doubles
    double* Tb = nullptr;         // qr_tb_elems(n, batch) doubles (T of each 128-column block)
    double* Ts = nullptr;         // qr_ts_elems(n, batch) doubles (T of each 256-column superblock)
    double* splitk = nullptr;     // qr_split_elems(n, batch) doubles: split-K partial products
    size_t splitk_elems = 0;
    hipStream_t panel_stream = nullptr;        // non-null: launch panels there (see run_panel)
    hipEvent_t ev_ready = nullptr, ev_done = nullptr;
    // Look-ahead (see structured_geqrf): a second stream for the far part of
    // each trailing update, with buffers of its own (batch 1 sizes).
    hipStream_t side_stream = nullptr;
    hipEvent_t ev_side_ready = nullptr, ev_side_done = nullptr;
    double* W_side = nullptr;     // qr_w_elems(n, 1) doubles
    double* W2_side = nullptr;    // qr_w_elems(n, 1) doubles
    double* splitk_side = nullptr;  // 4 qr_w_elems(n, 1) doubles
    size_t splitk_side_elems = 0;
    bool single_panels = false;   // one workgroup per matrix for panels of few rows (see run_panel)
    double* Rd = nullptr;         // batch * npanels * kPanelNB^2 doubles (R diagonal blocks)
    double* S = nullptr;          // qr_s_elems(batch) doubles
    double* partials = nullptr;   // qr_partials_elems: per-workgroup exchange slots (kPanelSlot doubles, two parities)
    unsigned* flags = nullptr;    // qr_flag_elems: per-workgroup panel sequence flags
    size_t flag_elems = 0;
    int* error_flag = nullptr;    // 1 int
    int max_coresident = 0;       // workgroups of the panel kernel that fit at once
};

inline size_t qr_w_elems(int n, int batch) { return (size_t)batch * kQrSuper * n; }
inline size_t qr_s_elems(int batch) { return (size_t)batch * 2 * kQrBlock * kQrBlock; }
inline size_t qr_ts_elems(int n, int batch) {
    return (size_t)batch * ((n + kQrSuper - 1) / kQrSuper) * kQrSuper * kQrSuper;
}
// Split-K partials: four pieces of the largest block-reflector product.
inline size_t qr_split_elems(int n, int batch) {
    const size_t e = 4 * qr_w_elems(n, batch);
    return e > kQrSplitElems ? e : kQrSplitElems;
}
inline size_t qr_tb_elems(int n, int batch) {
    return (size_t)batch * ((n + kQrBlock - 1) / kQrBlock) * kQrBlock * kQrBlock;
}

// Doubles each QrWork array needs for m x n, `batch` matrices, e extra rows.
// Panel exchange slot of one workgroup: the largest exchange is the one at
// the end of a 16-column leaf, 16 x (kPanelNB - 16) sums.
constexpr int kPanelSlot = 16 * (kPanelNB - 16);
inline int qr_panel_groups(int m, int e, int batch, int max_coresident) {
    int G = (m + e + 63) / 64;  // the most workgroups any row target can ask for
    int cap = max_coresident / (batch > 0 ? batch : 1);
    if (cap < 1) cap = 1;
    if (G > cap) G = cap;
    if (G < 1) G = 1;
    return G;
}
inline size_t qr_partials_elems(int m, int e, int batch, int max_coresident) {
    return (size_t)batch * 2 * (qr_panel_groups(m, e, batch, max_coresident) + 1) * kPanelSlot;
}
inline size_t qr_flag_elems(int m, int e, int batch, int max_coresident) {
    return (size_t)batch * (qr_panel_groups(m, e, batch, max_coresident) + 1);
}

// M_b[0:m] = X (ld ldx; X null: leave the dense block), M_b[m:m+n] = pivots[b] * I, b < batch <= 16.
hipError_t stack_init(int m, int n, const double* X, long long ldx, double* M, long long ld, long long sm,
                      const double* pivots, int batch, hipStream_t st);
// Householder QR of M_b ((m + e) x n, e = n for the stacked [Y; p I] of
// eq. (12) (Section 3.1: each block of 64 reflectors acts on the m + 64
// contiguous rows [p0, m + p0 + 64)), or e = 0 for a plain QR of an m x n
// matrix).  Panels of 64 columns are factored in pairs; each pair updates the
// rest of the matrix once, as one block reflector of 128 columns.  On exit M_b holds the Householder vectors (explicit unit lower
// trapezoidal), w.T the block-reflector factors and w.Rd the diagonal blocks of
// R; the rest of R is in the upper part of M_b (see assemble_r).
hipError_t structured_geqrf(int m, int e, int n, double* M, long long ld, long long sm, int batch,
                            const QrWork& w, hipStream_t st);
// Overwrites the output of structured_geqrf with the explicit thin Q
// ((m + e) x n); for e = n the bottom n x n block of Q is upper triangular.
hipError_t structured_orgqr(int m, int e, int n, double* M, long long ld, long long sm, int batch,
                            const QrWork& w, hipStream_t st);
// R_b (n x n, zeros below) from the output of structured_geqrf.
hipError_t assemble_r(int n, const double* M, long long ld, long long sm, int batch, const QrWork& w, double* R,
                      long long ldr, long long sr, hipStream_t st);

}  // namespace zolo
