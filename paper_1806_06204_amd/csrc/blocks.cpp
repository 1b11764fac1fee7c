// C ABI of the building blocks (zolo_blocks.h): thin wrappers that validate
// arguments, size the handle's workspace and call the batched kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "../../include/zolo_blocks.h"
#include "handle.hpp"
#include "misc.hpp"


namespace {

using namespace zolo;

int grow(zolo_handle h, size_t bytes) {
    if (h->arena_bytes >= bytes) return 0;
    if (h->arena) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(h->arena);
        h->arena = nullptr;
        h->arena_bytes = 0;
    }
    if (hipMalloc(&h->arena, bytes) != hipSuccess) return ZOLO_ALLOC;
    h->arena_bytes = bytes;
    return 0;
}

char* bump(char* base, size_t& off, size_t bytes) {
    off = (off + 255) & ~size_t(255);
    char* p = base + off;
    off += bytes;
    return p;
}

int sync_status(zolo_handle h, hipError_t e) {
    if (e != hipSuccess) return ZOLO_HIP;
    return hipStreamSynchronize(h->stream) == hipSuccess ? 0 : ZOLO_HIP;
}

template <class T>
int gemm_entry(zolo_handle h, int transa, int transb, int m, int n, int k, double alpha, const T* A, int lda,
               long long strideA, const T* B, int ldb, long long strideB, double beta, T* C, int ldc,
               long long strideC, int batch) {
    if (!h) return -1;
    if (m < 0) return -4;
    if (n < 0) return -5;
    if (k < 0) return -6;
    if (!A && m * (long long)k > 0) return -8;
    if (lda < std::max(1, transa ? k : m)) return -9;
    if (!B && k * (long long)n > 0) return -11;
    if (ldb < std::max(1, transb ? n : k)) return -12;
    if (!C && m * (long long)n > 0) return -15;
    if (ldc < std::max(1, m)) return -16;
    if (batch < 0) return -18;
    GemmDescT<T> g;
    g.m = m; g.n = n; g.k = k; g.transa = transa != 0; g.transb = transb != 0;
    g.A = A; g.lda = lda; g.strideA = strideA;
    g.B = B; g.ldb = ldb; g.strideB = strideB;
    g.Cin = C; g.ldcin = ldc; g.strideCin = strideC;
    g.C = C; g.ldc = ldc; g.strideC = strideC;
    g.alpha = alpha; g.beta = beta; g.batch = batch;
    return sync_status(h, gemm(g, h->stream));
}

template <class T>
int potrf_entry(zolo_handle h, int n, T* Z, int ldz, long long strideZ, int batch, int* info) {
    if (!h) return -1;
    if (n < 1) return -2;
    if (!Z) return -3;
    if (ldz < n) return -4;
    if (batch < 1) return -6;
    if (!info) return -7;
    size_t off = 0;
    const size_t need = 256 + 64 * 64 * sizeof(T) * (size_t)batch + 256 + sizeof(int) * batch + 512;
    if (int rc = grow(h, need)) return rc;
    T* work = (T*)bump(h->arena, off, 64 * 64 * sizeof(T) * (size_t)batch);
    int* dinfo = (int*)bump(h->arena, off, sizeof(int) * batch);
    hipError_t e = potrf_batched<T>(n, Z, ldz, strideZ, batch, dinfo, work, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(info, dinfo, sizeof(int) * batch, hipMemcpyDeviceToHost, h->stream);
    if (int rc = sync_status(h, e)) return rc;
    for (int b = 0; b < batch; ++b)
        if (info[b]) return ZOLO_BREAKDOWN;
    return 0;
}

template <class T>
int trtri_entry(zolo_handle h, int n, const T* R, int ldr, long long strideR, T* Rinv, int ldi, long long strideI,
                int batch) {
    if (!h) return -1;
    if (n < 1) return -2;
    if (!R) return -3;
    if (ldr < n) return -4;
    if (!Rinv) return -6;
    if (ldi < n) return -7;
    if (batch < 1) return -9;
    const long long work_elems = (long long)n * n * batch / 2 + 64 * 64 * (long long)batch + 64;
    size_t off = 0;
    if (int rc = grow(h, 512 + sizeof(T) * (size_t)work_elems)) return rc;
    T* work = (T*)bump(h->arena, off, sizeof(T) * (size_t)work_elems);
    return sync_status(h, trtri_batched<T>(n, R, ldr, strideR, Rinv, ldi, strideI, batch, work, work_elems,
                                           h->stream));
}

}  // namespace

extern "C" {

int zolo_dgemm(zolo_handle h, int transa, int transb, int m, int n, int k, double alpha, const double* A, int lda,
               long long strideA, const double* B, int ldb, long long strideB, double beta, double* C, int ldc,
               long long strideC, int batch) {
    return gemm_entry<double>(h, transa, transb, m, n, k, alpha, A, lda, strideA, B, ldb, strideB, beta, C, ldc,
                              strideC, batch);
}

int zolo_sgemm(zolo_handle h, int transa, int transb, int m, int n, int k, float alpha, const float* A, int lda,
               long long strideA, const float* B, int ldb, long long strideB, float beta, float* C, int ldc,
               long long strideC, int batch) {
    return gemm_entry<float>(h, transa, transb, m, n, k, alpha, A, lda, strideA, B, ldb, strideB, beta, C, ldc,
                             strideC, batch);
}

int zolo_dpotrf_batched(zolo_handle h, int n, double* Z, int ldz, long long strideZ, int batch, int* info) {
    return potrf_entry<double>(h, n, Z, ldz, strideZ, batch, info);
}

int zolo_spotrf_batched(zolo_handle h, int n, float* Z, int ldz, long long strideZ, int batch, int* info) {
    return potrf_entry<float>(h, n, Z, ldz, strideZ, batch, info);
}

int zolo_dtrtri_batched(zolo_handle h, int n, const double* R, int ldr, long long strideR, double* Rinv, int ldi,
                        long long strideI, int batch) {
    return trtri_entry<double>(h, n, R, ldr, strideR, Rinv, ldi, strideI, batch);
}

int zolo_strtri_batched(zolo_handle h, int n, const float* R, int ldr, long long strideR, float* Rinv, int ldi,
                        long long strideI, int batch) {
    return trtri_entry<float>(h, n, R, ldr, strideR, Rinv, ldi, strideI, batch);
}

int zolo_structured_qr_batched(zolo_handle h, int m, int n, const double* pivots, double* M, int ldm,
                               long long strideM, double* R, int ldr, long long strideR, int batch, int form_q) {
    if (!h) return -1;
    if (m < 1) return -2;
    if (n < 1 || (!pivots && n > m)) return -3;
    if (!M) return -5;
    const int e = pivots ? n : 0;
    if (ldm < m + e) return -6;
    if (R && ldr < n) return -9;
    if (batch < 1 || batch > kMaxInlineAlpha) return -11;
    if (pivots)
        for (int b = 0; b < batch; ++b)
            if (!(pivots[b] >= 0.0)) return -4;
    const int npanels = (n + kPanelNB - 1) / kPanelNB;
    const size_t blk = (size_t)batch * npanels * kPanelNB * kPanelNB;
    const size_t part = qr_partials_elems(m, e, batch, h->panel_coresident);
    size_t off = 0;
    const size_t need = 14 * 256 + sizeof(double) * (2 * qr_w_elems(n, batch) + qr_tb_elems(n, batch) +
                                                     qr_ts_elems(n, batch) + 2 * blk + qr_split_elems(n, batch) +
                                                     qr_s_elems(batch) + part) +
                        sizeof(unsigned) * qr_flag_elems(m, e, batch, h->panel_coresident) + 64;
    if (int rc = grow(h, need)) return rc;
    QrWork w;
    w.W = (double*)bump(h->arena, off, sizeof(double) * qr_w_elems(n, batch));
    w.W2 = (double*)bump(h->arena, off, sizeof(double) * qr_w_elems(n, batch));
    w.Tb = (double*)bump(h->arena, off, sizeof(double) * qr_tb_elems(n, batch));
    w.Ts = (double*)bump(h->arena, off, sizeof(double) * qr_ts_elems(n, batch));
    w.splitk = (double*)bump(h->arena, off, sizeof(double) * qr_split_elems(n, batch));
    w.splitk_elems = qr_split_elems(n, batch);
    w.T = (double*)bump(h->arena, off, sizeof(double) * blk);
    w.Rd = (double*)bump(h->arena, off, sizeof(double) * blk);
    w.S = (double*)bump(h->arena, off, sizeof(double) * qr_s_elems(batch));
    w.partials = (double*)bump(h->arena, off, sizeof(double) * part);
    w.flag_elems = qr_flag_elems(m, e, batch, h->panel_coresident);
    w.flags = (unsigned*)bump(h->arena, off, sizeof(unsigned) * w.flag_elems);
    w.error_flag = (int*)bump(h->arena, off, 64);
    w.max_coresident = h->panel_coresident;
    hipStream_t st = h->stream;
    hipError_t err = hipMemsetAsync(w.error_flag, 0, sizeof(int), st);
    if (err == hipSuccess && pivots) err = stack_init(m, n, nullptr, ldm, M, ldm, strideM, pivots, batch, st);
    if (err == hipSuccess) err = structured_geqrf(m, e, n, M, ldm, strideM, batch, w, st);
    if (err == hipSuccess && R) err = assemble_r(n, M, ldm, strideM, batch, w, R, ldr, strideR, st);
    if (err == hipSuccess && form_q) err = structured_orgqr(m, e, n, M, ldm, strideM, batch, w, st);
    if (int rc = sync_status(h, err)) return rc;
    int flag = 0;
    if (hipMemcpy(&flag, w.error_flag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return ZOLO_HIP;
    return flag ? ZOLO_KERNEL : 0;
}

}  // extern "C"
