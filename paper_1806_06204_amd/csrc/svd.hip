// Zolo-SVD (Algorithm 2 of the paper): A = Qp H by Zolo-PD, H = V diag(S) V^T
// by the plain FP64 symmetric eigensolver of eig.hip (Householder
// tridiagonalisation, divide and conquer, back-transformation), U = Qp V.
// The eigensolver and the product U = Qp V are timed apart from the polar
// decomposition (info->t_stage[5], [6]).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>

#include "../../include/zolo.h"
#include "../../include/zolo_blocks.h"
#include "handle.hpp"
#include "misc.hpp"

namespace zolo {
size_t syevd_work_bytes(int n);
hipError_t syevd(int n, double* A, long long lda, double* w_host, double* Z, long long ldz, char* work,
                 double* host, hipStream_t st);
}  // namespace zolo

using namespace zolo;

namespace {

// Device buffer of the handle's own for a call outside zolo_pd's arena.
struct Scratch {
    char* p = nullptr;
    ~Scratch() {
        if (p) (void)hipFree(p);
    }
};

// Pinned host buffer of n doubles (the handle's 4 KiB one when it suffices).
struct HostBuf {
    double* p = nullptr;
    bool own = false;
    ~HostBuf() {
        if (own && p) (void)hipHostFree(p);
    }
};

}  // namespace

extern "C" int zolo_dsyevd(zolo_handle h, int n, const double* A, int lda, double* w, double* Z, int ldz) {
    if (!h) return -1;
    if (n < 1) return -2;
    if (!A) return -3;
    if (lda < n) return -4;
    if (!w) return -5;
    if (!Z) return -6;
    if (ldz < n) return -7;
    hipStream_t st = h->stream;
    const size_t nn = (size_t)n * n;
    Scratch buf;
    if (hipMalloc(&buf.p, sizeof(double) * nn + 256 + syevd_work_bytes(n)) != hipSuccess) return ZOLO_ALLOC;
    double* Ac = reinterpret_cast<double*>(buf.p);
    char* work = buf.p + ((sizeof(double) * nn + 255) / 256) * 256;
    HostBuf hb;
    if ((size_t)n * sizeof(double) <= 4096) {
        hb.p = h->host;
    } else {
        if (hipHostMalloc((void**)&hb.p, sizeof(double) * n) != hipSuccess) return ZOLO_ALLOC;
        hb.own = true;
    }
    if (hipMemcpy2DAsync(Ac, sizeof(double) * n, A, sizeof(double) * lda, sizeof(double) * n, n,
                         hipMemcpyDeviceToDevice, st) != hipSuccess)
        return ZOLO_HIP;
    if (syevd(n, Ac, n, w, Z, ldz, work, hb.p, st) != hipSuccess) return ZOLO_HIP;
    return 0;
}

extern "C" int zolo_svd(zolo_handle h, int m, int n, const double* A, int lda, double alpha, double l, int r,
                        double* U, int ldu, double* S, double* V, int ldv, const zolo_opts* opts, zolo_info* info) {
    if (!h) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!A) return -4;
    if (lda < m) return -5;
    if (!U) return -9;
    if (ldu < m) return -10;
    if (!S) return -11;
    if (!V) return -12;
    if (ldv < n) return -13;
    hipStream_t st = h->stream;
    // Qp goes to U's storage, H to a buffer of our own, followed by the
    // eigensolver's workspace and a copy of Qp for U = Qp V.
    const size_t nn = (size_t)n * n, mn = (size_t)m * n;
    auto round = [](size_t b) { return ((b + 255) / 256) * 256; };
    Scratch buf;
    if (hipMalloc(&buf.p, round(sizeof(double) * nn) + round(sizeof(double) * mn) + syevd_work_bytes(n)) !=
        hipSuccess)
        return ZOLO_ALLOC;
    double* Hm = reinterpret_cast<double*>(buf.p);
    double* Qtmp = reinterpret_cast<double*>(buf.p + round(sizeof(double) * nn));
    char* work = buf.p + round(sizeof(double) * nn) + round(sizeof(double) * mn);
    HostBuf hb;
    if ((size_t)n * sizeof(double) <= 4096) {
        hb.p = h->host;
    } else {
        if (hipHostMalloc((void**)&hb.p, sizeof(double) * n) != hipSuccess) return ZOLO_ALLOC;
        hb.own = true;
    }
    zolo_info inf;
    int rc = zolo_pd(h, m, n, A, lda, alpha, l, r, U, ldu, Hm, n, opts, &inf);
    if (rc != 0 && rc != ZOLO_NOT_CONVERGED) {
        if (info) *info = inf;
        return rc;
    }
    const int pd_status = rc;
    auto fail = [&](int code) {
        inf.status = code;
        if (info) *info = inf;
        return code;
    };
    auto t0 = std::chrono::steady_clock::now();
    if (syevd(n, Hm, n, S, V, ldv, work, hb.p, st) != hipSuccess) return fail(ZOLO_HIP);
    // Tridiagonalisation 4/3 n^3 (full-storage update: 2 n^3), divide and
    // conquer about 8/3 n^3 in its block products, back-transformation 2 n^3.
    inf.flops_exec += (2.0 + 8.0 / 3.0 + 2.0) * (double)n * n * n;
    auto t1 = std::chrono::steady_clock::now();
    inf.t_stage[5] = std::chrono::duration<double, std::milli>(t1 - t0).count();
    // U = Qp V, with Qp held in U: copy Qp out first.
    if (hipMemcpy2DAsync(Qtmp, sizeof(double) * m, U, sizeof(double) * ldu, sizeof(double) * m, n,
                         hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(ZOLO_HIP);
    GemmDesc g;
    g.m = m; g.n = n; g.k = n;
    g.A = Qtmp; g.lda = m; g.B = V; g.ldb = ldv;
    g.C = U; g.ldc = ldu;
    hipError_t e = gemm(g, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(ZOLO_HIP);
    auto t2 = std::chrono::steady_clock::now();
    inf.t_stage[6] = std::chrono::duration<double, std::milli>(t2 - t1).count();
    inf.t_stage[7] += inf.t_stage[5] + inf.t_stage[6];
    inf.flops_exec += 2.0 * m * (double)n * n;
    return fail(pd_status);
}
