// Zolo-SVD (Algorithm 2 of the paper): A = Qp H by Zolo-PD, H = V diag(S) V^T
// by a plain FP64 symmetric eigensolver, U = Qp V.
//
// The eigensolver is the cyclic two-sided Jacobi method with the round-robin
// (circle) ordering: a sweep has n-1 rounds (n rounded up to even), each
// round rotates n/2 disjoint index pairs at once, so every rotation of a
// round is independent: one kernel computes the rotation angles, one applies
// them to the columns of H and V, one to the rows of H.  Sweeps repeat until
// the off-diagonal Frobenius mass is below 1e-15 ||H||_F.  It is simple and
// robust, not fast (each round streams H and V once); it is timed apart from
// the polar decomposition.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <vector>

#include "../../include/zolo.h"
#include "handle.hpp"
#include "misc.hpp"

namespace zolo {
namespace {

struct Rot {
    int p, q;
    double c, s;
};

// Pair t of round k for N (even) players: player 0 meets 1 + k mod (N-1);
// the others meet at mirrored positions around the circle.
__device__ inline void round_pair(int N, int k, int t, int& p, int& q) {
    const int M = N - 1;
    if (t == 0) {
        p = 0;
        q = 1 + k % M;
    } else {
        p = 1 + (k + t) % M;
        q = 1 + ((k - t) % M + M) % M;
    }
    if (p > q) {
        const int x = p;
        p = q;
        q = x;
    }
}

__global__ void jacobi_angles(int n, int N, int k, const double* __restrict__ A, long long lda, Rot* rots) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N / 2) return;
    int p, q;
    round_pair(N, k, t, p, q);
    Rot r{p, q, 1.0, 0.0};
    if (q < n) {
        const double app = A[p + (long long)p * lda], aqq = A[q + (long long)q * lda];
        const double apq = A[p + (long long)q * lda];
        if (fabs(apq) > 1e-300 && fabs(apq) > 1e-18 * fabs(aqq - app)) {
            const double th = (aqq - app) / (2.0 * apq);
            const double tt = th == 0.0 ? 1.0 : copysign(1.0, th) / (fabs(th) + sqrt(th * th + 1.0));
            r.c = 1.0 / sqrt(tt * tt + 1.0);
            r.s = tt * r.c;
        }
    } else {
        r.q = -1;  // the dummy player of an odd n
    }
    rots[t] = r;
}

// Columns p, q of A (and V) <- [c a_p - s a_q, s a_p + c a_q].
__global__ void jacobi_cols(int n, int npairs, double* __restrict__ A, long long lda, double* __restrict__ V,
                            long long ldv, const Rot* rots) {
    const int t = blockIdx.y;
    const Rot r = rots[t];
    if (r.q < 0 || r.s == 0.0) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double* ap = A + (long long)r.p * lda;
        double* aq = A + (long long)r.q * lda;
        double x = ap[i], y = aq[i];
        ap[i] = r.c * x - r.s * y;
        aq[i] = r.s * x + r.c * y;
        double* vp = V + (long long)r.p * ldv;
        double* vq = V + (long long)r.q * ldv;
        x = vp[i];
        y = vq[i];
        vp[i] = r.c * x - r.s * y;
        vq[i] = r.s * x + r.c * y;
    }
}

// Rows p, q of A <- [c a_p - s a_q, s a_p + c a_q]; the rotated pair entry is 0.
__global__ void jacobi_rows(int n, double* __restrict__ A, long long lda, const Rot* rots) {
    const int t = blockIdx.y;
    const Rot r = rots[t];
    if (r.q < 0 || r.s == 0.0) return;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        double* c = A + (long long)j * lda;
        const double x = c[r.p], y = c[r.q];
        c[r.p] = (j == r.q) ? 0.0 : r.c * x - r.s * y;
        c[r.q] = (j == r.p) ? 0.0 : r.s * x + r.c * y;
    }
}

__global__ void offdiag_partial(int n, const double* __restrict__ A, long long lda, double* part) {
    __shared__ double sh[4];
    double s = 0.0, t = 0.0;
    const long long total = (long long)n * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long j = e / n, i = e - j * n;
        const double v = A[i + j * lda];
        t += v * v;
        if (i != j) s += v * v;
    }
    s = wave_sum(s);
    t = wave_sum(t);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[2 * blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    if (lane == 0) sh[w] = t;
    __syncthreads();
    if (threadIdx.x == 0) part[2 * blockIdx.x + 1] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void offdiag_finish(int nparts, const double* part, double* out) {
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int p = 0; p < nparts; ++p) {
            a += part[2 * p];
            b += part[2 * p + 1];
        }
        out[0] = a;
        out[1] = b;
    }
}

__global__ void get_diag(int n, const double* A, long long lda, double* d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = A[i + (long long)i * lda];
}

// Vs[:, k] = V[:, perm[k]].
__global__ void gather_cols(int n, const double* V, long long ldv, const int* perm, double* Vs, long long ldo) {
    const int k = blockIdx.y;
    const int src = perm[k];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        Vs[i + (long long)k * ldo] = V[i + (long long)src * ldv];
}

}  // namespace
}  // namespace zolo

using namespace zolo;

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
    // Qp goes to U's storage, H to a buffer of our own (V, Rot and scratch follow).
    const size_t nn = (size_t)n * n;
    const int N = n + (n & 1);
    const size_t bytes = sizeof(double) * (2 * nn + 4 * (size_t)n + 2048) + sizeof(Rot) * (N / 2 + 1) +
                         sizeof(int) * (size_t)n + 4096;
    char* buf = nullptr;
    if (hipMalloc(&buf, bytes) != hipSuccess) return ZOLO_ALLOC;
    double* Hm = reinterpret_cast<double*>(buf);
    double* Vw = Hm + nn;
    double* diag = Vw + nn;
    double* part = diag + n;
    double* scal = part + 2048;
    Rot* rots = reinterpret_cast<Rot*>(scal + 3 * (size_t)n);
    int* perm_d = reinterpret_cast<int*>(rots + N / 2 + 1);
    zolo_info inf;
    int rc = zolo_pd(h, m, n, A, lda, alpha, l, r, U, ldu, Hm, n, opts, &inf);
    if (rc != 0 && rc != ZOLO_NOT_CONVERGED) {
        (void)hipFree(buf);
        if (info) *info = inf;
        return rc;
    }
    const int pd_status = rc;
    auto t0 = std::chrono::steady_clock::now();
    auto fail = [&](int code) {
        (void)hipFree(buf);
        inf.status = code;
        if (info) *info = inf;
        return code;
    };
    if (fill_matrix(n, n, Vw, n, 0, 1, 1.0, 0.0, st) != hipSuccess) return fail(ZOLO_HIP);
    const int nparts = 256;
    const dim3 cgrid((n + 255) / 256 > 64 ? 64 : (n + 255) / 256, N / 2);
    for (int sweep = 0; sweep < 60; ++sweep) {
        offdiag_partial<<<nparts, 256, 0, st>>>(n, Hm, n, part);
        offdiag_finish<<<1, 64, 0, st>>>(nparts, part, scal);
        if (hipMemcpyAsync(h->host, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return fail(ZOLO_HIP);
        if (std::sqrt(h->host[0]) <= 1e-15 * std::sqrt(h->host[1]) || N < 2) break;
        for (int k = 0; k < N - 1; ++k) {
            jacobi_angles<<<(N / 2 + 63) / 64, 64, 0, st>>>(n, N, k, Hm, n, rots);
            jacobi_cols<<<cgrid, 256, 0, st>>>(n, N / 2, Hm, n, Vw, n, rots);
            jacobi_rows<<<cgrid, 256, 0, st>>>(n, Hm, n, rots);
        }
        if (hipGetLastError() != hipSuccess) return fail(ZOLO_HIP);
    }
    get_diag<<<(n + 255) / 256, 256, 0, st>>>(n, Hm, n, diag);
    std::vector<double> w(n);
    if (hipMemcpyAsync(w.data(), diag, sizeof(double) * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(ZOLO_HIP);
    std::vector<int> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return w[a] > w[b]; });
    for (int k = 0; k < n; ++k) S[k] = w[perm[k]];
    if (hipMemcpyAsync(perm_d, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, st) != hipSuccess)
        return fail(ZOLO_HIP);
    gather_cols<<<dim3((n + 255) / 256 > 64 ? 64 : (n + 255) / 256, n), 256, 0, st>>>(n, Vw, n, perm_d, V, ldv);
    if (hipStreamSynchronize(st) != hipSuccess) return fail(ZOLO_HIP);
    auto t1 = std::chrono::steady_clock::now();
    inf.t_stage[5] = std::chrono::duration<double, std::milli>(t1 - t0).count();
    // U = Qp V, with Qp held in U: copy Qp out first.
    double* Qtmp = nullptr;
    if (hipMalloc(&Qtmp, sizeof(double) * (size_t)m * n) != hipSuccess) return fail(ZOLO_ALLOC);
    (void)hipMemcpy2DAsync(Qtmp, sizeof(double) * m, U, sizeof(double) * ldu, sizeof(double) * m, n,
                     hipMemcpyDeviceToDevice, st);
    GemmDesc g;
    g.m = m; g.n = n; g.k = n;
    g.A = Qtmp; g.lda = m; g.B = V; g.ldb = ldv;
    g.C = U; g.ldc = ldu;
    hipError_t e = gemm(g, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(Qtmp);
    if (e != hipSuccess) return fail(ZOLO_HIP);
    auto t2 = std::chrono::steady_clock::now();
    inf.t_stage[6] = std::chrono::duration<double, std::milli>(t2 - t1).count();
    inf.t_stage[7] += inf.t_stage[5] + inf.t_stage[6];
    inf.flops_exec += 2.0 * m * (double)n * n;
    return fail(pd_status);
}
