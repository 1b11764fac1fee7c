// Zolo-PD driver and C ABI (Algorithm 1 of the paper, Algorithm 3 steps 1-4
// on one GPU).  Every matrix operation is a kernel of this library; the host
// only computes the per-iteration scalars (coefficients, step kind, stop test)
// and reads one or two scalars back per iteration.
//
// Per iteration, with c, a, Mhat for the current l:
//   QR-type step (eq. (12)): Y_j = X, D_j = 0 for j = 1..r; one batched
//     structured QR of [sqrt(c_{2j-1}) I; Y_j] and its explicit Q; then
//     X <- Mhat X + sum_j (Mhat a_j / sqrt(c_{2j-1})) Q_{j,Y} Q_{j,D}^T as one
//     batch-reduced GEMM (Q_{j,D} is upper triangular, so the product is a TRMM).
//   Cholesky-type step (eq. (11), the factors of Algorithm 1 step 4(d)):
//     G = X^T X; Z_j = G + c_{2j-1} I = R_j^T R_j (batched POTRF);
//     F = I + sum_j a_j R_j^{-1} R_j^{-T} (batched TRTRI, then one
//     batch-reduced triangular GEMM); X <- Mhat X F.
//     Since X (X^T X + c I)^{-1} = X R^{-1} R^{-T}, this is the same matrix
//     as Mhat (X + sum_j a_j (X R_j^{-1}) R_j^{-T}); summing the n x n
//     inverses first replaces 2r triangular solves on m x n by one GEMM.
//   The Cholesky-type step is taken once (1 + c_1)/(l^2 + c_1) <= chol_switch,
//   i.e. every Z_j has condition number at most chol_switch; a non-positive
//   pivot redoes the step as QR-type.
// Stop rules: verified (default) or the paper's relative-change test.
// Finally H = (Qp^T A + (Qp^T A)^T) / 2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "../../include/zolo.h"
#include "../../include/zolo_blocks.h"
#include "../../include/zolo_learn.h"
#include "coeffs.hpp"
#include "handle.hpp"
#include "learn.hpp"
#include "misc.hpp"
#include "pd_core.hpp"

namespace zolo {
int panel_max_coresident();
hipError_t scratch_address(int device, char** out);
}

using namespace zolo;


namespace {

constexpr double kEps = 2.220446049250313e-16;
// Solves zolo_pd_batched runs at once by default.  Measured on gfx950 over
// 512 matrices with n in [64, 1024], m in [n, 2n]: with the HIP runtime's
// default of 4 hardware queues, 4 solves take 2.81 s and 8 or 16 take
// 2.23-2.26 s; with GPU_MAX_HW_QUEUES=16, 16 solves take 1.06 s.
constexpr int kBatchStreams = 16;

struct Arena {
    char* base;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base + off);
        off += count * sizeof(T);
        return p;
    }
};

// Buffers of one Cholesky-type step in precision T.
template <class T>
struct CholBufs {
    T *X, *Xn, *G, *F, *Z, *D, *trtri, *potrf;
};

struct Work {
    double *X, *Xn, *Y, *D, *G, *F, *trtri, *potrf, *part, *scal, *vec_v, *vec_u, *vec_w, *lam;
    int* iflags;  // [0] nonfinite, [1] panel error, [2..] potrf info per j
    QrWork qr;
    CholBufs<float> s;  // FP32 copies for the mixed schedule (null unless requested)
    double *sk, *feat;  // sketch scratch and the 39 features (learned l)
    float* mlp;         // network activations for one feature vector
    size_t bytes;
};

// Lay out (or size, if base == nullptr) the workspace for m x n and degree
// rmax; `mixed` adds the FP32 buffers of the mixed precision schedule.
Work layout(char* base, int m, int n, int rmax, int panel_coresident, bool mixed = false) {
    Arena ar{base};
    const size_t mn = (size_t)m * n, nn = (size_t)n * n;
    const int npanels = (n + kPanelNB - 1) / kPanelNB;
    Work w{};
    w.X = ar.take<double>(mn);
    w.Xn = ar.take<double>(mn);
    w.Y = ar.take<double>(((size_t)m + n) * n * rmax);  // stacked [X; sqrt(c) I] per j
    w.D = ar.take<double>(nn * rmax);
    w.G = ar.take<double>(nn);
    w.F = ar.take<double>(nn);
    w.trtri = ar.take<double>(nn * rmax / 2 + (size_t)64 * 64 * rmax + 64);
    w.potrf = ar.take<double>((size_t)64 * 64 * rmax);
    w.part = ar.take<double>(4096);
    w.scal = ar.take<double>(64);
    w.vec_v = ar.take<double>(n);
    w.vec_u = ar.take<double>(m);
    w.vec_w = ar.take<double>(n);
    w.lam = ar.take<double>(128);
    w.iflags = ar.take<int>(64);
    w.qr.W = ar.take<double>(qr_w_elems(n, rmax));
    w.qr.W2 = ar.take<double>(qr_w_elems(n, rmax));
    w.qr.T = ar.take<double>((size_t)rmax * npanels * kPanelNB * kPanelNB);
    w.qr.Tb = ar.take<double>(qr_tb_elems(n, rmax));
    w.qr.Ts = ar.take<double>(qr_ts_elems(n, rmax));
    w.qr.splitk = ar.take<double>(qr_split_elems(n, rmax));
    w.qr.splitk_elems = qr_split_elems(n, rmax);
    w.qr.W_side = ar.take<double>(qr_w_elems(n, 1));
    w.qr.W2_side = ar.take<double>(qr_w_elems(n, 1));
    w.qr.splitk_side = ar.take<double>(4 * qr_w_elems(n, 1));
    w.qr.splitk_side_elems = 4 * qr_w_elems(n, 1);
    w.qr.panel_stream = nullptr;
    w.qr.Rd = ar.take<double>((size_t)rmax * npanels * kPanelNB * kPanelNB);
    w.qr.S = ar.take<double>(qr_s_elems(rmax));
    w.qr.partials = ar.take<double>(std::max(qr_partials_elems(m, n, rmax, panel_coresident),
                                             qr_partials_elems(m, 0, 1, panel_coresident)));
    w.qr.flag_elems = std::max(qr_flag_elems(m, n, rmax, panel_coresident), qr_flag_elems(m, 0, 1, panel_coresident));
    w.qr.flags = ar.take<unsigned>(w.qr.flag_elems);
    w.qr.error_flag = w.iflags + 1;
    w.qr.max_coresident = panel_coresident;
    w.sk = ar.take<double>(sketch_scratch_elems(m, n));
    w.feat = ar.take<double>(64);
    w.mlp = ar.take<float>(kNF + 2 * kNH + 64);
    w.s = CholBufs<float>{};
    if (mixed) {
        w.s.X = ar.take<float>(mn);
        w.s.Xn = ar.take<float>(mn);
        w.s.G = ar.take<float>(nn);
        w.s.F = ar.take<float>(nn);
        w.s.Z = ar.take<float>(nn * rmax);
        w.s.D = ar.take<float>(nn * rmax);
        w.s.trtri = ar.take<float>(nn * rmax / 2 + (size_t)64 * 64 * rmax + 64);
        w.s.potrf = ar.take<float>((size_t)64 * 64 * rmax);
    }
    w.bytes = ar.off + 256;
    return w;
}

int ensure(zolo_handle h, size_t bytes) {
    if (h->arena_bytes >= bytes) return 0;
    if (h->arena) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(h->arena);
        h->arena = nullptr;
        h->arena_bytes = 0;
    }
    if (hipMalloc(&h->arena, bytes) != hipSuccess) {
        h->arena = nullptr;
        return ZOLO_ALLOC;
    }
    h->arena_bytes = bytes;
    return 0;
}

struct Timer {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double lap() {
        auto t = std::chrono::steady_clock::now();
        double ms = std::chrono::duration<double, std::milli>(t - t0).count();
        t0 = t;
        return ms;
    }
};

#define HIPCHECK(x)                                  \
    do {                                             \
        if ((x) != hipSuccess) return ZOLO_HIP;      \
    } while (0)

int readback(zolo_handle h, const void* dev, size_t bytes) {
    HIPCHECK(hipMemcpyAsync(h->host, dev, bytes, hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    return 0;
}

// G = X^T X (upper tiles; symmetric result in the upper triangle).
template <class T>
hipError_t gram(int m, int n, const T* X, long long ldx, T* G, hipStream_t st) {
    GemmDescT<T> g;
    g.m = n; g.n = n; g.k = m; g.transa = 1;
    g.A = X; g.lda = ldx; g.B = X; g.ldb = ldx;
    g.C = G; g.ldc = n;
    g.flags = kCUpperTiles | kCStoreUpper;
    return gemm(g, st);
}

struct StepCtx {
    zolo_handle h;
    const Work* w;
    int m, n;
    double flops_exec = 0.0;
    bool dense_qr = false;   // QR-type steps factor [X; sqrt(c) I] as a plain dense matrix
};

// One Cholesky-type step b.X -> b.Xn in precision T.  Returns 0,
// ZOLO_BREAKDOWN, or an error.  g_valid: b.G already holds X^T X.
template <class T>
int chol_core(StepCtx& cx, const Coeffs& co, const CholBufs<T>& b, bool g_valid) {
    const Work& w = *cx.w;
    const int m = cx.m, n = cx.n, r = co.r;
    hipStream_t st = cx.h->stream;
    const long long nn = (long long)n * n;
    if (!g_valid) {
        HIPCHECK(gram<T>(m, n, b.X, m, b.G, st));
        cx.flops_exec += (double)m * n * n;
    }
    ShiftArgs sh;
    sh.batch = r;
    for (int j = 0; j < r; ++j) sh.shift[j] = co.c[2 * j];
    HIPCHECK(shift_copy<T>(n, b.G, n, b.Z, n, nn, sh, st));
    HIPCHECK(potrf_batched<T>(n, b.Z, n, nn, r, w.iflags + 2, b.potrf, st));
    int rc = readback(cx.h, w.iflags + 2, sizeof(int) * r);
    if (rc) return rc;
    for (int j = 0; j < r; ++j)
        if (reinterpret_cast<int*>(cx.h->host)[j] != 0) return ZOLO_BREAKDOWN;
    HIPCHECK(trtri_batched<T>(n, b.Z, n, nn, b.D, n, nn, r, b.trtri, (long long)nn * r / 2 + 64 * 64 * r, st));
    // F = sum_j a_j R_j^{-1} R_j^{-T} (upper tiles), then mirror and add I.
    GemmDescT<T> f;
    f.m = n; f.n = n; f.k = n; f.transb = 1;
    f.A = b.D; f.lda = n; f.strideA = nn;
    f.B = b.D; f.ldb = n; f.strideB = nn;
    f.C = b.G; f.ldc = n;
    f.batch = r; f.reduce = 1; f.nalpha = r;
    for (int j = 0; j < r; ++j) f.alphas[j] = co.a[j];
    f.flags = kAUpper | kBLower | kCUpperTiles | kCStoreUpper;
    HIPCHECK(gemm(f, st));
    HIPCHECK(symmetrize<T>(n, b.G, n, b.F, n, 1, 1.0, st));
    GemmDescT<T> x;
    x.m = m; x.n = n; x.k = n;
    x.A = b.X; x.lda = m; x.B = b.F; x.ldb = n;
    x.C = b.Xn; x.ldc = m; x.alpha = co.mhat;
    HIPCHECK(gemm(x, st));
    cx.flops_exec += r * (double)n * n * n + 2.0 * m * (double)n * n;
    return 0;
}

// FP64 Cholesky-type step on the main buffers (Z_j live in the QR stack buffer).
int chol_step(StepCtx& cx, const Coeffs& co, bool g_valid) {
    const Work& w = *cx.w;
    return chol_core<double>(cx, co, CholBufs<double>{w.X, w.Xn, w.G, w.F, w.Y, w.D, w.trtri, w.potrf}, g_valid);
}

// The same step in FP32 (mixed schedule): X is rounded to FP32, the step runs
// on the FP32 matrix cores and its result is widened back into Xn.
int chol_step_fp32(StepCtx& cx, const Coeffs& co) {
    const Work& w = *cx.w;
    const int m = cx.m, n = cx.n;
    hipStream_t st = cx.h->stream;
    HIPCHECK((convert<double, float>(m, n, w.X, m, w.s.X, m, 1.0, st)));
    const int rc = chol_core<float>(cx, co, w.s, false);
    if (rc) return rc;
    HIPCHECK((convert<float, double>(m, n, w.s.Xn, m, w.Xn, m, 1.0, st)));
    return 0;
}

// Condition estimate (the reading used when l is not given): X = Q R by a
// Householder QR (no identity block), then l = 1 / (sqrt(n) ||R^{-1}||_1),
// which is <= 1 / ||R^{-1}||_2 = sigma_min(X).  Overwrites Y, D and G.
int condition_estimate(StepCtx& cx, const double* X, double* l_out) {
    const Work& w = *cx.w;
    const int m = cx.m, n = cx.n;
    const long long mn = (long long)m * n, nn = (long long)n * n;
    hipStream_t st = cx.h->stream;
    HIPCHECK(hipMemcpyAsync(w.Y, X, sizeof(double) * mn, hipMemcpyDeviceToDevice, st));
    HIPCHECK(structured_geqrf(m, 0, n, w.Y, m, mn, 1, w.qr, st));
    HIPCHECK(assemble_r(n, w.Y, m, mn, 1, w.qr, w.D, n, nn, st));
    HIPCHECK(trtri_batched(n, w.D, n, nn, w.G, n, nn, 1, w.trtri, nn / 2 + 64 * 64, st));
    HIPCHECK(norm1_upper(n, w.G, n, w.vec_u, w.scal, st));
    // The norm and the panel error flag (a cooperative panel whose bounded
    // wait gave up leaves R stale) in one read-back.
    HIPCHECK(hipMemcpyAsync(w.scal + 1, w.iflags + 1, sizeof(int), hipMemcpyDeviceToDevice, st));
    if (int rc = readback(cx.h, w.scal, 2 * sizeof(double))) return rc;
    if (*reinterpret_cast<const int*>(cx.h->host + 1) != 0) return ZOLO_KERNEL;
    const double nrm = cx.h->host[0];
    *l_out = (std::isfinite(nrm) && nrm > 0.0) ? 1.0 / (std::sqrt((double)n) * nrm) : kLMin;
    cx.flops_exec += 2.0 * m * (double)n * n + (double)n * n * n / 3.0;
    return 0;
}

int qr_step(StepCtx& cx, const Coeffs& co) {
    const Work& w = *cx.w;
    const int m = cx.m, n = cx.n, r = co.r;
    hipStream_t st = cx.h->stream;
    const long long ld = (long long)m + n, sm = ld * n;
    double piv[kMaxInlineAlpha];
    for (int j = 0; j < r; ++j) piv[j] = std::sqrt(co.c[2 * j]);
    HIPCHECK(stack_init(m, n, w.X, m, w.Y, ld, sm, piv, r, st));
    if (cx.dense_qr) {
        // Ablation of Section 3.1 (Table 2): the same blocked Householder
        // QR and Q formation on the (m + n) x n stacked matrix taken as a
        // dense one, every reflector spanning all rows below its pivot and
        // Q_{j2} used as a full matrix.
        HIPCHECK(structured_geqrf(m + n, 0, n, w.Y, ld, sm, r, w.qr, st));
        HIPCHECK(structured_orgqr(m + n, 0, n, w.Y, ld, sm, r, w.qr, st));
    } else {
        HIPCHECK(structured_geqrf(m, n, n, w.Y, ld, sm, r, w.qr, st));
        HIPCHECK(structured_orgqr(m, n, n, w.Y, ld, sm, r, w.qr, st));
    }
    // X_new = Mhat X + sum_j (Mhat a_j / sqrt(c_{2j-1})) Q_{j1} Q_{j2}^T; Q_{j2} is upper triangular.
    GemmDesc g;
    g.m = m; g.n = n; g.k = n; g.transb = 1;
    g.A = w.Y; g.lda = ld; g.strideA = sm;
    g.B = w.Y + m; g.ldb = ld; g.strideB = sm;
    g.Cin = w.X; g.ldcin = m; g.beta = co.mhat;
    g.C = w.Xn; g.ldc = m;
    g.alpha = co.mhat; g.batch = r; g.reduce = 1; g.nalpha = r;
    for (int j = 0; j < r; ++j) g.alphas[j] = co.a[j] / piv[j];
    g.flags = cx.dense_qr ? 0u : kBLower;
    HIPCHECK(gemm(g, st));
    if (cx.dense_qr) {
        const double M = (double)m + n, N = n;
        cx.flops_exec += r * (2.0 * (2.0 * M * N * N - 2.0 * N * N * N / 3.0) + 2.0 * m * N * N);
    } else {
        cx.flops_exec += 5.0 * r * m * (double)n * n;
    }
    return 0;
}

// Worker handles of zolo_pd_batched (kept in the parent handle).
void release_workers(zolo_handle h) {
    for (zolo_handle_s* x : h->workers) {
        if (x->stream) (void)hipStreamSynchronize(x->stream);
        if (x->arena) (void)hipFree(x->arena);
        if (x->host) (void)hipHostFree(x->host);
        if (x->ev_ready) (void)hipEventDestroy(x->ev_ready);
        if (x->ev_done) (void)hipEventDestroy(x->ev_done);
        if (x->stream) (void)hipStreamDestroy(x->stream);
        delete x;
    }
    h->workers.clear();
    if (h->worker_panel_stream) {
        (void)hipStreamSynchronize(h->worker_panel_stream);
        (void)hipStreamDestroy(h->worker_panel_stream);
        h->worker_panel_stream = nullptr;
    }
}

// Makes h->workers hold up to `want` workers with workspaces of `need`
// bytes; keeps the ones it could set up.  Returns how many are usable.
int ensure_workers(zolo_handle h, int want, size_t need) {
    if (!h->worker_panel_stream && hipStreamCreate(&h->worker_panel_stream) != hipSuccess) {
        h->worker_panel_stream = nullptr;
        return 0;
    }
    while ((int)h->workers.size() < want) {
        zolo_handle_s* x = new (std::nothrow) zolo_handle_s();
        if (!x) break;
        x->device = h->device;
        x->panel_coresident = h->panel_coresident;
        x->panel_stream = h->worker_panel_stream;
        x->single_panels = true;
        bool ok = hipStreamCreate(&x->stream) == hipSuccess;
        ok = ok && hipHostMalloc((void**)&x->host, 4096) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&x->ev_ready, hipEventDisableTiming) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&x->ev_done, hipEventDisableTiming) == hipSuccess;
        h->workers.push_back(x);
        if (!ok) {
            h->workers.pop_back();
            if (x->stream) (void)hipStreamDestroy(x->stream);
            if (x->host) (void)hipHostFree(x->host);
            if (x->ev_ready) (void)hipEventDestroy(x->ev_ready);
            if (x->ev_done) (void)hipEventDestroy(x->ev_done);
            delete x;
            break;
        }
    }
    int usable = 0;
    for (int t = 0; t < (int)h->workers.size() && t < want; ++t) {
        if (ensure(h->workers[t], need)) break;
        ++usable;
    }
    return usable;
}

bool opts_ok(const zolo_opts& o) {
    return o.max_iter >= 1 && o.max_iter <= ZOLO_MAX_ITER && (o.stop_rule == 0 || o.stop_rule == 1) &&
           o.tau > 0.0 && o.chol_switch >= 1.0 && (o.qr_variant == 0 || o.qr_variant == 1) &&
           (o.precision == 0 || o.precision == 1) && (o.l_source == 0 || o.l_source == 1) &&
           (o.r_policy == 0 || o.r_policy == 1);
}

}  // namespace

namespace zolo {

// Writes the status into *info (when given) for returns before a solve starts.
int report(zolo_info* info, int status) {
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->status = status;
        info->orth_check = info->bwd_err = info->orth_err = -1.0;
    }
    return status;
}

// Argument checks of zolo_pd (LAPACK-style negative codes); fills *opts.
int check_pd_args(zolo_handle h, int m, int n, const double* A, int lda, double alpha, double l, int r,
                  const double* Qp, int ldq, const double* H, int ldh, const zolo_opts* opts_in, zolo_opts* opts) {
    if (!h) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!A) return -4;
    if (lda < m) return -5;
    if (std::isnan(alpha)) return -6;
    if (std::isnan(l) || l > 1.0) return -7;
    if (r > kMaxR) return -8;
    if (!Qp) return -9;
    if (ldq < m) return -10;
    if (!H) return -11;
    if (ldh < n) return -12;
    zolo_default_opts(opts);
    if (opts_in) *opts = *opts_in;
    if (!opts_ok(*opts)) return -13;
    return 0;
}

// Device workspace one solve of m x n with degree r (<= 0: any) needs.
size_t workspace_bytes(zolo_handle h, int m, int n, int r, const zolo_opts& opts) {
    const int rmax = r >= 1 ? r : kMaxR;
    // The dense QR variant factors (m + n) x n matrices as plain ones.
    const int mq = opts.qr_variant == 1 ? m + n : m;
    return layout(nullptr, mq, n, rmax, h->panel_coresident, opts.precision == 1).bytes;
}

#define HIPFIN(x)                                         \
    do {                                                  \
        if ((x) != hipSuccess) return finish(ZOLO_HIP);   \
    } while (0)

// The whole of zolo_pd on the workspace at `base` (workspace_bytes long).
int pd_core(zolo_handle h, char* base, int m, int n, const double* A, int lda, double alpha, double l, int r,
            double* Qp, int ldq, double* H, int ldh, const zolo_opts& opts, zolo_info* info) {
    zolo_info inf;
    std::memset(&inf, 0, sizeof(inf));
    inf.orth_check = -1.0;
    inf.bwd_err = -1.0;
    inf.orth_err = -1.0;
    Timer whole, stage;
    const int rmax = r >= 1 ? r : kMaxR;
    const bool mixed = opts.precision == 1;
    const bool dense_qr = opts.qr_variant == 1;
    Work w = layout(base, dense_qr ? m + n : m, n, rmax, h->panel_coresident, mixed);
    w.qr.panel_stream = h->panel_stream;
    w.qr.single_panels = h->single_panels;
    w.qr.ev_ready = h->ev_ready;
    w.qr.ev_done = h->ev_done;
    w.qr.side_stream = h->side_stream;
    w.qr.ev_side_ready = h->ev_side_ready;
    w.qr.ev_side_done = h->ev_side_done;
    hipStream_t st = h->stream;
    int* hi = reinterpret_cast<int*>(h->host);
    int rc = 0;
    // Stage times: drain the stream first so queued work is charged to the
    // stage that queued it.
    auto lap = [&]() {
        (void)hipStreamSynchronize(st);
        return stage.lap();
    };
    auto finish = [&](int status) {
        inf.status = status;
        inf.t_stage[7] = whole.lap();
        if (info) *info = inf;
        return status;
    };

    StepCtx cx{h, &w, m, n};
    cx.dense_qr = dense_qr;
    HIPFIN(zero_ints(w.iflags, 64, st));
    // Step 1: alpha (upper bound of sigma_max) and X0 = A / alpha.
    double lam = -1.0;  // Rayleigh quotient of A^T A, a lower bound on sigma_max(A)^2, if computed
    if (!(alpha > 0.0)) {
        HIPFIN(fill_vector(n, w.vec_v, 1.0 / std::sqrt((double)n), st));
        double lam_prev = 0.0;
        bool done = false;
        for (int chunk = 0; chunk < 10 && !done; ++chunk) {
            for (int it = 0; it < 10; ++it)
                HIPFIN(power_step(m, n, A, lda, w.vec_v, w.vec_u, w.vec_w, w.lam + it, st));
            if ((rc = readback(h, w.lam, sizeof(double) * 10))) return finish(rc);
            for (int it = 0; it < 10; ++it) {
                lam = h->host[it];
                if ((chunk > 0 || it > 0) && std::fabs(lam - lam_prev) <= 1e-10 * lam) done = true;
                lam_prev = lam;
            }
        }
        inf.flops_exec += 4.0 * m * (double)n * 100;
        alpha = 1.01 * std::sqrt(std::max(lam, 0.0));
        if (!(alpha > 0.0)) return finish(-6);
    }
    inf.alpha = alpha;
    HIPFIN(scale_copy(m, n, A, lda, w.X, m, 1.0 / alpha, w.iflags, st));
    if ((rc = readback(h, w.iflags, sizeof(int)))) return finish(rc);
    if (hi[0]) return finish(ZOLO_NONFINITE);

    // Step 2: l, a lower bound on sigma_min(X0).
    if (!(l > 0.0) && opts.l_source == 1 && h->est) {
        // Learned estimate.  The network predicts log10(sigma_min/sigma_max)
        // from the features of a matrix whose sigma_max is 1 (its training
        // spectra), while sigma_max(X0) = sigma_max(A)/alpha can be smaller.
        // b, a lower bound on sigma_max(X0) (the Rayleigh quotient of the
        // power iteration that gave alpha, else of four power steps on X0),
        // rescales the features of X0 to those of X0 / b, and
        // l = 10^y0 * b is then a lower bound on sigma_min(X0) whenever
        // 10^y0 is one on sigma_min/sigma_max.
        double b = 1.0;
        if (lam > 0.0) {
            b = std::sqrt(lam) / alpha;
        } else {
            HIPFIN(fill_vector(n, w.vec_v, 1.0 / std::sqrt((double)n), st));
            for (int it = 0; it < 4; ++it)
                HIPFIN(power_step(m, n, w.X, m, w.vec_v, w.vec_u, w.vec_w, w.lam + it, st));
            if ((rc = readback(h, w.lam + 3, sizeof(double)))) return finish(rc);
            b = std::sqrt(std::max(h->host[0], 0.0));
            inf.flops_exec += 4.0 * m * (double)n * 4;
        }
        b = std::min(1.0, b);
        HIPFIN(sketch_features(m, n, w.X, m, ZOLO_SKETCH_SEED, w.feat, w.sk, st));
        if (b > 0.0 && b < 1.0) {
            // log10 of the norms of X0 / b: f0, f32, f34 and f38 (G3) shift by -log10 b.
            if ((rc = readback(h, w.feat, sizeof(double) * kNF))) return finish(rc);
            const double sh = -std::log10(b);
            for (int i : {0, 32, 34, 38}) h->host[i] += sh;
            HIPFIN(hipMemcpyAsync(w.feat, h->host, sizeof(double) * kNF, hipMemcpyHostToDevice, st));
        }
        MlpBufs a{w.mlp, w.mlp + kNF, w.mlp + kNF + kNH, w.mlp + kNF + 2 * kNH};
        HIPFIN(mlp_forward(1, h->est, w.feat, nullptr, a, st));
        HIPFIN(hipMemcpyAsync(h->host, a.Y, 2 * sizeof(float), hipMemcpyDeviceToHost, st));
        HIPFIN(hipStreamSynchronize(st));
        const float* yo = reinterpret_cast<const float*>(h->host);
        if (b > 0.0 && std::isfinite(yo[0]) && std::isfinite(yo[1])) {
            l = b * std::pow(10.0, std::min(0.0, std::max(-20.0, (double)yo[0])));
            if (r < 1 && opts.r_policy == 0) r = std::min(kMaxR, std::max(1, (int)std::lround(yo[1])));
            inf.l_from = 2;
        }
        inf.flops_exec += 2.0 * m * (double)n * kNS + 2.0 * m * (double)kNS * kNS;
    }
    if (!(l > 0.0)) {
        inf.l_from = 1;
        if ((rc = condition_estimate(cx, w.X, &l))) return finish(rc);
    }
    if (l < kLMin) l = kLMin;
    if (l > 1.0) l = 1.0;
    inf.l0 = l;
    // Step 3: r (Table 1 rule, or the least predicted time).
    if (r < 1) r = opts.r_policy == 1 ? choose_r_time(l, m, n, opts.chol_switch) : choose_r(l);
    r = std::min(r, rmax);
    inf.r_used = r;
    inf.t_stage[0] += lap();

    bool g_valid = false;   // G holds X^T X of the current X
    int status = ZOLO_NOT_CONVERGED;
    Coeffs co;
    for (int it = 0; it < opts.max_iter; ++it) {
        compute_coeffs(l, r, &co);
        inf.l_seq[it] = l;
        char kind = co.kappa_z > opts.chol_switch ? 'Q' : 'C';
        // Mixed schedule: a Cholesky-type step that is not predicted to be
        // the last one runs in FP32; the last step, every QR-type step and H
        // stay in FP64.
        char prec = (mixed && kind == 'C' && co.l_next < kConverged) ? 's' : 'd';
        if (kind == 'C') {
            rc = prec == 's' ? chol_step_fp32(cx, co) : chol_step(cx, co, g_valid);
            if (rc == ZOLO_BREAKDOWN) {
                ++inf.chol_fallbacks;
                kind = 'Q';
                prec = 'd';
            } else if (rc) {
                return finish(rc);
            }
            inf.t_stage[2] += lap();
        }
        if (kind == 'Q') {
            if ((rc = qr_step(cx, co))) return finish(rc);
            if ((rc = readback(h, w.iflags + 1, sizeof(int)))) return finish(rc);
            if (hi[0]) return finish(ZOLO_KERNEL);
            inf.t_stage[1] += lap();
        }
        g_valid = false;
        inf.kind[it] = kind;
        inf.prec[it] = prec;
        inf.iters = it + 1;
        inf.flops_paper += kind == 'Q' ? 5.0 * r * m * (double)n * n
                                       : m * (double)n * n + r * ((double)n * n * n / 3.0 + 2.0 * m * (double)n * n);
        const double l_pred = co.l_next;
        if (opts.stop_rule == 1) {
            HIPFIN(frob2(m, n, w.Xn, m, w.X, m, w.part, w.scal, st));
            std::swap(w.X, w.Xn);
            if ((rc = readback(h, w.scal, 2 * sizeof(double)))) return finish(rc);
            const double rel = std::sqrt(h->host[0]) / std::sqrt(h->host[1]);
            l = l_pred;
            inf.t_stage[3] += lap();
            if (rel <= std::pow(kEps, 1.0 / (2 * r + 1))) {
                status = 0;
                break;
            }
        } else {
            std::swap(w.X, w.Xn);
            if (l_pred >= kConverged) {
                HIPFIN(gram(m, n, w.X, m, w.G, st));
                HIPFIN(orth2(n, w.G, n, w.part, w.scal, st));
                if ((rc = readback(h, w.scal, sizeof(double)))) return finish(rc);
                cx.flops_exec += (double)m * n * n;
                inf.flops_paper += (double)m * n * n;
                ++inf.checks;
                g_valid = true;
                const double d = std::sqrt(std::max(h->host[0], 0.0)) / std::sqrt((double)n);
                inf.orth_check = d;
                inf.t_stage[3] += lap();
                if (d <= opts.tau) {
                    status = 0;
                    break;
                }
                const double bnd = std::sqrt((double)n) * d;
                if (bnd < 1.0) {
                    l = std::sqrt(std::max(kLMin * kLMin, 1.0 - bnd));
                } else {
                    // The bound from d is void: l was above sigma_min and
                    // some singular values are still far from 1.  Restart
                    // from the condition estimate of the current X.
                    if ((rc = condition_estimate(cx, w.X, &l))) return finish(rc);
                    l = std::min(1.0, std::max(kLMin, l));
                    g_valid = false;
                    ++inf.l_reestimates;
                    inf.t_stage[0] += lap();
                }
            } else {
                l = l_pred;
            }
        }
    }
    inf.kind[inf.iters] = 0;
    inf.prec[inf.iters] = 0;

    // Step 5: Qp = X, H = (Qp^T A + (Qp^T A)^T) / 2.
    HIPFIN(hipMemcpy2DAsync(Qp, sizeof(double) * ldq, w.X, sizeof(double) * m, sizeof(double) * m, n,
                            hipMemcpyDeviceToDevice, st));
    GemmDesc hg;
    hg.m = n; hg.n = n; hg.k = m; hg.transa = 1;
    hg.A = w.X; hg.lda = m; hg.B = A; hg.ldb = lda;
    hg.C = w.F; hg.ldc = n;
    HIPFIN(gemm(hg, st));
    HIPFIN(symmetrize(n, w.F, n, H, ldh, 0, 0.0, st));
    cx.flops_exec += 2.0 * m * (double)n * n;
    inf.flops_paper += 2.0 * m * (double)n * n;
    HIPFIN(hipStreamSynchronize(st));
    inf.t_stage[4] += lap();

    if (opts.compute_errors) {
        GemmDesc pg;  // Xn = Qp H
        pg.m = m; pg.n = n; pg.k = n;
        pg.A = Qp; pg.lda = ldq; pg.B = H; pg.ldb = ldh;
        pg.C = w.Xn; pg.ldc = m;
        HIPFIN(gemm(pg, st));
        HIPFIN(frob2(m, n, A, lda, w.Xn, m, w.part, w.scal, st));
        HIPFIN(gram(m, n, Qp, ldq, w.G, st));
        HIPFIN(orth2(n, w.G, n, w.part, w.scal + 2, st));
        if ((rc = readback(h, w.scal, 3 * sizeof(double)))) return finish(rc);
        inf.bwd_err = std::sqrt(h->host[0]) / std::sqrt(h->host[1]);
        inf.orth_err = std::sqrt(std::max(h->host[2], 0.0)) / std::sqrt((double)n);
    }
    inf.flops_exec += cx.flops_exec;
    return finish(status);
}

#undef HIPFIN

}  // namespace zolo

extern "C" {

void zolo_default_opts(zolo_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->max_iter = 10;
    o->stop_rule = 0;
    o->tau = 5e-14;
    o->chol_switch = 100.0;
    o->qr_variant = 0;
    o->precision = 0;
    o->compute_errors = 0;
}

int zolo_create(zolo_handle* out, void* stream) {
    if (!out) return -1;
    *out = nullptr;
    zolo_handle h = new (std::nothrow) zolo_handle_s();
    if (!h) return ZOLO_ALLOC;
    h->stream = (hipStream_t)stream;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return ZOLO_HIP;
    }
    if (hipHostMalloc((void**)&h->host, 4096) != hipSuccess) {
        delete h;
        return ZOLO_HIP;
    }
    h->panel_coresident = panel_max_coresident();
    char* scratch = nullptr;  // the device's fixed workspace of zolo_pd_noalloc, looked up once
    if (h->panel_coresident <= 0 || scratch_address(h->device, &scratch) != hipSuccess) {
        (void)hipHostFree(h->host);
        delete h;
        return ZOLO_HIP;
    }
    *out = h;
    return 0;
}

int zolo_set_stream(zolo_handle h, void* stream) {
    if (!h) return -1;
    h->stream = (hipStream_t)stream;
    return 0;
}

int zolo_destroy(zolo_handle h) {
    if (!h) return -1;
    (void)hipStreamSynchronize(h->stream);
    release_workers(h);
    if (h->side_stream) {
        (void)hipStreamSynchronize(h->side_stream);
        (void)hipEventDestroy(h->ev_side_ready);
        (void)hipEventDestroy(h->ev_side_done);
        (void)hipStreamDestroy(h->side_stream);
    }
    if (h->arena) (void)hipFree(h->arena);
    if (h->host) (void)hipHostFree(h->host);
    if (h->est) (void)hipFree(h->est);
    delete h;
    return 0;
}

int zolo_coeffs(double l, int r, double* c, double* a, double* mhat, double* l_next) {
    Coeffs co;
    const int rc = compute_coeffs(l, r, &co);
    if (rc) return rc;
    if (c)
        for (int i = 0; i < 2 * r; ++i) c[i] = co.c[i];
    if (a)
        for (int j = 0; j < r; ++j) a[j] = co.a[j];
    if (mhat) *mhat = co.mhat;
    if (l_next) *l_next = co.l_next;
    return 0;
}

int zolo_predict(double l, int r, int m, int n, double chol_switch, char* kinds, double* ms) {
    if (!(l > 0.0) || l > 1.0) return -1;
    if (r < 1 || r > kMaxR) return -2;
    if (m < n) return -3;
    if (n < 1) return -4;
    if (!(chol_switch >= 1.0)) chol_switch = 100.0;
    char buf[ZOLO_MAX_ITER + 1];
    const double t = predict_ms(std::max(l, kLMin), r, m, n, chol_switch, buf);
    if (kinds) std::memcpy(kinds, buf, sizeof(buf));
    if (ms) *ms = t;
    return 0;
}

// The QR look-ahead's stream and events (non-blocking, default priority);
// without them the look-ahead's two parts run on the caller's stream.
static void ensure_side_stream(zolo_handle h) {
    if (h->side_stream) return;
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    if (hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return;
    }
    if (hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) {
        (void)hipEventDestroy(a);
        (void)hipStreamDestroy(s);
        return;
    }
    h->side_stream = s;
    h->ev_side_ready = a;
    h->ev_side_done = b;
}

int zolo_pd(zolo_handle h, int m, int n, const double* A, int lda, double alpha, double l, int r, double* Qp,
            int ldq, double* H, int ldh, const zolo_opts* opts_in, zolo_info* info) {
    zolo_opts opts;
    int rc = check_pd_args(h, m, n, A, lda, alpha, l, r, Qp, ldq, H, ldh, opts_in, &opts);
    if (rc) return report(info, rc);
    const size_t bytes = workspace_bytes(h, m, n, r, opts);
    if ((rc = ensure(h, bytes))) return report(info, rc);
    ensure_side_stream(h);
    return pd_core(h, h->arena, m, n, A, lda, alpha, l, r, Qp, ldq, H, ldh, opts, info);
}

int zolo_pd_batched(zolo_handle h, int count, const int* m, const int* n, const double* const* A, const int* lda,
                    const double* alpha, const double* l, const int* r, double* const* Qp, const int* ldq,
                    double* const* H, const int* ldh, const zolo_opts* opts, zolo_info* info) {
    if (!h) return -1;
    if (count < 0) return -2;
    if (count == 0) return 0;
    if (!m) return -3;
    if (!n) return -4;
    if (!A) return -5;
    if (!lda) return -6;
    if (!Qp) return -10;
    if (!ldq) return -11;
    if (!H) return -12;
    if (!ldh) return -13;
    zolo_opts o;
    zolo_default_opts(&o);
    if (opts) o = *opts;
    if (!opts_ok(o)) return -14;
    // Validate everything and size the workspace for the largest problem
    // first, so one allocation serves the whole batch.
    size_t need = 0;
    for (int i = 0; i < count; ++i) {
        if (m[i] < 1) return -3;
        if (n[i] < 1 || n[i] > m[i]) return -4;
        if (!A[i]) return -5;
        if (lda[i] < m[i]) return -6;
        if (r && r[i] > kMaxR) return -9;
        if (!Qp[i]) return -10;
        if (ldq[i] < m[i]) return -11;
        if (!H[i]) return -12;
        if (ldh[i] < n[i]) return -13;
        need = std::max(need, workspace_bytes(h, m[i], n[i], r ? r[i] : 0, o));
    }
    const int streams = std::min(count, (opts && opts->batch_streams > 0) ? opts->batch_streams : kBatchStreams);
    if (streams <= 1) {
        if (int rc = ensure(h, need)) return rc;
        int worst = 0;
        h->single_panels = true;
        for (int i = 0; i < count; ++i) {
            const int rc = zolo_pd(h, m[i], n[i], A[i], lda[i], alpha ? alpha[i] : 0.0, l ? l[i] : 0.0,
                                   r ? r[i] : 0, Qp[i], ldq[i], H[i], ldh[i], opts, info ? info + i : nullptr);
            if (rc < 0 || rc > ZOLO_NOT_CONVERGED) {
                h->single_panels = false;
                return rc;
            }
            worst = std::max(worst, rc);
        }
        h->single_panels = false;
        return worst;
    }
    // Several solves at once: the handle's worker handles (each with its own
    // stream, pinned read-back buffer and workspace, kept between calls)
    // pull matrices from a shared counter; their cooperative panels all go
    // to one shared panel stream.  If fewer workers than asked for can be
    // set up (streams or memory run out), the ones that could are used.
    // The inputs may still be in flight on the caller's stream.
    if (hipStreamSynchronize(h->stream) != hipSuccess) return ZOLO_HIP;
    const int usable = ensure_workers(h, streams, need);
    if (usable < 1) return ZOLO_ALLOC;
    for (int t = 0; t < usable; ++t) h->workers[t]->est = h->est;
    std::atomic<int> next(0), worst(0), failed(0);
    auto work = [&](zolo_handle_s* x) {
        if (hipSetDevice(x->device) != hipSuccess) {
            failed.store(ZOLO_HIP);
            return;
        }
        for (;;) {
            if (failed.load()) return;
            const int i = next.fetch_add(1);
            if (i >= count) return;
            const int rc = zolo_pd(x, m[i], n[i], A[i], lda[i], alpha ? alpha[i] : 0.0, l ? l[i] : 0.0,
                                   r ? r[i] : 0, Qp[i], ldq[i], H[i], ldh[i], opts, info ? info + i : nullptr);
            if (rc < 0 || rc > ZOLO_NOT_CONVERGED) {
                int expected = 0;
                failed.compare_exchange_strong(expected, rc);
                return;
            }
            int cur = worst.load();
            while (rc > cur && !worst.compare_exchange_weak(cur, rc)) {
            }
        }
    };
    std::vector<std::thread> threads;
    for (int t = 1; t < usable; ++t) threads.emplace_back(work, h->workers[t]);
    work(h->workers[0]);
    for (std::thread& th : threads) th.join();
    int sync = 0;
    for (int t = 0; t < usable; ++t)
        if (hipStreamSynchronize(h->workers[t]->stream) != hipSuccess) sync = ZOLO_HIP;
    if (hipStreamSynchronize(h->worker_panel_stream) != hipSuccess) sync = ZOLO_HIP;
    if (failed.load()) return failed.load();
    if (sync) return sync;
    return worst.load();
}

}  // extern "C"
