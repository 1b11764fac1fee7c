// C ABI of the learned l/r estimator (zolo_learn.h): argument checks,
// workspace from the handle's arena, and the training loop that queues
// forward, loss, backward and Adam for many steps without host round trips.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/zolo_learn.h"
#include "coeffs.hpp"
#include "handle.hpp"
#include "learn.hpp"

using namespace zolo;

namespace {

int grow_arena(zolo_handle h, size_t bytes) {
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

int finish(zolo_handle h, hipError_t e) {
    if (e != hipSuccess) return ZOLO_HIP;
    return hipStreamSynchronize(h->stream) == hipSuccess ? 0 : ZOLO_HIP;
}

// Work buffer layout of a batch: X (39 B), H1, H2, dH2, dH1 (64 B each).
MlpBufs bufs_of(float* work, int batch, float* y) {
    MlpBufs a;
    a.X = work;
    a.H1 = a.X + (size_t)kNF * batch;
    a.H2 = a.H1 + (size_t)kNH * batch;
    a.Y = y;
    return a;
}
float* dh2_of(float* work, int batch) { return work + (size_t)(kNF + 2 * kNH) * batch; }
float* dh1_of(float* work, int batch) { return work + (size_t)(kNF + 3 * kNH) * batch; }

}  // namespace

extern "C" {

long long zolo_mlp_work_elems(int batch) { return (long long)(kNF + 4 * kNH) * (batch > 0 ? batch : 0) + 64; }

int zolo_sketch_features(zolo_handle h, int m, int n, const double* X0, int ldx, unsigned long long seed,
                         double* feat) {
    if (!h) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!X0) return -4;
    if (ldx < m) return -5;
    if (!feat) return -7;
    const size_t elems = sketch_scratch_elems(m, n) + 64;
    if (int rc = grow_arena(h, sizeof(double) * elems + 512)) return rc;
    double* scratch = reinterpret_cast<double*>(h->arena);
    double* f = scratch + sketch_scratch_elems(m, n);
    hipError_t e = sketch_features(m, n, X0, ldx, seed, f, scratch, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(feat, f, sizeof(double) * kNF, hipMemcpyDeviceToHost, h->stream);
    return finish(h, e);
}

int zolo_surrogate_features(zolo_handle h, int count, const int* m, const int* n, const double* sigma,
                            int ldsigma, unsigned long long seed, unsigned long long first_index, double* feat) {
    if (!h) return -1;
    if (count < 0) return -2;
    if (count == 0) return 0;
    if (!m) return -3;
    if (!n) return -4;
    if (!sigma) return -5;
    for (int b = 0; b < count; ++b) {
        if (n[b] < 1 || n[b] > ldsigma) return -4;
        if (m[b] < n[b]) return -3;
    }
    if (!feat) return -9;
    if (int rc = grow_arena(h, sizeof(int) * 2 * (size_t)count + 512)) return rc;
    int* mv = reinterpret_cast<int*>(h->arena);
    int* nv = mv + count;
    hipError_t e = hipMemcpyAsync(mv, m, sizeof(int) * count, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(nv, n, sizeof(int) * count, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = surrogate_features(count, mv, nv, sigma, ldsigma, seed, first_index, feat, h->stream);
    return finish(h, e);
}

int zolo_mlp_stats(zolo_handle h, int count, const double* feat, float* params) {
    if (!h) return -1;
    if (count < 1) return -2;
    if (!feat) return -3;
    if (!params) return -4;
    return finish(h, mlp_stats(count, feat, params, h->stream));
}

int zolo_mlp_forward(zolo_handle h, int batch, const float* params, const double* feat, float* y, float* work) {
    if (!h) return -1;
    if (batch < 1) return -2;
    if (!params) return -3;
    if (!feat) return -4;
    if (!y) return -5;
    if (!work) return -6;
    return finish(h, mlp_forward(batch, params, feat, nullptr, bufs_of(work, batch, y), h->stream));
}

int zolo_mlp_loss(zolo_handle h, int batch, const float* y, const float* t, float q, float c_r, float* dy,
                  float* loss) {
    if (!h) return -1;
    if (batch < 1) return -2;
    if (!y) return -3;
    if (!t) return -4;
    if (!(q > 0.0f && q < 1.0f)) return -5;
    if (!(c_r >= 0.0f)) return -6;
    if (!dy) return -7;
    if (!loss) return -8;
    if (int rc = grow_arena(h, 512)) return rc;
    float* ld = reinterpret_cast<float*>(h->arena);
    hipError_t e = mlp_loss(batch, y, t, nullptr, q, c_r, dy, ld, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(loss, ld, sizeof(float), hipMemcpyDeviceToHost, h->stream);
    return finish(h, e);
}

int zolo_mlp_backward(zolo_handle h, int batch, const float* params, float* work, const float* dy, float* grad) {
    if (!h) return -1;
    if (batch < 1) return -2;
    if (!params) return -3;
    if (!work) return -4;
    if (!dy) return -5;
    if (!grad) return -6;
    const MlpBufs a = bufs_of(work, batch, nullptr);
    return finish(h, mlp_backward(batch, params, a, dy, grad, dh2_of(work, batch), dh1_of(work, batch), h->stream));
}

int zolo_mlp_adam(zolo_handle h, float* params, const float* grad, float* m, float* v, int t, float lr, float b1,
                  float b2, float eps) {
    if (!h) return -1;
    if (!params) return -2;
    if (!grad) return -3;
    if (!m) return -4;
    if (!v) return -5;
    if (t < 1) return -6;
    return finish(h, mlp_adam(params, grad, m, v, t, lr, b1, b2, eps, h->stream));
}

int zolo_mlp_train(zolo_handle h, int steps, int batch, int count, const double* feat, const float* t,
                   const int* idx, float* params, float* m, float* v, int t0, float lr, float q, float c_r,
                   float* work, float* grad, float* losses) {
    if (!h) return -1;
    if (steps < 0) return -2;
    if (batch < 1) return -3;
    if (count < 1) return -4;
    if (!feat) return -5;
    if (!t) return -6;
    if (!idx) return -7;
    if (!params) return -8;
    if (!m) return -9;
    if (!v) return -10;
    if (t0 < 1) return -11;
    if (!(q > 0.0f && q < 1.0f)) return -13;
    if (!work) return -15;
    if (!grad) return -16;
    if (!losses) return -17;
    hipStream_t st = h->stream;
    float* y = work + zolo_mlp_work_elems(batch);
    float* dy = y + 2 * (size_t)batch;
    const MlpBufs a = bufs_of(work, batch, y);
    for (int s = 0; s < steps; ++s) {
        const int* ib = idx + (size_t)s * batch;
        hipError_t e = mlp_forward(batch, params, feat, ib, a, st);
        if (e == hipSuccess) e = mlp_loss(batch, y, t, ib, q, c_r, dy, losses + s, st);
        if (e == hipSuccess) e = mlp_backward(batch, params, a, dy, grad, dh2_of(work, batch), dh1_of(work, batch), st);
        if (e == hipSuccess) e = mlp_adam(params, grad, m, v, t0 + s, lr, 0.9f, 0.999f, 1e-8f, st);
        if (e != hipSuccess) return ZOLO_HIP;
    }
    return finish(h, hipSuccess);
}

int zolo_set_estimator(zolo_handle h, const float* params, int nparams) {
    if (!h) return -1;
    if (params && nparams != kNParams) return -3;
    if (!params) {
        if (h->est) {
            (void)hipStreamSynchronize(h->stream);
            (void)hipFree(h->est);
            h->est = nullptr;
        }
        return 0;
    }
    if (!h->est && hipMalloc(&h->est, sizeof(float) * kNParams) != hipSuccess) {
        h->est = nullptr;
        return ZOLO_ALLOC;
    }
    if (hipMemcpyAsync(h->est, params, sizeof(float) * kNParams, hipMemcpyHostToDevice, h->stream) != hipSuccess)
        return ZOLO_HIP;
    return finish(h, hipSuccess);
}

int zolo_choose_r(double l) {
    if (!(l > 0.0)) l = kLMin;
    if (l > 1.0) l = 1.0;
    return choose_r(l < kLMin ? kLMin : l);
}

}  // extern "C"
