// Device side of the learned l/r estimator: counter-based Gaussian sketch,
// sketch features, the training surrogate and the FP32 three-layer MLP
// (forward, loss, backward, Adam).  Definitions G1-G7 are those of the C ABI
// header zolo_learn.h.
#pragma once

#include "common.hpp"

namespace zolo {

constexpr int kNF = 39;        // features
constexpr int kNH = 64;        // hidden width
constexpr int kNO = 2;         // outputs
constexpr int kNS = 32;        // sketch columns
constexpr int kNStats = 2 * kNF;
constexpr int kNParams = kNStats + kNH * kNF + kNH + kNH * kNH + kNH + kNO * kNH + kNO;
constexpr double kLogFloor = -6.0;

// Offsets in the flat parameter vector.
constexpr int kOffMu = 0, kOffSd = kNF, kOffW1 = kNStats, kOffB1 = kOffW1 + kNH * kNF, kOffW2 = kOffB1 + kNH,
              kOffB2 = kOffW2 + kNH * kNH, kOffW3 = kOffB2 + kNH, kOffB3 = kOffW3 + kNO * kNH;

// Doubles of device scratch the sketch features of an m x n matrix need.
inline size_t sketch_scratch_elems(int m, int n) {
    return (size_t)kNS * n + (size_t)kNS * m + kNS * kNS + n + 16 * (size_t)m + 64;
}

// f[0..38] (device, double) = features of X0 (m x n, device) with sketch
// stream `seed`; scratch: sketch_scratch_elems(m, n) doubles.
hipError_t sketch_features(int m, int n, const double* X0, long long ldx, unsigned long long seed, double* f,
                           double* scratch, hipStream_t st);

// Surrogate features of `count` spectra: sigma column b (ld ldsig) holds the
// n_dev[b] singular values of matrix b with m_dev[b] rows; feat is 39 x count.
hipError_t surrogate_features(int count, const int* m_dev, const int* n_dev, const double* sigma, long long ldsig,
                              unsigned long long seed, unsigned long long first_index, double* feat,
                              hipStream_t st);

// Fill out[k] = Gaussian number offset + k of the stream, k < count.
hipError_t gaussian_fill(unsigned long long seed, unsigned long long offset, long long count, double* out,
                         hipStream_t st);

// params[0:78] = mean and population std (floored at 1e-6) of count feature
// vectors (39 x count, double).
hipError_t mlp_stats(int count, const double* feat, float* params, hipStream_t st);

// Activations of a batch: X (39 x B), H1, H2 (64 x B), Y (2 x B), float.
struct MlpBufs {
    float *X, *H1, *H2, *Y;
};

// Forward pass on feature columns feat[:, idx[b]] (idx null: b).
hipError_t mlp_forward(int batch, const float* params, const double* feat, const int* idx, const MlpBufs& a,
                       hipStream_t st);
// dY and the batch loss (*loss, device) for targets t[:, idx[b]] (2 x N).
hipError_t mlp_loss(int batch, const float* Y, const float* t, const int* idx, float q, float c_r, float* dY,
                    float* loss, hipStream_t st);
// grad (flat, zeros in the first 78 entries) of the loss with dL/dY = dY;
// dH2, dH1 (64 x B) are scratch.
hipError_t mlp_backward(int batch, const float* params, const MlpBufs& a, const float* dY, float* grad, float* dH2,
                        float* dH1, hipStream_t st);
// One Adam step (t >= 1) on params[78:].
hipError_t mlp_adam(float* params, const float* grad, float* m, float* v, int t, float lr, float b1, float b2,
                    float eps, hipStream_t st);

}  // namespace zolo
