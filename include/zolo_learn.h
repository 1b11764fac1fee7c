/*
 * zolo_learn.h - the learned estimate of l and r for Zolo-PD.
 *
 * Algorithm 1 (steps 2-3) of Li, Liu & Du (arXiv 1806.06204) needs a lower
 * bound l on sigma_min(X0), X0 = A / alpha, and a degree r; the paper takes
 * them as known (Section 3.2 reports their cost, Table 3).  zolo_pd can get l
 * from a condition estimate (a QR of X0) or, with zolo_opts.l_source = 1,
 * from a small network that reads 39 features of a 32-column Gaussian sketch
 * of X0.  This header exposes that path: the features, the training data,
 * and the network's forward pass, loss, backward pass and optimiser, all on
 * the GPU, so that the network is trained by these kernels.
 *
 * Definitions (every function below computes exactly these):
 * G1 Random numbers: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014).  Output k
 *    of stream s is mix(s + (k + 1) * 0x9E3779B97F4A7C15) with
 *    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9, z = (z ^ (z >> 27)) *
 *    0x94D049BB133111EB, z ^ (z >> 31) (mod 2^64); uniform number k =
 *    ((x_k >> 11) + 0.5) * 2^-53; Gaussian number k = sqrt(-2 ln u_{2k})
 *    cos(2 pi u_{2k+1}).
 * G2 Sketch: Omega (n x 32), Omega[i][j] = Gaussian number i + j n; Y = X0
 *    Omega; s_1 >= ... >= s_32 = square roots of the eigenvalues of Y^T Y.
 * G3 Features f[0..38] (norms clamped at 1e-20 before each log10):
 *    f0 = log10 s_1; f_i = max(log10(s_{i+1} / s_1), -6) for i = 1..31
 *    (below 1e-6 the Gram matrix's rounding dominates); f32, f33 = mean and
 *    population std of log10 of the column norms of X0; f34, f35 = the same
 *    for the row norms; f36 = log10 n; f37 = log10(m / n);
 *    f38 = log10(||X0||_F / sqrt(n)).
 * G4 Surrogate features of a spectrum sigma (n values, m rows): the law of
 *    the features of U diag(sigma) V^T for Haar U, V.  Matrix b of a call uses
 *    Gaussian numbers offset by (first_index + b) * 2^32: the sketch
 *    singular values are those of diag(sigma) G, G[i][j] = number i + j n;
 *    column norms are the 32 samples ||sigma * g|| / ||g|| (g = numbers
 *    32n + t n .. 32n + (t+1) n - 1); row norms the 32 samples
 *    ||sigma * g[0:n]|| / ||g|| (g = numbers 64n + t m .. 64n + (t+1) m - 1);
 *    f32..f35 are over these samples; the rest as G3 with ||X0||_F = ||sigma||.
 * G5 Network, FP32: x = (f - mu) / sd, h1 = tanh(W1 x + b1),
 *    h2 = tanh(W2 h1 + b2), y = W3 h2 + b3; y0 estimates
 *    log10(sigma_min / sigma_max), y1 the degree r.  l = 10^y0 clamped to
 *    [1e-20, 1], r = round(y1) clamped to [1, 8].
 * G6 Loss: batch mean of w (t0 - y0)^2 + c_r (t1 - y1)^2, w = 1 - q if
 *    y0 > t0 else q (q < 1/2 penalises an over-estimated l more).
 * G7 Adam (Kingma & Ba 2015) on the trainable parameters (not mu, sd).
 *
 * Parameters: ZOLO_MLP_NPARAMS floats, in the order mu[39], sd[39],
 * W1[64][39], b1[64], W2[64][64], b2[64], W3[2][64], b3[2] (W row-major).
 * Feature sets are column-major 39 x count (double); targets 2 x count
 * (float: t0, t1 per column).  Conventions of zolo.h: device pointers for
 * arrays unless stated, work on the handle's stream, complete on return,
 * -i for an invalid i-th argument, ZOLO_HIP for a HIP failure.
 */
#ifndef ZOLO_LEARN_H
#define ZOLO_LEARN_H

#include "zolo.h"

#ifdef __cplusplus
extern "C" {
#endif

#define ZOLO_NF 39
#define ZOLO_MLP_NSTATS 78
#define ZOLO_MLP_NPARAMS 6928
/* Sketch stream used by zolo_pd when opts.l_source = 1. */
#define ZOLO_SKETCH_SEED 0x5EEDF00DULL

/* G2-G3: feat (HOST, 39 doubles) = features of X0 (m x n, m >= n >= 1,
 * device, ldx >= m) with the sketch of stream `seed`. */
int zolo_sketch_features(zolo_handle h, int m, int n, const double* X0, int ldx, unsigned long long seed,
                         double* feat);

/* G4: feat (39 x count) = surrogate features of `count` spectra.  m, n are
 * HOST arrays (m[b] >= n[b] >= 1); sigma (device) holds spectrum b in column
 * b (ldsigma >= max n). */
int zolo_surrogate_features(zolo_handle h, int count, const int* m, const int* n, const double* sigma,
                            int ldsigma, unsigned long long seed, unsigned long long first_index, double* feat);

/* params[0:78] = mean and population std (floored at 1e-6) of the feature
 * set (39 x count). */
int zolo_mlp_stats(zolo_handle h, int count, const double* feat, float* params);

/* Floats of the work buffer that forward/backward/train use for a batch. */
long long zolo_mlp_work_elems(int batch);

/* G5 on feature columns 0..batch-1: y (2 x batch).  work keeps the
 * activations that zolo_mlp_backward reads. */
int zolo_mlp_forward(zolo_handle h, int batch, const float* params, const double* feat, float* y, float* work);

/* G6: dy (2 x batch) = dLoss/dy; *loss (HOST) = the loss. */
int zolo_mlp_loss(zolo_handle h, int batch, const float* y, const float* t, float q, float c_r, float* dy,
                  float* loss);

/* Gradient (ZOLO_MLP_NPARAMS floats, zeros for mu and sd) of a loss with
 * dLoss/dy = dy, using the activations that the last zolo_mlp_forward of
 * the same batch left in work. */
int zolo_mlp_backward(zolo_handle h, int batch, const float* params, float* work, const float* dy, float* grad);

/* G7: one Adam step number t >= 1 (m, v: optimiser state, zero at t = 1). */
int zolo_mlp_adam(zolo_handle h, float* params, const float* grad, float* m, float* v, int t, float lr, float b1,
                  float b2, float eps);

/* `steps` training steps, queued without host round trips: step s takes the
 * minibatch of feature columns idx[s * batch .. (s+1) * batch - 1] (device
 * ints into the set of `count`), runs forward, loss (q, c_r), backward and
 * Adam step t0 + s (lr, b1 = 0.9, b2 = 0.999, eps = 1e-8) and writes its
 * loss to losses[s] (device).  work: zolo_mlp_work_elems(batch) floats plus
 * 4 * batch (y and dy, 2 x batch each); grad: ZOLO_MLP_NPARAMS floats. */
int zolo_mlp_train(zolo_handle h, int steps, int batch, int count, const double* feat, const float* t,
                   const int* idx, float* params, float* m, float* v, int t0, float lr, float q, float c_r,
                   float* work, float* grad, float* losses);

/* Install trained parameters (HOST, nparams == ZOLO_MLP_NPARAMS) in the
 * handle; zolo_pd with opts.l_source = 1 then estimates l (and r, when
 * r <= 0) with them.  params == NULL removes the estimator. */
int zolo_set_estimator(zolo_handle h, const float* params, int nparams);

/* The degree policy of Algorithm 1 step 3 (host only): the smallest r in
 * [1, 8] whose l-recursion reaches 1 - 1e-15 within two steps, else 8. */
int zolo_choose_r(double l);

#ifdef __cplusplus
}
#endif

#endif /* ZOLO_LEARN_H */
