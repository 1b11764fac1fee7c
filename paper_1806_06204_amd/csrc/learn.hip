// Kernels of the learned l/r estimator.  The paper takes the lower bound l
// on sigma_min(X0) as known (Algorithm 1 step 2; Section 3.2); the library
// can estimate it from a 32-column Gaussian sketch of X0 with a small FP32
// network trained on spectra the method generates.
//
// Sketch features (G1-G3 of zolo_learn.h): Omega from the SplitMix64
// counter-based generator (Box-Muller), Y = X0 Omega and the Gram matrix
// Y^T Y on the FP64 MFMA GEMM, column and row norms in one pass over X0,
// then one workgroup takes the 32 x 32 eigenvalues by parallel cyclic Jacobi
// (16 disjoint rotations per round, the circle-method pairing) and assembles
// the 39 features.  Training surrogate (G4): one workgroup per spectrum
// builds the Gram matrix of diag(sigma) G with G generated on the fly.
// Network (G5-G7): the three layers are FP32 MFMA GEMMs of this library with
// small fused bias/tanh kernels; backward and Adam follow the same layout.
#include "learn.hpp"
#include "misc.hpp"

namespace zolo {
namespace {

constexpr int kT = 256;

__device__ inline unsigned long long splitmix(unsigned long long seed, unsigned long long k) {
    unsigned long long z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline double unif(unsigned long long seed, unsigned long long k) {
    return ((double)(splitmix(seed, k) >> 11) + 0.5) * 0x1.0p-53;
}

__device__ inline double gauss(unsigned long long seed, unsigned long long k) {
    const double u1 = unif(seed, 2ull * k), u2 = unif(seed, 2ull * k + 1ull);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

__device__ inline double log10c(double x) { return log10(fmax(x, 1e-20)); }

// Sum over the workgroup, returned to every thread (fixed order).
__device__ double block_sum_all(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    return s;
}

struct JacobiLds {
    double A[kNS][kNS + 1];
    double lam[kNS];
    double c[kNS / 2], s[kNS / 2];
    int p[kNS / 2], q[kNS / 2];
    double sh[4];
};

// Eigenvalues of the symmetric 32 x 32 matrix in L.A, descending, into L.lam.
// Each round rotates the 16 disjoint pairs (L_k, L_{31-k}) of the circle
// method, L_0 = 0, L_i = 1 + (r + i - 1) mod 31; 31 rounds meet every pair.
__device__ void jacobi32(JacobiLds& L) {
    const int tid = threadIdx.x;
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < kNS * kNS; e += kT) {
            const int i = e % kNS, j = e / kNS;
            const double v = L.A[i][j];
            tot += v * v;
            if (i != j) off += v * v;
        }
        off = block_sum_all(off, L.sh);
        tot = block_sum_all(tot, L.sh);
        if (off <= 1e-30 * tot) break;
        for (int r = 0; r < kNS - 1; ++r) {
            if (tid < kNS / 2) {
                const int a = tid == 0 ? 0 : 1 + (r + tid - 1) % (kNS - 1);
                const int b = 1 + (r + kNS - 2 - tid) % (kNS - 1);
                const int p = min(a, b), q = max(a, b);
                const double app = L.A[p][p], aqq = L.A[q][q], apq = L.A[p][q];
                double c = 1.0, s = 0.0;
                if (fabs(apq) > 1e-300 && fabs(apq) > 1e-18 * fabs(aqq - app)) {
                    const double th = (aqq - app) / (2.0 * apq);
                    const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                    c = 1.0 / sqrt(t * t + 1.0);
                    s = t * c;
                }
                L.c[tid] = c;
                L.s[tid] = s;
                L.p[tid] = p;
                L.q[tid] = q;
            }
            __syncthreads();
            for (int e = tid; e < (kNS / 2) * kNS; e += kT) {  // columns p, q
                const int k = e / kNS, i = e % kNS, p = L.p[k], q = L.q[k];
                const double c = L.c[k], s = L.s[k], aip = L.A[i][p], aiq = L.A[i][q];
                L.A[i][p] = c * aip - s * aiq;
                L.A[i][q] = s * aip + c * aiq;
            }
            __syncthreads();
            for (int e = tid; e < (kNS / 2) * kNS; e += kT) {  // rows p, q
                const int k = e / kNS, j = e % kNS, p = L.p[k], q = L.q[k];
                const double c = L.c[k], s = L.s[k], apj = L.A[p][j], aqj = L.A[q][j];
                L.A[p][j] = c * apj - s * aqj;
                L.A[q][j] = s * apj + c * aqj;
            }
            __syncthreads();
            if (tid < kNS / 2 && L.s[tid] != 0.0) {
                L.A[L.p[tid]][L.q[tid]] = 0.0;
                L.A[L.q[tid]][L.p[tid]] = 0.0;
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        for (int i = 0; i < kNS; ++i) L.lam[i] = L.A[i][i];
        for (int i = 1; i < kNS; ++i) {
            const double v = L.lam[i];
            int j = i - 1;
            while (j >= 0 && L.lam[j] < v) {
                L.lam[j + 1] = L.lam[j];
                --j;
            }
            L.lam[j + 1] = v;
        }
    }
    __syncthreads();
}

// Mean and population standard deviation of log10(max(sqrt(x_i), 1e-20)),
// i < count, where x_i = get(i); two passes, fixed order.
template <class Get>
__device__ void log_stats(int count, Get get, double* sh, double& mean, double& sd) {
    double s = 0.0;
    for (int i = threadIdx.x; i < count; i += kT) s += log10c(sqrt(get(i)));
    mean = block_sum_all(s, sh) / count;
    double v = 0.0;
    for (int i = threadIdx.x; i < count; i += kT) {
        const double d = log10c(sqrt(get(i))) - mean;
        v += d * d;
    }
    sd = sqrt(block_sum_all(v, sh) / count);
}

// f[0..38] from the sorted eigenvalues of the sketch Gram matrix (thread 0).
__device__ void assemble(double* f, const double* lam, double cmean, double csd, double rmean, double rsd, int m,
                         int n, double frob) {
    const double l1 = log10c(sqrt(fmax(lam[0], 0.0)));
    f[0] = l1;
    for (int i = 1; i < kNS; ++i) f[i] = fmax(log10c(sqrt(fmax(lam[i], 0.0))) - l1, kLogFloor);
    f[32] = cmean;
    f[33] = csd;
    f[34] = rmean;
    f[35] = rsd;
    f[36] = log10((double)n);
    f[37] = log10((double)m / (double)n);
    f[38] = log10c(frob / sqrt((double)n));
}

__global__ void gaussian_fill_kernel(unsigned long long seed, unsigned long long offset, long long count,
                                     double* out) {
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < count;
         k += (long long)gridDim.x * blockDim.x)
        out[k] = gauss(seed, offset + (unsigned long long)k);
}

// out[j] = ||X e_j||^2, one workgroup per column.
__global__ __launch_bounds__(kT) void colnorm2_kernel(int m, const double* __restrict__ X, long long ld,
                                                      double* out) {
    __shared__ double sh[4];
    const double* x = X + blockIdx.x * ld;
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += kT) s += x[i] * x[i];
    s = block_sum_all(s, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// part[i + p m] = sum over column chunk p of X[i][j]^2 (coalesced over rows).
__global__ __launch_bounds__(kT) void rownorm2_partial_kernel(int m, int n, const double* __restrict__ X,
                                                              long long ld, int P, double* part) {
    const int i = blockIdx.x * kT + threadIdx.x, p = blockIdx.y;
    if (i >= m) return;
    const int j0 = (int)((long long)p * n / P), j1 = (int)((long long)(p + 1) * n / P);
    double s = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double v = X[i + j * ld];
        s += v * v;
    }
    part[i + (long long)p * m] = s;
}

__global__ __launch_bounds__(kT) void sketch_features_kernel(int m, int n, const double* __restrict__ G,
                                                             const double* __restrict__ cn2,
                                                             const double* __restrict__ rpart, int P, double* f) {
    __shared__ JacobiLds L;
    const int tid = threadIdx.x;
    for (int e = tid; e < kNS * kNS; e += kT) L.A[e % kNS][e / kNS] = G[e];
    __syncthreads();
    jacobi32(L);
    double cmean, csd, rmean, rsd;
    log_stats(n, [&](int j) { return cn2[j]; }, L.sh, cmean, csd);
    log_stats(m, [&](int i) {
        double s = 0.0;
        for (int p = 0; p < P; ++p) s += rpart[i + (long long)p * m];
        return s;
    }, L.sh, rmean, rsd);
    double fr = 0.0;
    for (int j = tid; j < n; j += kT) fr += cn2[j];
    fr = block_sum_all(fr, L.sh);
    if (tid == 0) assemble(f, L.lam, cmean, csd, rmean, rsd, m, n, sqrt(fr));
}

// One workgroup per spectrum: the Gram matrix of diag(sigma) G with
// G[i][j] = Gaussian number base + i + j n, 32 column-norm samples and 32
// row-norm samples (G4), then the features.
__global__ __launch_bounds__(kT) void surrogate_kernel(const int* __restrict__ mv, const int* __restrict__ nv,
                                                       const double* __restrict__ sigma, long long ldsig,
                                                       unsigned long long seed, unsigned long long first,
                                                       double* feat) {
    __shared__ JacobiLds L;
    __shared__ double gl[64][kNS + 1];
    __shared__ double samp[2 * kNS];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int m = mv[b], n = nv[b];
    const double* sg = sigma + b * ldsig;
    const unsigned long long base = (first + (unsigned long long)b) << 32;
    double acc[kNS * kNS / kT];
#pragma unroll
    for (int u = 0; u < kNS * kNS / kT; ++u) acc[u] = 0.0;
    for (int i0 = 0; i0 < n; i0 += 64) {
        const int rows = min(64, n - i0);
        for (int e = tid; e < 64 * kNS; e += kT) {
            const int ii = e % 64, j = e / 64;
            gl[ii][j] = ii < rows ? sg[i0 + ii] * gauss(seed, base + (unsigned long long)(i0 + ii) +
                                                                  (unsigned long long)j * n)
                                  : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kNS * kNS / kT; ++u) {
            const int e = tid + kT * u, p = e % kNS, q = e / kNS;
            double s = acc[u];
            for (int ii = 0; ii < rows; ++ii) s += gl[ii][p] * gl[ii][q];
            acc[u] = s;
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kNS * kNS / kT; ++u) {
        const int e = tid + kT * u;
        L.A[e % kNS][e / kNS] = acc[u];
    }
    // Norm samples: 8 consecutive lanes per sample.
    const int t = tid >> 3, l = tid & 7;
    double a1 = 0.0, a2 = 0.0;
    for (int i = l; i < n; i += 8) {
        const double g = gauss(seed, base + 32ull * n + (unsigned long long)t * n + i);
        a1 += sg[i] * sg[i] * g * g;
        a2 += g * g;
    }
    for (int off = 1; off < 8; off <<= 1) {
        a1 += __shfl_xor(a1, off, 64);
        a2 += __shfl_xor(a2, off, 64);
    }
    if (l == 0) samp[t] = a1 / a2;
    a1 = a2 = 0.0;
    for (int i = l; i < m; i += 8) {
        const double g = gauss(seed, base + 64ull * n + (unsigned long long)t * m + i);
        if (i < n) a1 += sg[i] * sg[i] * g * g;
        a2 += g * g;
    }
    for (int off = 1; off < 8; off <<= 1) {
        a1 += __shfl_xor(a1, off, 64);
        a2 += __shfl_xor(a2, off, 64);
    }
    if (l == 0) samp[kNS + t] = a1 / a2;
    double fr = 0.0;
    for (int i = tid; i < n; i += kT) fr += sg[i] * sg[i];
    fr = block_sum_all(fr, L.sh);
    __syncthreads();
    jacobi32(L);
    double cmean, csd, rmean, rsd;
    log_stats(kNS, [&](int i) { return samp[i]; }, L.sh, cmean, csd);
    log_stats(kNS, [&](int i) { return samp[kNS + i]; }, L.sh, rmean, rsd);
    if (tid == 0) assemble(feat + (long long)b * kNF, L.lam, cmean, csd, rmean, rsd, m, n, sqrt(fr));
}

// --- network ----------------------------------------------------------------
__global__ void mlp_prep_kernel(int batch, const double* __restrict__ feat, const int* __restrict__ idx,
                                const float* __restrict__ P, float* __restrict__ X) {
    const long long total = (long long)kNF * batch;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e % kNF);
        const long long b = e / kNF;
        const long long c = idx ? idx[b] : b;
        X[e] = (float)((feat[i + c * kNF] - (double)P[kOffMu + i]) / (double)P[kOffSd + i]);
    }
}

// Z <- act(Z + bias) on a rows x batch matrix (act: tanh or identity).
__global__ void bias_act_kernel(int rows, int batch, float* __restrict__ Z, const float* __restrict__ bias,
                                int act) {
    const long long total = (long long)rows * batch;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const float v = Z[e] + bias[e % rows];
        Z[e] = act ? tanhf(v) : v;
    }
}

// dH <- dH * (1 - H^2).
__global__ void dtanh_kernel(long long total, const float* __restrict__ H, float* __restrict__ dH) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x)
        dH[e] *= 1.0f - H[e] * H[e];
}

// out[r] = sum_b D[r + b rows], one workgroup per row.
__global__ __launch_bounds__(kT) void rowsum_kernel(int rows, int batch, const float* __restrict__ D,
                                                    float* __restrict__ out) {
    __shared__ double sh[4];
    double s = 0.0;
    for (int b = threadIdx.x; b < batch; b += kT) s += D[blockIdx.x + (long long)b * rows];
    s = block_sum_all(s, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = (float)s;
}

__global__ __launch_bounds__(kT) void mlp_loss_kernel(int batch, const float* __restrict__ Y,
                                                      const float* __restrict__ T, const int* __restrict__ idx,
                                                      float q, float c_r, float* __restrict__ dY, float* loss) {
    __shared__ double sh[4];
    double acc = 0.0;
    const float inv = 1.0f / (float)batch;
    for (int b = threadIdx.x; b < batch; b += kT) {
        const long long c = idx ? idx[b] : b;
        const float y0 = Y[2 * b], y1 = Y[2 * b + 1], t0 = T[2 * c], t1 = T[2 * c + 1];
        const float e0 = t0 - y0, e1 = t1 - y1;
        const float w = y0 > t0 ? 1.0f - q : q;
        acc += (double)(w * e0 * e0) + (double)(c_r * e1 * e1);
        dY[2 * b] = -2.0f * w * e0 * inv;
        dY[2 * b + 1] = -2.0f * c_r * e1 * inv;
    }
    acc = block_sum_all(acc, sh);
    if (threadIdx.x == 0) *loss = (float)(acc / batch);
}

__global__ void adam_kernel(int n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float bc1, float bc2) {
    for (int e = kNStats + blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const float gi = g[e];
        const float mi = b1 * m[e] + (1.0f - b1) * gi;
        const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
        m[e] = mi;
        v[e] = vi;
        p[e] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

// mean and std of feature i over the samples, one workgroup per feature.
__global__ __launch_bounds__(kT) void mlp_stats_kernel(int count, const double* __restrict__ feat, float* P) {
    __shared__ double sh[4];
    const int i = blockIdx.x;
    double s = 0.0;
    for (int c = threadIdx.x; c < count; c += kT) s += feat[i + (long long)c * kNF];
    const double mean = block_sum_all(s, sh) / count;
    double v = 0.0;
    for (int c = threadIdx.x; c < count; c += kT) {
        const double d = feat[i + (long long)c * kNF] - mean;
        v += d * d;
    }
    const double sd = sqrt(block_sum_all(v, sh) / count);
    if (threadIdx.x == 0) {
        P[kOffMu + i] = (float)mean;
        P[kOffSd + i] = (float)fmax(sd, 1e-6);
    }
}

inline int grid_of(long long total) {
    long long g = (total + kT - 1) / kT;
    if (g > 2048) g = 2048;
    return (int)(g < 1 ? 1 : g);
}

hipError_t sgemm(int m, int n, int k, int ta, int tb, const float* A, int lda, const float* B, int ldb, float* C,
                 int ldc, hipStream_t st) {
    SGemmDesc g;
    g.m = m; g.n = n; g.k = k; g.transa = ta; g.transb = tb;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
    return gemm(g, st);
}

}  // namespace

hipError_t gaussian_fill(unsigned long long seed, unsigned long long offset, long long count, double* out,
                         hipStream_t st) {
    gaussian_fill_kernel<<<grid_of(count), kT, 0, st>>>(seed, offset, count, out);
    return hipGetLastError();
}

hipError_t sketch_features(int m, int n, const double* X0, long long ldx, unsigned long long seed, double* f,
                           double* scratch, hipStream_t st) {
    double* Om = scratch;
    double* Y = Om + (size_t)kNS * n;
    double* G = Y + (size_t)kNS * m;
    double* cn2 = G + kNS * kNS;
    double* rpart = cn2 + n;
    const int P = n < 16 ? n : 16;
    hipError_t e = gaussian_fill(seed, 0, (long long)kNS * n, Om, st);
    if (e != hipSuccess) return e;
    GemmDesc y;  // Y = X0 Omega (m x 32)
    y.m = m; y.n = kNS; y.k = n;
    y.A = X0; y.lda = ldx; y.B = Om; y.ldb = n; y.C = Y; y.ldc = m;
    if ((e = gemm(y, st)) != hipSuccess) return e;
    GemmDesc g;  // G = Y^T Y (32 x 32)
    g.m = kNS; g.n = kNS; g.k = m; g.transa = 1;
    g.A = Y; g.lda = m; g.B = Y; g.ldb = m; g.C = G; g.ldc = kNS;
    if ((e = gemm(g, st)) != hipSuccess) return e;
    colnorm2_kernel<<<n, kT, 0, st>>>(m, X0, ldx, cn2);
    rownorm2_partial_kernel<<<dim3((m + kT - 1) / kT, P), kT, 0, st>>>(m, n, X0, ldx, P, rpart);
    sketch_features_kernel<<<1, kT, 0, st>>>(m, n, G, cn2, rpart, P, f);
    return hipGetLastError();
}

hipError_t surrogate_features(int count, const int* m_dev, const int* n_dev, const double* sigma, long long ldsig,
                              unsigned long long seed, unsigned long long first_index, double* feat,
                              hipStream_t st) {
    if (count <= 0) return hipSuccess;
    surrogate_kernel<<<count, kT, 0, st>>>(m_dev, n_dev, sigma, ldsig, seed, first_index, feat);
    return hipGetLastError();
}

hipError_t mlp_stats(int count, const double* feat, float* params, hipStream_t st) {
    mlp_stats_kernel<<<kNF, kT, 0, st>>>(count, feat, params);
    return hipGetLastError();
}

hipError_t mlp_forward(int batch, const float* P, const double* feat, const int* idx, const MlpBufs& a,
                       hipStream_t st) {
    mlp_prep_kernel<<<grid_of((long long)kNF * batch), kT, 0, st>>>(batch, feat, idx, P, a.X);
    hipError_t e;
    if ((e = sgemm(kNH, batch, kNF, 1, 0, P + kOffW1, kNF, a.X, kNF, a.H1, kNH, st)) != hipSuccess) return e;
    bias_act_kernel<<<grid_of((long long)kNH * batch), kT, 0, st>>>(kNH, batch, a.H1, P + kOffB1, 1);
    if ((e = sgemm(kNH, batch, kNH, 1, 0, P + kOffW2, kNH, a.H1, kNH, a.H2, kNH, st)) != hipSuccess) return e;
    bias_act_kernel<<<grid_of((long long)kNH * batch), kT, 0, st>>>(kNH, batch, a.H2, P + kOffB2, 1);
    if ((e = sgemm(kNO, batch, kNH, 1, 0, P + kOffW3, kNH, a.H2, kNH, a.Y, kNO, st)) != hipSuccess) return e;
    bias_act_kernel<<<grid_of((long long)kNO * batch), kT, 0, st>>>(kNO, batch, a.Y, P + kOffB3, 0);
    return hipGetLastError();
}

hipError_t mlp_loss(int batch, const float* Y, const float* t, const int* idx, float q, float c_r, float* dY,
                    float* loss, hipStream_t st) {
    mlp_loss_kernel<<<1, kT, 0, st>>>(batch, Y, t, idx, q, c_r, dY, loss);
    return hipGetLastError();
}

hipError_t mlp_backward(int batch, const float* P, const MlpBufs& a, const float* dY, float* grad, float* dH2,
                        float* dH1, hipStream_t st) {
    hipError_t e = fill_matrix<float>(kNStats, 1, grad, kNStats, 0, 1, 0.0, 0.0, st);
    if (e != hipSuccess) return e;
    // Layer 3: dW3 (stored 64 x 2) = H2 dY^T, db3, dH2 = W3^T dY.
    if ((e = sgemm(kNH, kNO, batch, 0, 1, a.H2, kNH, dY, kNO, grad + kOffW3, kNH, st)) != hipSuccess) return e;
    rowsum_kernel<<<kNO, kT, 0, st>>>(kNO, batch, dY, grad + kOffB3);
    if ((e = sgemm(kNH, batch, kNO, 0, 0, P + kOffW3, kNH, dY, kNO, dH2, kNH, st)) != hipSuccess) return e;
    dtanh_kernel<<<grid_of((long long)kNH * batch), kT, 0, st>>>((long long)kNH * batch, a.H2, dH2);
    // Layer 2.
    if ((e = sgemm(kNH, kNH, batch, 0, 1, a.H1, kNH, dH2, kNH, grad + kOffW2, kNH, st)) != hipSuccess) return e;
    rowsum_kernel<<<kNH, kT, 0, st>>>(kNH, batch, dH2, grad + kOffB2);
    if ((e = sgemm(kNH, batch, kNH, 0, 0, P + kOffW2, kNH, dH2, kNH, dH1, kNH, st)) != hipSuccess) return e;
    dtanh_kernel<<<grid_of((long long)kNH * batch), kT, 0, st>>>((long long)kNH * batch, a.H1, dH1);
    // Layer 1 (dW1 stored 39 x 64).
    if ((e = sgemm(kNF, kNH, batch, 0, 1, a.X, kNF, dH1, kNH, grad + kOffW1, kNF, st)) != hipSuccess) return e;
    rowsum_kernel<<<kNH, kT, 0, st>>>(kNH, batch, dH1, grad + kOffB1);
    return hipGetLastError();
}

hipError_t mlp_adam(float* params, const float* grad, float* m, float* v, int t, float lr, float b1, float b2,
                    float eps, hipStream_t st) {
    const float bc1 = 1.0f - powf(b1, (float)t), bc2 = 1.0f - powf(b2, (float)t);
    adam_kernel<<<grid_of(kNParams), kT, 0, st>>>(kNParams, params, grad, m, v, lr, b1, b2, eps, bc1, bc2);
    return hipGetLastError();
}

}  // namespace zolo
