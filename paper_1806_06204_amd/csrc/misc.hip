// Memory-bound helper kernels of the Zolo-PD iteration: scaling, copies with
// structure, deterministic two-pass reductions (Frobenius norms, the
// orthogonality residual of a Gram matrix), symmetrisation of H, and the
// matrix-vector products of the power iteration for alpha.
//
// Reductions write one partial per workgroup and a second single-workgroup
// pass sums them in a fixed order, so results do not depend on scheduling.
#include "misc.hpp"

namespace zolo {
namespace {

constexpr int kThreads = 256;

__device__ inline double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    __syncthreads();
    return s;  // valid in thread 0
}

// X = A * s, reporting non-finite entries of A in *flag.
__global__ void scale_copy_kernel(int m, int n, const double* __restrict__ A, long long lda,
                                  double* __restrict__ X, long long ldx, double s, int* flag) {
    const long long total = (long long)m * n;
    int bad = 0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long j = e / m, i = e - j * m;
        const double v = A[i + j * lda];
        if (!isfinite(v)) bad = 1;
        X[i + j * ldx] = v * s;
    }
    if (bad && flag) atomicOr(flag, 1);
}

// Y_b = X for b < batch (X is m x n with ld ldx; Y_b has ld ldy, stride sy).
__global__ void broadcast_copy_kernel(int m, int n, const double* __restrict__ X, long long ldx,
                                      double* __restrict__ Y, long long ldy, long long sy, int batch) {
    const long long total = (long long)m * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long j = e / m, i = e - j * m;
        const double v = X[i + j * ldx];
        for (int b = 0; b < batch; ++b) Y[b * sy + i + j * ldy] = v;
    }
}

// Z_b = G (upper triangle and diagonal) + shift_b I, strict lower part zero.
template <class T>
__global__ void shift_copy_kernel(int n, const T* __restrict__ G, long long ldg,
                                  T* __restrict__ Z, long long ldz, long long sz,
                                  ShiftArgs sh) {
    const long long total = (long long)n * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long j = e / n, i = e - j * n;
        const T g = i <= j ? G[i + j * ldg] : (T)0;
        for (int b = 0; b < sh.batch; ++b)
            Z[b * sz + i + j * ldz] = (i == j) ? g + (T)sh.shift[b] : g;
    }
}

// Y = s * X with a change of precision (FP64 <-> FP32).
template <class S, class D>
__global__ void convert_kernel(int m, int n, const S* __restrict__ X, long long ldx, D* __restrict__ Y,
                               long long ldy, double s) {
    const long long total = (long long)m * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long j = e / m, i = e - j * m;
        Y[i + j * ldy] = (D)(s * (double)X[i + j * ldx]);
    }
}

// Fill an n x n matrix (batched) with value `diag` on the diagonal and `off` elsewhere,
// or only the strict lower triangle with zero (mode 1).
template <class T>
__global__ void fill_kernel(int m, int n, T* __restrict__ Z, long long ldz, long long sz, int batch,
                            int mode, double diag, double off) {
    const long long total = (long long)m * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long j = e / m, i = e - j * m;
        for (int b = 0; b < batch; ++b) {
            T* p = Z + b * sz + i + j * ldz;
            if (mode == 0) *p = (T)((i == j) ? diag : off);
            else if (i > j) *p = (T)0;
        }
    }
}

// S = (U + U^T)/2 from the upper triangle? mode 0: S = (C + C^T)/2 (full C);
// mode 1: S[i][j] = C[min][max] + add_diag * delta_ij (mirror the upper triangle).
template <class T>
__global__ void symmetrize_kernel(int n, const T* __restrict__ C, long long ldc,
                                  T* __restrict__ S, long long lds, int mode, double add_diag) {
    const long long total = (long long)n * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long j = e / n, i = e - j * n;
        T v;
        if (mode == 0) v = (T)0.5 * (C[i + j * ldc] + C[j + i * ldc]);
        else v = (i <= j ? C[i + j * ldc] : C[j + i * ldc]) + (i == j ? (T)add_diag : (T)0);
        S[i + j * lds] = v;
    }
}

// Partial sums for ||X - Y||_F^2 and ||X||_F^2 (Y may be null).
__global__ void frob_partial_kernel(int m, int n, const double* __restrict__ X, long long ldx,
                                    const double* __restrict__ Y, long long ldy, double* part) {
    __shared__ double sh[kThreads / 64];
    const long long total = (long long)m * n;
    double sd = 0.0, sx = 0.0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long j = e / m, i = e - j * m;
        const double x = X[i + j * ldx];
        sx += x * x;
        if (Y) {
            const double dd = x - Y[i + j * ldy];
            sd += dd * dd;
        }
    }
    const double a = block_sum(sd, sh);
    const double b = block_sum(sx, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// Partial sums of ||G - I||_F^2 from the upper triangle of a symmetric G.
__global__ void orth_partial_kernel(int n, const double* __restrict__ G, long long ldg, double* part) {
    __shared__ double sh[kThreads / 64];
    const long long total = (long long)n * n;
    double s = 0.0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long j = e / n, i = e - j * n;
        if (i <= j) {
            const double v = G[i + j * ldg] - (i == j ? 1.0 : 0.0);
            s += (i == j ? 1.0 : 2.0) * v * v;
        }
    }
    const double a = block_sum(s, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = 0.0;
    }
}

// out[0..1] = sums of the (pairs of) partials, in order.
__global__ void finish_sum_kernel(int nparts, const double* part, double* out) {
    __shared__ double sh[kThreads / 64];
    double a = 0.0, b = 0.0;
    for (int p = threadIdx.x; p < nparts; p += blockDim.x) {
        a += part[2 * p];
        b += part[2 * p + 1];
    }
    const double sa = block_sum(a, sh);
    const double sb = block_sum(b, sh);
    if (threadIdx.x == 0) {
        out[0] = sa;
        out[1] = sb;
    }
}

// y = A x  (A m x n, column-major): one thread per row.
__global__ void gemv_n_kernel(int m, int n, const double* __restrict__ A, long long lda,
                              const double* __restrict__ x, double* __restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += A[i + (long long)j * lda] * x[j];
    y[i] = s;
}

// y = A^T x: one workgroup per column.
__global__ void gemv_t_kernel(int m, int n, const double* __restrict__ A, long long lda,
                              const double* __restrict__ x, double* __restrict__ y) {
    __shared__ double sh[kThreads / 64];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += blockDim.x) s += A[i + (long long)j * lda] * x[i];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) y[j] = t;
}

// One power-iteration step on A^T A, v <- w / ||w||, lam_out[it] = v^T w
// (single workgroup; n-vectors).
__global__ void power_normalize_kernel(int n, const double* __restrict__ v, double* __restrict__ w,
                                       double* __restrict__ vnext, double* lam_out) {
    __shared__ double sh[kThreads / 64];
    __shared__ double s_norm;
    double a = 0.0, b = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        a += v[j] * w[j];
        b += w[j] * w[j];
    }
    const double lam = block_sum(a, sh);
    const double nw2 = block_sum(b, sh);
    if (threadIdx.x == 0) {
        *lam_out = lam;
        s_norm = sqrt(nw2);
    }
    __syncthreads();
    const double inv = s_norm > 0.0 ? 1.0 / s_norm : 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) vnext[j] = w[j] * inv;
}

__global__ void fill_vec_kernel(int n, double* v, double val) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) v[j] = val;
}

// max_j sum_i |R[i][j]| over the upper triangle: one workgroup per column,
// partial column sums written to colsum[j].
__global__ void colsum_abs_upper_kernel(int n, const double* __restrict__ R, long long ldr, double* colsum) {
    __shared__ double sh[kThreads / 64];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i <= j && i < n; i += blockDim.x) s += fabs(R[i + (long long)j * ldr]);
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) colsum[j] = t;
}

__global__ void max_kernel(int n, const double* v, double* out) {
    __shared__ double sh[kThreads];
    double m = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) m = fmax(m, v[j]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

inline int grid_for(long long total) {
    long long g = (total + kThreads - 1) / kThreads;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

hipError_t scale_copy(int m, int n, const double* A, long long lda, double* X, long long ldx, double s,
                      int* flag, hipStream_t st) {
    scale_copy_kernel<<<grid_for((long long)m * n), kThreads, 0, st>>>(m, n, A, lda, X, ldx, s, flag);
    return hipGetLastError();
}

hipError_t broadcast_copy(int m, int n, const double* X, long long ldx, double* Y, long long ldy, long long sy,
                          int batch, hipStream_t st) {
    broadcast_copy_kernel<<<grid_for((long long)m * n), kThreads, 0, st>>>(m, n, X, ldx, Y, ldy, sy, batch);
    return hipGetLastError();
}

template <class T>
hipError_t shift_copy(int n, const T* G, long long ldg, T* Z, long long ldz, long long sz, const ShiftArgs& sh,
                      hipStream_t st) {
    shift_copy_kernel<T><<<grid_for((long long)n * n), kThreads, 0, st>>>(n, G, ldg, Z, ldz, sz, sh);
    return hipGetLastError();
}
template hipError_t shift_copy<double>(int, const double*, long long, double*, long long, long long,
                                       const ShiftArgs&, hipStream_t);
template hipError_t shift_copy<float>(int, const float*, long long, float*, long long, long long, const ShiftArgs&,
                                      hipStream_t);

template <class T>
hipError_t fill_matrix(int m, int n, T* Z, long long ldz, long long sz, int batch, double diag, double off,
                       hipStream_t st) {
    fill_kernel<T><<<grid_for((long long)m * n), kThreads, 0, st>>>(m, n, Z, ldz, sz, batch, 0, diag, off);
    return hipGetLastError();
}
template hipError_t fill_matrix<double>(int, int, double*, long long, long long, int, double, double, hipStream_t);
template hipError_t fill_matrix<float>(int, int, float*, long long, long long, int, double, double, hipStream_t);

template <class T>
hipError_t zero_strict_lower(int n, T* Z, long long ldz, long long sz, int batch, hipStream_t st) {
    fill_kernel<T><<<grid_for((long long)n * n), kThreads, 0, st>>>(n, n, Z, ldz, sz, batch, 1, 0.0, 0.0);
    return hipGetLastError();
}
template hipError_t zero_strict_lower<double>(int, double*, long long, long long, int, hipStream_t);
template hipError_t zero_strict_lower<float>(int, float*, long long, long long, int, hipStream_t);

template <class T>
hipError_t symmetrize(int n, const T* C, long long ldc, T* S, long long lds, int mode, double add_diag,
                      hipStream_t st) {
    symmetrize_kernel<T><<<grid_for((long long)n * n), kThreads, 0, st>>>(n, C, ldc, S, lds, mode, add_diag);
    return hipGetLastError();
}
template hipError_t symmetrize<double>(int, const double*, long long, double*, long long, int, double, hipStream_t);
template hipError_t symmetrize<float>(int, const float*, long long, float*, long long, int, double, hipStream_t);

template <class S, class D>
hipError_t convert(int m, int n, const S* X, long long ldx, D* Y, long long ldy, double s, hipStream_t st) {
    convert_kernel<S, D><<<grid_for((long long)m * n), kThreads, 0, st>>>(m, n, X, ldx, Y, ldy, s);
    return hipGetLastError();
}
template hipError_t convert<double, float>(int, int, const double*, long long, float*, long long, double,
                                           hipStream_t);
template hipError_t convert<float, double>(int, int, const float*, long long, double*, long long, double,
                                           hipStream_t);

hipError_t frob2(int m, int n, const double* X, long long ldx, const double* Y, long long ldy, double* part,
                 double* out, hipStream_t st) {
    const int g = grid_for((long long)m * n) > 1024 ? 1024 : grid_for((long long)m * n);
    frob_partial_kernel<<<g, kThreads, 0, st>>>(m, n, X, ldx, Y, ldy, part);
    finish_sum_kernel<<<1, kThreads, 0, st>>>(g, part, out);
    return hipGetLastError();
}

hipError_t orth2(int n, const double* G, long long ldg, double* part, double* out, hipStream_t st) {
    const int g = grid_for((long long)n * n) > 1024 ? 1024 : grid_for((long long)n * n);
    orth_partial_kernel<<<g, kThreads, 0, st>>>(n, G, ldg, part);
    finish_sum_kernel<<<1, kThreads, 0, st>>>(g, part, out);
    return hipGetLastError();
}

hipError_t power_step(int m, int n, const double* A, long long lda, double* v, double* u, double* w, double* lam,
                      hipStream_t st) {
    gemv_n_kernel<<<(m + kThreads - 1) / kThreads, kThreads, 0, st>>>(m, n, A, lda, v, u);
    gemv_t_kernel<<<n, kThreads, 0, st>>>(m, n, A, lda, u, w);
    power_normalize_kernel<<<1, kThreads, 0, st>>>(n, v, w, v, lam);
    return hipGetLastError();
}

__global__ void zero_ints_kernel(int* p, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0;
}

hipError_t zero_ints(int* p, int count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int grid = (count + kThreads - 1) / kThreads;
    if (grid > 1024) grid = 1024;
    zero_ints_kernel<<<grid, kThreads, 0, st>>>(p, count);
    return hipGetLastError();
}

hipError_t fill_vector(int n, double* v, double val, hipStream_t st) {
    fill_vec_kernel<<<(n + kThreads - 1) / kThreads, kThreads, 0, st>>>(n, v, val);
    return hipGetLastError();
}

hipError_t norm1_upper(int n, const double* R, long long ldr, double* colsum, double* out, hipStream_t st) {
    colsum_abs_upper_kernel<<<n, kThreads, 0, st>>>(n, R, ldr, colsum);
    max_kernel<<<1, kThreads, 0, st>>>(n, colsum, out);
    return hipGetLastError();
}

}  // namespace zolo
