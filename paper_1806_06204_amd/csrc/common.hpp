// Shared definitions for the gfx950 Zolo-PD library (device helpers, launch
// descriptors).  Every kernel of the library is written for CDNA4: 64-lane
// wavefronts, FP64 MFMA 16x16x4 tiles, LDS staging.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace zolo {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// GEMM descriptor:  D_b = alpha * alpha_b * op(A_b) op(B_b) + beta * Cin_b
// (or, with `reduce`, one D = beta * Cin + sum_b alpha*alpha_b op(A_b) op(B_b)).
// Column-major, op(X) = X or X^T.  Structural flags let a tile skip k-blocks
// that are known to be zero (triangular operands) and skip whole tiles of a
// symmetric result.  Zero regions of triangular operands must hold zeros in
// memory: only whole BK-blocks are skipped.
// ---------------------------------------------------------------------------
enum GemmFlags : unsigned {
    kAUpper = 1u,        // op(A)[i][k] == 0 for k < i   (k-range starts at tile row 0)
    kALower = 2u,        // op(A)[i][k] == 0 for k > i   (k-range ends at last tile row)
    kBUpper = 4u,        // op(B)[k][j] == 0 for k > j   (k-range ends at last tile column)
    kBLower = 8u,        // op(B)[k][j] == 0 for k < j   (k-range starts at tile column 0)
    kCUpperTiles = 16u,  // compute only tiles that meet the upper triangle (i <= j)
    kCStoreUpper = 32u,  // store only elements with i <= j
    kCStoreLower = 64u,  // store only elements with i >= j
};

constexpr int kMaxInlineAlpha = 16;

// T = double (FP64 path) or float (the FP32 steps of the mixed schedule).
template <class T>
struct GemmDescT {
    int m = 0, n = 0, k = 0;
    int transa = 0, transb = 0;
    const T* A = nullptr; long long lda = 0, strideA = 0;
    const T* B = nullptr; long long ldb = 0, strideB = 0;
    const T* Cin = nullptr; long long ldcin = 0, strideCin = 0;
    T* C = nullptr; long long ldc = 0, strideC = 0;
    double alpha = 1.0;
    double beta = 0.0;
    int batch = 1;
    int reduce = 0;          // sum the batch into one output
    // Optional second (outer) batch dimension, never reduced.
    int batch2 = 1;
    long long strideA2 = 0, strideB2 = 0, strideCin2 = 0, strideC2 = 0;
    unsigned flags = 0;
    int nalpha = 0;          // if > 0, alpha_b = alphas[b] (b < nalpha <= 16)
    double alphas[kMaxInlineAlpha] = {};
    // Split-K (batch2 must be 1): the k-range is cut into `splitk` pieces whose
    // partial products go to `work` (splitk x outputs x m x n, ld m) and a
    // second kernel sums them in order into C.
    int splitk = 1;
    T* work = nullptr;
    // Set by the launcher when the work per tile is uneven (triangular
    // operands, upper-tile outputs): XCD x takes the tiles [xsplit[x],
    // xsplit[x+1]) of the launch order, ranges cut to equal estimated work.
    int xbal = 0;
    int xsplit[9] = {};
    // Set by the launcher of a kernel that applies alpha and beta * Cin
    // itself (split-K pieces then hold scaled partials, piece 0 with Cin).
    int prescaled = 0;
};
using GemmDesc = GemmDescT<double>;
using SGemmDesc = GemmDescT<float>;

// Launches D = ... on `stream`.  Returns hipSuccess or the launch error.
hipError_t gemm(const GemmDesc& d, hipStream_t stream);
hipError_t gemm(const SGemmDesc& d, hipStream_t stream);
// As gemm(), but a product whose output has too few tiles to fill the chip
// and a long k-range is split along k into `work` (up to work_elems doubles).
hipError_t gemm_split(GemmDesc d, double* work, size_t work_elems, hipStream_t stream);

// Nonzeros of a trapezoidal operand with `r` rows (the side that is not k)
// and depth k: "from diagonal" = zero where k < r-index (upper op(A), lower
// op(B)), otherwise zero where k > r-index.
inline double trapezoid_nnz(double r, double k, bool from_diagonal) {
    if (from_diagonal) {
        const double s = r < k ? r : k;
        return s * k - s * (s - 1) / 2;
    }
    return r <= k ? r * (r + 1) / 2 : k * (k + 1) / 2 + (r - k) * k;
}

// Floating-point operations a descriptor executes: 2 m n k per product, a
// triangular or trapezoidal operand counted by its nonzeros (both
// triangular: one third of the full product, as for square triangles), and
// half for upper-tile outputs.
template <class T>
double gemm_flops(const GemmDescT<T>& d) {
    const double nb = (double)d.batch * d.batch2, m = d.m, n = d.n, k = d.k;
    const bool ta = d.flags & (kAUpper | kALower), tb = d.flags & (kBUpper | kBLower);
    double f;
    if (ta && tb) f = 2.0 * m * n * k / 3.0;
    else if (ta) f = 2.0 * n * trapezoid_nnz(m, k, d.flags & kAUpper);
    else if (tb) f = 2.0 * m * trapezoid_nnz(n, k, d.flags & kBLower);
    else f = 2.0 * m * n * k;
    if (d.flags & kCUpperTiles) f *= 0.5;
    return f * nb;
}

// Algorithmic memory traffic of a descriptor in bytes: the nonzeros of A and
// B once per batch, Cin when beta != 0 and C once per output (upper-tile
// outputs halved).
template <class T>
double gemm_bytes(const GemmDescT<T>& d) {
    const double nb = (double)d.batch * d.batch2, nout = (double)(d.reduce ? 1 : d.batch) * d.batch2;
    double a = (double)d.m * d.k, b = (double)d.k * d.n, c = (double)d.m * d.n;
    if (d.flags & (kAUpper | kALower)) a = trapezoid_nnz(d.m, d.k, d.flags & kAUpper);
    if (d.flags & (kBUpper | kBLower)) b = trapezoid_nnz(d.n, d.k, d.flags & kBLower);
    if (d.flags & kCUpperTiles) c *= 0.5;
    const double cin = (d.Cin && d.beta != 0.0) ? c : 0.0;
    return sizeof(T) * (nb * (a + b) + nout * (c + cin));
}

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------
__device__ inline d4 mfma_f64_16x16x4(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// 16 x 16 x 4 MFMA tiles for either precision.  Both take A[l % 16][l / 16]
// and B[l / 16][l % 16] from lane l; the accumulator rows differ:
// FP64 holds D[l / 16 + 4 e][l % 16], FP32 holds D[4 (l / 16) + e][l % 16].
template <class T> struct Mfma;
template <> struct Mfma<double> {
    typedef d4 acc;
    __device__ static acc run(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int e) { return (lane >> 4) + 4 * e; }
};
template <> struct Mfma<float> {
    typedef f4 acc;
    __device__ static acc run(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int e) { return 4 * (lane >> 4) + e; }
};

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Number of XCDs on MI355X; consecutive workgroup ids are dealt round-robin.
constexpr int kNumXcd = 8;

// Bijective remap of a linear block id so that consecutive logical ids land
// on the same XCD (and so share its L2).
__device__ inline int xcd_remap(int b, int nblocks) {
    if (nblocks < 2 * kNumXcd) return b;
    int q = nblocks / kNumXcd, rem = nblocks % kNumXcd;
    int x = b % kNumXcd, idx = b / kNumXcd;
    int base = x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q;
    return base + idx;
}

}  // namespace zolo
