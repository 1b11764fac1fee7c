// Shared definitions for the gfx950 Zolo-PD library (device helpers, launch
// descriptors).  Every kernel of the library is written for CDNA4: 64-lane
// wavefronts, FP64 MFMA 16x16x4 tiles, LDS staging.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace zolo {

typedef double d4 __attribute__((ext_vector_type(4)));

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

struct GemmDesc {
    int m = 0, n = 0, k = 0;
    int transa = 0, transb = 0;
    const double* A = nullptr; long long lda = 0, strideA = 0;
    const double* B = nullptr; long long ldb = 0, strideB = 0;
    const double* Cin = nullptr; long long ldcin = 0, strideCin = 0;
    double* C = nullptr; long long ldc = 0, strideC = 0;
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
};

// Launches D = ... on `stream`.  Returns hipSuccess or the launch error.
hipError_t gemm(const GemmDesc& d, hipStream_t stream);

// Rough count of the floating-point operations a descriptor executes
// (2 m n k per product, halved per triangular operand / upper-tile output).
double gemm_flops(const GemmDesc& d);

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------
__device__ inline d4 mfma_f64_16x16x4(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

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
