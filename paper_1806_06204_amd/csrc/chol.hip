// Batched upper Cholesky and triangular inverse (FP64, and FP32 for the mixed
// precision schedule) for the Cholesky-type step of Zolo-PD (Algorithm 1
// step 4(d)): Z_j = X^T X + c_{2j-1} I = R_j^T R_j for all j at once, then
// R_j^{-1}.
//
// POTRF is right-looking with 64-column blocks grouped in bands of 256: a
// 64 x 64 diagonal block is factored in LDS by one workgroup per matrix
// (which also inverts it), the row panel to its right becomes R_kk^{-T} Z_12
// (one GEMM), the rows of the band below the block take its rank-64 update,
// and once the band is done the matrix below it takes one rank-256 update on
// its upper tiles.  The trailing matrix is thus read and written once per
// 256 columns rather than once per 64.
//
// TRTRI is recursive and level-batched: all 64 x 64 diagonal blocks are
// inverted at once, then for block sizes s = 64, 128, 256, ... every pair of
// neighbouring s-blocks is merged with two GEMMs,
//     inv([R11 R12; 0 R22]) = [R11^{-1}, -R11^{-1} R12 R22^{-1}; 0, R22^{-1}],
// batched over all pairs of a level and all matrices.
#include "misc.hpp"
#include "stats.hpp"

namespace zolo {
namespace {

constexpr int kB = 64;
constexpr int kBand = 256;   // columns whose trailing update is applied at once

constexpr int kDB = 16;  // column block of the in-LDS factorisation

// Wave-uniform broadcast of lane l's value (readlane, no LDS round trip).
template <class T>
__device__ inline T lane_bcast(T x, int l) {
    if constexpr (sizeof(T) == 8) {
        const long long v = __double_as_longlong(x);
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)v, l);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(v >> 32), l);
        return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    } else {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
    }
}

// Inverse of the upper-triangular 64 x 64 matrix S (LDS; identity beyond the
// matrix) into Si (LDS), by the workgroup's 256 threads.  The four 16 x 16
// diagonal blocks are inverted at once (wave w inverts block w: lane j
// back-substitutes column j in registers); then the off-diagonal blocks at
// distance d = 1, 2, 3 follow from
//     Si[I][J] = -Si[I][I] sum_{K=I+1..J} S[I][K] Si[K][J].
template <class T>
__device__ void lds_upper_inverse(const T (*S)[kB + 1], T (*Si)[kB + 1]) {
    __shared__ T Y[3][kDB][kDB + 1];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int o = w * kDB;
    for (int e = tid; e < kB * kB; e += 256) Si[e % kB][e / kB] = 0;
    __syncthreads();
    if (lane < kDB) {
        const int j = lane;
        T x[kDB];
#pragma unroll
        for (int i = kDB - 1; i >= 0; --i) {
            T s = (i == j) ? (T)1 : (T)0;
#pragma unroll
            for (int k = i + 1; k < kDB; ++k) s -= S[o + i][o + k] * x[k];
            x[i] = i <= j ? s / S[o + i][o + i] : (T)0;
        }
#pragma unroll
        for (int i = 0; i < kDB; ++i) Si[o + i][o + j] = x[i];
    }
    __syncthreads();
    for (int d = 1; d < 4; ++d) {
        const int nblk = 4 - d;
        // Y_I = sum_{K=I+1..I+d} S[I][K] Si[K][I+d]
        for (int e = tid; e < nblk * kDB * kDB; e += 256) {
            const int I = e / (kDB * kDB), r = e % kDB, c = (e / kDB) % kDB;
            const int J = I + d;
            T acc = 0;
            for (int k = (I + 1) * kDB; k < (J + 1) * kDB; ++k) acc += S[I * kDB + r][k] * Si[k][J * kDB + c];
            Y[I][r][c] = acc;
        }
        __syncthreads();
        // Si[I][J] = -Si[I][I] Y_I
        for (int e = tid; e < nblk * kDB * kDB; e += 256) {
            const int I = e / (kDB * kDB), r = e % kDB, c = (e / kDB) % kDB;
            const int J = I + d;
            T acc = 0;
#pragma unroll
            for (int k = 0; k < kDB; ++k) acc += Si[I * kDB + r][I * kDB + k] * Y[I][k][c];
            Si[I * kDB + r][J * kDB + c] = -acc;
        }
        __syncthreads();
    }
}


// Upper Cholesky of the kb x kb diagonal block at (k0, k0) of each matrix
// (one workgroup per matrix), its inverse into work.  16-column blocks: wave
// 0 factors the 16 x 16 diagonal block in registers (lane j holds column j,
// rows broadcast with readlane), one thread per column solves the row panel
// to its right, and the trailing block takes the rank-16 update, so the
// factorisation needs 3 barriers per 16 columns.  A non-positive pivot is
// reported (1-based global column) and replaced by 1 so that every wave
// finishes; the caller discards the result.
template <class T>
__global__ __launch_bounds__(256) void potrf_diag_kernel(int k0, int kb, T* Z, long long ldz, long long sz,
                                                         int* info, T* work) {
    __shared__ T S[kB][kB + 1];
    __shared__ T Si[kB][kB + 1];
    __shared__ T s_rcp[kDB];
    __shared__ int s_bad;
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    T* Zb = Z + b * sz + k0 + (long long)k0 * ldz;
    for (int e = tid; e < kB * kB; e += 256) {
        const int i = e % kB, j = e / kB;
        S[i][j] = (i < kb && j < kb && i <= j) ? Zb[i + (long long)j * ldz] : (T)0;
    }
    if (tid == 0) s_bad = 0;
    __syncthreads();
    for (int jb = 0; jb < kb; jb += kDB) {
        const int bw = kb - jb < kDB ? kb - jb : kDB;
        if (tid < 64) {
            // Lane j < 16 holds column jb + j of the diagonal block.
            T c[kDB];
#pragma unroll
            for (int i = 0; i < kDB; ++i) c[i] = (lane < bw && i < bw) ? S[jb + i][jb + (lane & 15)] : (T)0;
            int bad = 0;
#pragma unroll
            for (int i = 0; i < kDB; ++i) {
                if (i < bw) {
                    T d = lane_bcast(c[i], i);
                    if (!(d > (T)0) || !isfinite(d)) {
                        if (bad == 0) bad = k0 + jb + i + 1;
                        d = 1;
                    }
                    const T r = sqrt(d), ri = (T)1 / r;
                    if (lane == 0) s_rcp[i] = ri;
                    c[i] = lane == i ? r : (lane > i ? c[i] * ri : c[i]);
#pragma unroll
                    for (int l = i + 1; l < kDB; ++l) {
                        const T ril = lane_bcast(c[i], l);  // R[i][jb + l]
                        if (lane >= l) c[l] -= ril * c[i];
                    }
                }
            }
            if (lane < bw) {
#pragma unroll
                for (int i = 0; i < kDB; ++i)
                    if (i < bw) S[jb + i][jb + lane] = i <= lane ? c[i] : (T)0;
            }
            if (lane == 0 && bad != 0 && s_bad == 0) s_bad = bad;
        }
        __syncthreads();
        const int c0 = jb + bw, w = kb - c0;
        if (w <= 0) break;
        // Row panel: R[jb:jb+bw, c] = R_d^{-T} Z[jb:jb+bw, c], one thread per column.
        if (tid < w) {
            const int col = c0 + tid;
            T x[kDB];
#pragma unroll
            for (int i = 0; i < kDB; ++i) {
                if (i < bw) {
                    T s0 = S[jb + i][col];
#pragma unroll
                    for (int k = 0; k < i; ++k) s0 -= S[jb + k][jb + i] * x[k];
                    x[i] = s0 * s_rcp[i];
                    S[jb + i][col] = x[i];
                }
            }
        }
        __syncthreads();
        // Trailing block (upper part): S[i][j] -= sum_k R[jb+k][i] R[jb+k][j].
        for (int e = tid; e < w * w; e += 256) {
            const int i = c0 + e % w, j = c0 + e / w;
            if (i <= j) {
                T acc = 0;
#pragma unroll
                for (int k = 0; k < kDB; ++k)
                    if (k < bw) acc += S[jb + k][i] * S[jb + k][j];
                S[i][j] -= acc;
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < kb * kb; e += 256) {
        const int i = e % kb, j = e / kb;
        Zb[i + (long long)j * ldz] = (i <= j) ? S[i][j] : (T)0;
    }
    if (tid >= kb && tid < kB) S[tid][tid] = 1;  // identity beyond the block
    __syncthreads();
    lds_upper_inverse<T>(S, Si);
    __syncthreads();
    T* wb = work + (long long)b * kB * kB;
    for (int e = tid; e < kB * kB; e += 256) {
        const int i = e % kB, j = e / kB;
        wb[e] = Si[i][j];
    }
    if (tid == 0 && s_bad != 0 && info[b] == 0) info[b] = s_bad;
}

// Invert every 64 x 64 diagonal block of R_b into Rinv_b.
template <class T>
__global__ __launch_bounds__(256) void trtri_diag_kernel(int n, const T* R, long long ldr, long long sr, T* Rinv,
                                                         long long ldi, long long si) {
    __shared__ T S[kB][kB + 1];
    __shared__ T Si[kB][kB + 1];
    const int blk = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
    const int o = blk * kB, kb = min(kB, n - o);
    const T* Rb = R + b * sr + o + (long long)o * ldr;
    T* Ib = Rinv + b * si + o + (long long)o * ldi;
    for (int e = tid; e < kB * kB; e += 256) {
        const int i = e % kB, j = e / kB;
        S[i][j] = (i < kb && j < kb && i <= j) ? Rb[i + (long long)j * ldr] : (T)(i == j ? 1 : 0);
    }
    __syncthreads();
    lds_upper_inverse<T>(S, Si);
    for (int e = tid; e < kb * kb; e += 256) {
        const int i = e % kb, j = e / kb;
        Ib[i + (long long)j * ldi] = Si[i][j];
    }
}

}  // namespace

template <class T>
hipError_t potrf_batched(int n, T* Z, long long ldz, long long sz, int batch, int* info_dev, T* work,
                         hipStream_t st) {
    hipError_t e = zero_ints(info_dev, batch, st);
    if (e != hipSuccess) return e;
    for (int k0 = 0; k0 < n; k0 += kBand) {
        const int band = n - k0 < kBand ? n - k0 : kBand;
        for (int j0 = k0; j0 < k0 + band; j0 += kB) {
            const int kb = k0 + band - j0 < kB ? k0 + band - j0 : kB;
            StatScope sc(sizeof(T) == 8 ? "potrf_diag_kernel<double>" : "potrf_diag_kernel<float>", st,
                         batch * (double)kb * kb * kb / 3.0);
            potrf_diag_kernel<T><<<batch, 256, 0, st>>>(j0, kb, Z, ldz, sz, info_dev, work);
            sc.end();
            if ((e = hipGetLastError()) != hipSuccess) return e;
            const int rest = n - j0 - kb;
            if (rest <= 0) break;
            T* Z12 = Z + j0 + (long long)(j0 + kb) * ldz;
            // R12 = R_kk^{-T} Z12 over the whole width, in place (one tile
            // row covers all kb rows).
            GemmDescT<T> g;
            g.m = kb; g.n = rest; g.k = kb; g.transa = 1; g.transb = 0;
            g.A = work; g.lda = kB; g.strideA = (long long)kB * kB;
            g.B = Z12; g.ldb = ldz; g.strideB = sz;
            g.C = Z12; g.ldc = ldz; g.strideC = sz;
            g.beta = 0.0; g.batch = batch; g.flags = kALower;
            if ((e = gemm(g, st)) != hipSuccess) return e;
            // Rows of the band below this block take its rank-kb update now
            // (the next blocks of the band need them); the matrix below the
            // band waits for the band's combined update.
            const int rows = k0 + band - j0 - kb;
            if (rows > 0) {
                T* Z22 = Z + (j0 + kb) + (long long)(j0 + kb) * ldz;
                GemmDescT<T> u;
                u.m = rows; u.n = rest; u.k = kb; u.transa = 1; u.transb = 0;
                u.A = Z12; u.lda = ldz; u.strideA = sz;
                u.B = Z12; u.ldb = ldz; u.strideB = sz;
                u.Cin = Z22; u.ldcin = ldz; u.strideCin = sz;
                u.C = Z22; u.ldc = ldz; u.strideC = sz;
                u.alpha = -1.0; u.beta = 1.0; u.batch = batch;
                u.flags = kCUpperTiles | kCStoreUpper;
                if ((e = gemm(u, st)) != hipSuccess) return e;
            }
        }
        // Below the band: Z22 -= P^T P with P = the band's rows of R to the
        // right of the band (one rank-`band` update instead of band/64).
        const int rest = n - k0 - band;
        if (rest <= 0) break;
        T* P = Z + k0 + (long long)(k0 + band) * ldz;
        T* Z22 = Z + (k0 + band) + (long long)(k0 + band) * ldz;
        GemmDescT<T> s;
        s.m = rest; s.n = rest; s.k = band; s.transa = 1; s.transb = 0;
        s.A = P; s.lda = ldz; s.strideA = sz;
        s.B = P; s.ldb = ldz; s.strideB = sz;
        s.Cin = Z22; s.ldcin = ldz; s.strideCin = sz;
        s.C = Z22; s.ldc = ldz; s.strideC = sz;
        s.alpha = -1.0; s.beta = 1.0; s.batch = batch;
        s.flags = kCUpperTiles | kCStoreUpper;
        if ((e = gemm(s, st)) != hipSuccess) return e;
    }
    return zero_strict_lower<T>(n, Z, ldz, sz, batch, st);
}
template hipError_t potrf_batched<double>(int, double*, long long, long long, int, int*, double*, hipStream_t);
template hipError_t potrf_batched<float>(int, float*, long long, long long, int, int*, float*, hipStream_t);

template <class T>
hipError_t trtri_batched(int n, const T* R, long long ldr, long long sr, T* Rinv, long long ldi, long long si,
                         int batch, T* work, long long work_elems, hipStream_t st) {
    hipError_t e = fill_matrix<T>(n, n, Rinv, ldi, si, batch, 0.0, 0.0, st);
    if (e != hipSuccess) return e;
    const int nblk = (n + kB - 1) / kB;
    trtri_diag_kernel<T><<<dim3(nblk, batch), 256, 0, st>>>(n, R, ldr, sr, Rinv, ldi, si);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (long long s = kB; s < n; s *= 2) {
        const long long full = n / (2 * s);           // pairs with both blocks of size s
        const long long o_rag = full * 2 * s;          // a ragged pair starts here if o_rag + s < n
        const long long s2_rag = n - o_rag - s;
        const long long per_b = full * s * s + (s2_rag > 0 ? s * s2_rag : 0);
        if (per_b * batch > work_elems) return hipErrorInvalidValue;
        for (int part = 0; part < 2; ++part) {
            const long long npairs = part == 0 ? full : (s2_rag > 0 ? 1 : 0);
            if (npairs == 0) continue;
            const long long o = part == 0 ? 0 : o_rag;
            const long long s2 = part == 0 ? s : s2_rag;
            T* Wp = work + (part == 0 ? 0 : full * s * s);
            // W = R12 * R22^{-1}
            GemmDescT<T> g;
            g.m = (int)s; g.n = (int)s2; g.k = (int)s2;
            g.A = R + o + (o + s) * ldr; g.lda = ldr; g.strideA = 2 * s * (ldr + 1);
            g.B = Rinv + (o + s) + (o + s) * ldi; g.ldb = ldi; g.strideB = 2 * s * (ldi + 1);
            g.C = Wp; g.ldc = s; g.strideC = s * s2;
            g.batch = (int)npairs; g.flags = kBUpper;
            g.batch2 = batch; g.strideA2 = sr; g.strideB2 = si; g.strideC2 = per_b;
            if ((e = gemm(g, st)) != hipSuccess) return e;
            // Rinv12 = -R11^{-1} W
            GemmDescT<T> h;
            h.m = (int)s; h.n = (int)s2; h.k = (int)s;
            h.A = Rinv + o + o * ldi; h.lda = ldi; h.strideA = 2 * s * (ldi + 1);
            h.B = Wp; h.ldb = s; h.strideB = s * s2;
            h.C = Rinv + o + (o + s) * ldi; h.ldc = ldi; h.strideC = 2 * s * (ldi + 1);
            h.alpha = -1.0; h.batch = (int)npairs; h.flags = kAUpper;
            h.batch2 = batch; h.strideA2 = si; h.strideB2 = per_b; h.strideC2 = si;
            if ((e = gemm(h, st)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

template hipError_t trtri_batched<double>(int, const double*, long long, long long, double*, long long, long long,
                                          int, double*, long long, hipStream_t);
template hipError_t trtri_batched<float>(int, const float*, long long, long long, float*, long long, long long, int,
                                         float*, long long, hipStream_t);

}  // namespace zolo
