// Structured Householder QR of the stacked matrices [D_b; Y_b], D_b = p_b I
// (n x n, the identity block of eq. (12) scaled by p_b = sqrt(c_{2b-1})),
// Y_b dense m x n, for all b at once (Section 3.1 of the paper).
//
// Storage puts the identity block on top.  Then every reflector pivots on its
// own row of D and touches that row plus the m rows of Y: it has m + 1
// nonzeros, its D-part is a unit vector, and a block of NB = 64 reflectors
// has m + NB live rows, as in the paper's structured routines.  V = [I; Y_V],
// so only Y_V is stored (in place of Y) and V^T V = I + Y_V^T Y_V.
//
// Panel: one cooperative launch per panel factors all b together.  Each
// matrix gets G workgroups, each owning a slab of Y rows; per column k the
// workgroups apply reflector k-1 to their rows and accumulate the dot
// products of column k with every panel column in the same pass, so one
// cross-workgroup reduction per column gives the norm, the new R row and the
// next column of T (compact WY, Q = I - V T V^T).  The reduction is
// deterministic (fixed summation order) and its barrier has a bounded wait.
//
// Trailing update and Q formation are three GEMMs per panel on the MFMA
// kernel:  W = Y_V^T C_Y,  C_D = -T^T W (written into R's row block),
// C_Y += Y_V C_D.  ORGQR applies the panels last to first to [I; 0].
#include "misc.hpp"

namespace zolo {
namespace {

constexpr int kNB = kPanelNB;
constexpr int kPT = 256;                 // threads per panel workgroup
constexpr int kColsPerWave = kNB / 4;    // panel columns owned by each wave

struct PanelArgs {
    int m, nb, G, rows_per_wg;
    double* Y; long long ldy, sy;        // column p0 of Y_0
    double* D; long long ldd, sd;        // D_0[p0][p0]
    double* T; long long st;             // T_b, kNB x kNB column-major
    double* partials;                    // [batch][2][G][kNB]
    unsigned* counters;                  // [batch]
    int* error_flag;
    unsigned spin_limit;
    double pivot[kMaxInlineAlpha];
};

__global__ __launch_bounds__(kPT) void panel_kernel(PanelArgs a) {
    __shared__ double sT[kNB][kNB + 1];
    __shared__ double s_d[kNB], s_coef[kNB], s_wsum[kNB], s_z[kNB];
    const int g = blockIdx.x % a.G, b = blockIdx.x / a.G;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long ldy = a.ldy;
    double* __restrict__ Y = a.Y + b * a.sy;
    const int r0 = g * a.rows_per_wg;
    const int r1 = min(a.m, r0 + a.rows_per_wg);
    const int nb = a.nb;
    for (int e = tid; e < kNB * kNB; e += kPT) sT[e / kNB][e % kNB] = 0.0;
    if (tid < kNB) s_coef[tid] = 0.0;
    __syncthreads();
    const double alpha = a.pivot[b];
    unsigned* ctr = a.counters + b;

    for (int k = 0; k < nb; ++k) {
        // Phase A: apply reflector k-1 to columns > k of this slab (each wave
        // owns columns wave, wave+4, ...) and accumulate dots with column k.
        double acc[kColsPerWave];
#pragma unroll
        for (int q = 0; q < kColsPerWave; ++q) acc[q] = 0.0;
        const double ck = k > 0 ? s_coef[k] : 0.0;
        for (int row = r0 + lane; row < r1; row += 64) {
            const double vprev = k > 0 ? Y[row + (k - 1) * ldy] : 0.0;
            const double yk = Y[row + k * ldy] - ck * vprev;
#pragma unroll
            for (int q = 0; q < kColsPerWave; ++q) {
                const int i = wave + 4 * q;
                if (i < nb) {
                    double val;
                    if (i == k) {
                        val = yk;
                    } else {
                        val = Y[row + i * ldy];
                        if (i > k && k > 0) {
                            val -= s_coef[i] * vprev;
                            Y[row + i * ldy] = val;
                        }
                    }
                    acc[q] += yk * val;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kColsPerWave; ++q) {
            const double s = wave_sum(acc[q]);
            const int i = wave + 4 * q;
            if (lane == 0 && i < nb) s_wsum[i] = s;
        }
        __syncthreads();

        // Phase B: publish this slab's partial dots, wait for the other slabs
        // of the same matrix, and sum all partials in a fixed order.
        double* part = a.partials + (((long long)b * 2 + (k & 1)) * a.G + g) * kNB;
        if (tid < nb) __hip_atomic_store(&part[tid], s_wsum[tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        if (tid == 0) {
            __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned target = (unsigned)(k + 1) * (unsigned)a.G;
            unsigned spins = 0;
            while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (++spins > a.spin_limit) {
                    atomicOr(a.error_flag, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
        if (tid < nb) {
            const double* pb = a.partials + ((long long)b * 2 + (k & 1)) * a.G * kNB;
            double s = 0.0;
            for (int gg = 0; gg < a.G; ++gg)
                s += __hip_atomic_load(&pb[gg * kNB + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_d[tid] = s;
        }
        __syncthreads();

        // Phase C: reflector k.  x = [alpha; y_k], beta = -sqrt(alpha^2 + |y_k|^2)
        // (alpha > 0, so alpha - beta never cancels), v = [1; y_k/(alpha-beta)].
        const double beta = -sqrt(alpha * alpha + s_d[k]);
        const double tau = (beta - alpha) / beta;
        const double scale = 1.0 / (alpha - beta);
        if (tid < nb) {
            if (tid > k) s_coef[tid] = tau * scale * s_d[tid];   // tau * (v_k^T column)
            if (tid < k) s_z[tid] = scale * s_d[tid];            // v_i^T v_k
        }
        __syncthreads();
        if (tid < k) {
            double s = 0.0;
            for (int l = tid; l < k; ++l) s += sT[tid][l] * s_z[l];
            sT[tid][k] = -tau * s;
        }
        if (tid == 0) sT[k][k] = tau;
        if (g == 0 && tid < nb) {
            double* Db = a.D + b * a.sd;
            if (tid == k) Db[k + k * a.ldd] = beta;
            if (tid > k) Db[k + tid * a.ldd] = -s_coef[tid];
        }
        // Phase D: store v_k = scale * (column k after reflector k-1).
        for (int row = r0 + tid; row < r1; row += kPT) {
            const double vprev = k > 0 ? Y[row + (k - 1) * ldy] : 0.0;
            Y[row + k * ldy] = scale * (Y[row + k * ldy] - ck * vprev);
        }
        __syncthreads();
    }
    if (g == 0) {
        double* Tb = a.T + b * a.st;
        for (int e = tid; e < kNB * kNB; e += kPT) Tb[e] = sT[e % kNB][e / kNB];
    }
}

// D_b[p0+i][p0+j] = delta_ij - T_b[i][j] for the panel's diagonal block.
__global__ void i_minus_t_kernel(int nb, double* D, long long ldd, long long sd, const double* T, long long st) {
    const int b = blockIdx.x;
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
        const int i = e % nb, j = e / nb;
        D[b * sd + i + j * ldd] = (i == j ? 1.0 : 0.0) - T[b * st + i + j * kNB];
    }
}

struct Geometry {
    int G, rows;
};

Geometry panel_geometry(int m, int batch, int max_coresident) {
    // Aim for ~256 rows per workgroup and keep every workgroup resident.
    int G = (m + 255) / 256;
    if (G < 1) G = 1;
    int cap = max_coresident / batch;
    if (cap < 1) cap = 1;
    if (G > cap) G = cap;
    int rows = (m + G - 1) / G;
    G = (m + rows - 1) / rows;
    return {G, rows};
}

hipError_t launch_panel(PanelArgs& pa, int batch, hipStream_t st) {
    void* args[] = {&pa};
    return hipLaunchCooperativeKernel((const void*)panel_kernel, dim3(pa.G * batch), dim3(kPT), args, 0, st);
}

}  // namespace

int panel_max_coresident() {
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)panel_kernel, kPT, 0) != hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t structured_geqrf(int m, int n, double* Y, long long ldy, long long sy, double* D, long long ldd,
                            long long sd, const double* pivots, int batch, const QrWork& w, hipStream_t st) {
    if (batch > kMaxInlineAlpha) return hipErrorInvalidValue;
    const int npanels = (n + kNB - 1) / kNB;
    const Geometry geo = panel_geometry(m, batch, w.max_coresident);
    hipError_t e = hipMemsetAsync(w.counters, 0, sizeof(unsigned) * (size_t)batch * npanels, st);
    if (e != hipSuccess) return e;
    for (int p = 0; p < npanels; ++p) {
        const int p0 = p * kNB;
        const int nb = n - p0 < kNB ? n - p0 : kNB;
        PanelArgs pa;
        pa.m = m; pa.nb = nb; pa.G = geo.G; pa.rows_per_wg = geo.rows;
        pa.Y = Y + (long long)p0 * ldy; pa.ldy = ldy; pa.sy = sy;
        pa.D = D + p0 + (long long)p0 * ldd; pa.ldd = ldd; pa.sd = sd;
        pa.T = w.T + (long long)p * kNB * kNB; pa.st = (long long)npanels * kNB * kNB;
        pa.partials = w.partials;
        pa.counters = w.counters + (long long)p * batch;
        pa.error_flag = w.error_flag;
        pa.spin_limit = 1u << 22;
        for (int b = 0; b < batch; ++b) pa.pivot[b] = pivots[b];
        if ((e = launch_panel(pa, batch, st)) != hipSuccess) return e;
        const int trail = n - p0 - nb;
        if (trail <= 0) continue;
        double* YV = Y + (long long)p0 * ldy;
        double* Yt = Y + (long long)(p0 + nb) * ldy;
        double* Dt = D + p0 + (long long)(p0 + nb) * ldd;
        // W = Y_V^T Y_trail
        GemmDesc g1;
        g1.m = nb; g1.n = trail; g1.k = m; g1.transa = 1;
        g1.A = YV; g1.lda = ldy; g1.strideA = sy;
        g1.B = Yt; g1.ldb = ldy; g1.strideB = sy;
        g1.C = w.W; g1.ldc = kNB; g1.strideC = (long long)kNB * n;
        g1.batch = batch;
        if ((e = gemm(g1, st)) != hipSuccess) return e;
        // R row block = -T^T W
        GemmDesc g2;
        g2.m = nb; g2.n = trail; g2.k = nb; g2.transa = 1;
        g2.A = pa.T; g2.lda = kNB; g2.strideA = pa.st;
        g2.B = w.W; g2.ldb = kNB; g2.strideB = (long long)kNB * n;
        g2.C = Dt; g2.ldc = ldd; g2.strideC = sd;
        g2.alpha = -1.0; g2.batch = batch; g2.flags = kALower;
        if ((e = gemm(g2, st)) != hipSuccess) return e;
        // Y_trail += Y_V (R row block)
        GemmDesc g3;
        g3.m = m; g3.n = trail; g3.k = nb;
        g3.A = YV; g3.lda = ldy; g3.strideA = sy;
        g3.B = Dt; g3.ldb = ldd; g3.strideB = sd;
        g3.Cin = Yt; g3.ldcin = ldy; g3.strideCin = sy;
        g3.C = Yt; g3.ldc = ldy; g3.strideC = sy;
        g3.beta = 1.0; g3.batch = batch;
        if ((e = gemm(g3, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t structured_orgqr(int m, int n, double* Y, long long ldy, long long sy, double* D, long long ldd,
                            long long sd, int batch, const QrWork& w, hipStream_t st) {
    const int npanels = (n + kNB - 1) / kNB;
    const long long stT = (long long)npanels * kNB * kNB;
    hipError_t e;
    for (int p = npanels - 1; p >= 0; --p) {
        const int p0 = p * kNB;
        const int nb = n - p0 < kNB ? n - p0 : kNB;
        const int trail = n - p0 - nb;
        const double* Tp = w.T + (long long)p * kNB * kNB;
        double* YV = Y + (long long)p0 * ldy;
        if (trail > 0) {
            double* Yt = Y + (long long)(p0 + nb) * ldy;
            double* Dt = D + p0 + (long long)(p0 + nb) * ldd;
            // W = Y_V^T Q_Y[:, trail]
            GemmDesc g1;
            g1.m = nb; g1.n = trail; g1.k = m; g1.transa = 1;
            g1.A = YV; g1.lda = ldy; g1.strideA = sy;
            g1.B = Yt; g1.ldb = ldy; g1.strideB = sy;
            g1.C = w.W; g1.ldc = kNB; g1.strideC = (long long)kNB * n;
            g1.batch = batch;
            if ((e = gemm(g1, st)) != hipSuccess) return e;
            // Q_D[panel rows, trail] = -T W
            GemmDesc g2;
            g2.m = nb; g2.n = trail; g2.k = nb;
            g2.A = Tp; g2.lda = kNB; g2.strideA = stT;
            g2.B = w.W; g2.ldb = kNB; g2.strideB = (long long)kNB * n;
            g2.C = Dt; g2.ldc = ldd; g2.strideC = sd;
            g2.alpha = -1.0; g2.batch = batch; g2.flags = kAUpper;
            if ((e = gemm(g2, st)) != hipSuccess) return e;
            // Q_Y[:, trail] += Y_V Q_D[panel rows, trail]
            GemmDesc g3;
            g3.m = m; g3.n = trail; g3.k = nb;
            g3.A = YV; g3.lda = ldy; g3.strideA = sy;
            g3.B = Dt; g3.ldb = ldd; g3.strideB = sd;
            g3.Cin = Yt; g3.ldcin = ldy; g3.strideCin = sy;
            g3.C = Yt; g3.ldc = ldy; g3.strideC = sy;
            g3.beta = 1.0; g3.batch = batch;
            if ((e = gemm(g3, st)) != hipSuccess) return e;
        }
        // Panel columns: Q_D block = I - T, Q_Y[:, panel] = -Y_V T (in place;
        // one tile column covers all nb <= 64 columns).
        i_minus_t_kernel<<<batch, 256, 0, st>>>(nb, D + p0 + (long long)p0 * ldd, ldd, sd, Tp, stT);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        GemmDesc g4;
        g4.m = m; g4.n = nb; g4.k = nb;
        g4.A = YV; g4.lda = ldy; g4.strideA = sy;
        g4.B = Tp; g4.ldb = kNB; g4.strideB = stT;
        g4.C = YV; g4.ldc = ldy; g4.strideC = sy;
        g4.alpha = -1.0; g4.batch = batch; g4.flags = kBUpper;
        if ((e = gemm(g4, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace zolo
