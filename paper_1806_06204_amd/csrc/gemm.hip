// GEMM on CDNA4 matrix cores: FP64 (v_mfma_f64_16x16x4f64) and, for the FP32
// steps of the mixed precision schedule, FP32 (v_mfma_f32_16x16x4f32).
//
// Every BLAS3 phase of Zolo-PD (trailing updates and Q formation of the
// structured QR, the Gram matrix X^T X, the Cholesky trailing updates,
// triangular inverses, the Zolotarev combination and H = Qp^T A) is a call of
// this kernel with different structure flags.
//
// Tiling: a 256-thread workgroup (4 waves, 2 x 2) owns a BM x BN tile of the
// result; each wave owns (BM/2) x (BN/2) as a grid of 16 x 16 MFMA blocks held
// in accumulator registers.  K is walked in BK = 16 slices staged through LDS
// (k-major, so that a fragment load is 16 consecutive doubles); the next slice
// is fetched into registers while the current one feeds the MFMAs.
// Lane layout (lane l, accumulator element e): A[l % 16][l / 16],
// B[l / 16][l % 16]; D[l / 16 + 4 e][l % 16] for FP64, D[4 (l / 16) + e][l % 16]
// for FP32.  Tiles are
// ordered in groups of 8 tile-rows and the workgroup ids are remapped so that
// neighbouring tiles run on the same XCD and reuse its L2.
#include "common.hpp"
#include "stats.hpp"

#include <algorithm>
#include <atomic>
#include <mutex>
#include <unordered_map>
#include <type_traits>
#include <cstdio>
#include <cstdlib>

namespace zolo {
namespace {

constexpr int kBK = 16;
constexpr int kPad = 4;
constexpr int kTileGroup = 8;   // tiles are ordered in groups of 8 tile-rows

// 128 x 128 tiles hold 128 accumulator doubles per lane: one wave per SIMD
// (512 registers); smaller tiles run two.
template <class T, int BM, int BN, bool TA, bool TB>
__global__ __launch_bounds__(256, (BM * BN >= 128 * 128) ? 1 : 2) void gemm_kernel(GemmDescT<T> d) {
    typedef typename Mfma<T>::acc acc_t;
    constexpr int BK = kBK;
    constexpr int FM = BM / 32, FN = BN / 32;
    constexpr int APT = BM * BK / 256, BPT = BN * BK / 256;
    __shared__ T As[2][BK][BM + kPad];
    __shared__ T Bs[2][BK][BN + kPad];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * (BN / 2);
    const int tiles_m = (d.m + BM - 1) / BM, tiles_n = (d.n + BN - 1) / BN;
    const int nblocks = tiles_m * tiles_n;
    int lin;
    if (d.xbal) {
        // Workgroup ids are dealt to the XCDs round-robin (the grid's x
        // extent is a multiple of 8): XCD x walks its own range of tiles.
        const int x = blockIdx.x % kNumXcd, idx = blockIdx.x / kNumXcd;
        lin = d.xsplit[x] + idx;
        if (lin >= d.xsplit[x + 1]) return;
    } else {
        lin = xcd_remap(blockIdx.x, nblocks);
    }
    constexpr int GROUP = kTileGroup;
    const int in_group = GROUP * tiles_n;
    const int first_m = (lin / in_group) * GROUP;
    const int gsize = min(tiles_m - first_m, GROUP);
    const int tm = first_m + (lin % in_group) % gsize;
    const int tn = (lin % in_group) / gsize;
    const int row0 = tm * BM, col0 = tn * BN;
    if ((d.flags & kCUpperTiles) && row0 > col0 + BN - 1) return;

    const unsigned fl = d.flags;
    int kb = 0, ke = d.k;
    if (fl & kAUpper) kb = max(kb, row0);
    if (fl & kBLower) kb = max(kb, col0);
    if (fl & kALower) ke = min(ke, row0 + BM);
    if (fl & kBUpper) ke = min(ke, col0 + BN);
    const int nk = ke > kb ? (ke - kb + BK - 1) / BK : 0;
    const int nbatch = d.reduce ? d.batch : 1;
    const int bfirst = d.reduce ? 0 : blockIdx.y;
    const int ntiles = nk * nbatch;   // (batch, k) slices walked as one sequence
    const bool split = d.splitk > 1;
    const int z2 = split ? 0 : blockIdx.z;                 // outer batch index
    const int t_begin = split ? (int)((long long)blockIdx.z * ntiles / d.splitk) : 0;
    const int t_end = split ? (int)((long long)(blockIdx.z + 1) * ntiles / d.splitk) : ntiles;
    const int nt = t_end - t_begin;

    acc_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    // Staging registers: raw loaded values, their validity bits and the
    // batch multiplier; masking and scaling happen at the LDS store so that
    // nothing consumes a load before the MFMAs of the current slice.
    T ra[APT], rb[BPT];
    unsigned amask = 0, bmask = 0;
    T al_cur = 1;
    // Loads are unconditional from a clamped (always valid) address and then
    // masked with a select, so no branch separates them from the MFMAs.
    auto gload = [&](int t) {
        const int bi = t / nk;
        const int k0 = kb + (t - bi * nk) * BK;
        const int b = bfirst + bi;
        const T* __restrict__ A = d.A + (long long)b * d.strideA + (long long)z2 * d.strideA2;
        const T* __restrict__ B = d.B + (long long)b * d.strideB + (long long)z2 * d.strideB2;
        al_cur = d.nalpha > 0 ? (T)d.alphas[b] : (T)1;
        amask = 0;
        bmask = 0;
#pragma unroll
        for (int s = 0; s < APT; ++s) {
            const int e = tid + 256 * s;
            const int i = TA ? e / BK : e % BM;
            const int kk = TA ? e % BK : e / BM;
            const int gi = row0 + i, gk = k0 + kk;
            bool ok = gi < d.m && gk < ke;
            if (fl & kAUpper) ok = ok && gk >= gi;
            if (fl & kALower) ok = ok && gk <= gi;
            const long long off = TA ? gk + (long long)gi * d.lda : gi + (long long)gk * d.lda;
            ra[s] = A[ok ? off : 0];
            amask |= ok ? (1u << s) : 0u;
        }
#pragma unroll
        for (int s = 0; s < BPT; ++s) {
            const int e = tid + 256 * s;
            const int j = TB ? e % BN : e / BK;
            const int kk = TB ? e / BN : e % BK;
            const int gj = col0 + j, gk = k0 + kk;
            bool ok = gj < d.n && gk < ke;
            if (fl & kBUpper) ok = ok && gk <= gj;
            if (fl & kBLower) ok = ok && gk >= gj;
            const long long off = TB ? gj + (long long)gk * d.ldb : gk + (long long)gj * d.ldb;
            rb[s] = B[ok ? off : 0];
            bmask |= ok ? (1u << s) : 0u;
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int s = 0; s < APT; ++s) {
            const int e = tid + 256 * s;
            const int i = TA ? e / BK : e % BM;
            const int kk = TA ? e % BK : e / BM;
            As[buf][kk][i] = (amask >> s) & 1u ? ra[s] * al_cur : (T)0;
        }
#pragma unroll
        for (int s = 0; s < BPT; ++s) {
            const int e = tid + 256 * s;
            const int j = TB ? e % BN : e / BK;
            const int kk = TB ? e / BN : e % BK;
            Bs[buf][kk][j] = (bmask >> s) & 1u ? rb[s] : (T)0;
        }
    };

    // The Cin tile is loaded before the k-loop so that its latency hides
    // behind the MFMAs (read in the epilogue, one load would wait for the
    // previous store: Cin and C may be the same array).  Out-of-range lanes
    // load a valid address and drop the value.
    const int ob = d.reduce ? 0 : blockIdx.y;
    T* __restrict__ C = d.C + (long long)ob * d.strideC + (long long)z2 * d.strideC2;
    const T* Cin = d.Cin ? d.Cin + (long long)ob * d.strideCin + (long long)z2 * d.strideCin2 : nullptr;
    const T alpha = (T)d.alpha, beta = (T)d.beta;
    const bool use_cin = !split && Cin != nullptr && d.beta != 0.0;
    T cin[FM][FN][4];
    if (use_cin) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int gi = row0 + wm + i * 16 + Mfma<T>::row(lane, e);
                    const int gj = col0 + wn + j * 16 + (lane & 15);
                    const bool ok = gi < d.m && gj < d.n;
                    cin[i][j][e] = Cin[ok ? gi + (long long)gj * d.ldcin : 0];
                }
    }

    if (nt > 0) {
        gload(t_begin);
        lstore(0);
        __syncthreads();
        if (nt > 1) gload(t_begin + 1);
        for (int u = 0; u < nt; ++u) {
            const int cur = u & 1;
            // Fragments of the next 4-deep step are read into the other
            // register set while the MFMAs of this one run.
            T af[2][FM], bf[2][FN];
            {
                const int kr = lane >> 4;
#pragma unroll
                for (int i = 0; i < FM; ++i) af[0][i] = As[cur][kr][wm + i * 16 + (lane & 15)];
#pragma unroll
                for (int j = 0; j < FN; ++j) bf[0][j] = Bs[cur][kr][wn + j * 16 + (lane & 15)];
            }
#pragma unroll
            for (int k4 = 0; k4 < BK; k4 += 4) {
                const int p = (k4 >> 2) & 1;
                if (k4 + 4 < BK) {
                    const int kr = k4 + 4 + (lane >> 4);
#pragma unroll
                    for (int i = 0; i < FM; ++i) af[p ^ 1][i] = As[cur][kr][wm + i * 16 + (lane & 15)];
#pragma unroll
                    for (int j = 0; j < FN; ++j) bf[p ^ 1][j] = Bs[cur][kr][wn + j * 16 + (lane & 15)];
                }
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc[i][j] = Mfma<T>::run(af[p][i], bf[p][j], acc[i][j]);
            }
            if (u + 1 < nt) {
                // The other buffer was last read in iteration u-1, before the
                // barrier that ended it, so it can be refilled now.  Keep the
                // stores (which wait for the loads in flight) after the MFMAs.
                __builtin_amdgcn_sched_barrier(0);
                lstore(cur ^ 1);
                __syncthreads();
                if (u + 2 < nt) gload(t_begin + u + 2);
            }
        }
    }

    if (split) {
        // Raw partial product of this k-piece; the reduce kernel scales,
        // adds Cin and applies the store masks.
        const int nout = d.reduce ? 1 : d.batch;
        T* __restrict__ Wp = d.work + ((long long)blockIdx.z * nout + ob) * ((long long)d.m * d.n);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int gi = row0 + wm + i * 16 + Mfma<T>::row(lane, e);
                    const int gj = col0 + wn + j * 16 + (lane & 15);
                    if (gi < d.m && gj < d.n) Wp[gi + (long long)gj * d.m] = acc[i][j][e];
                }
        return;
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gi = row0 + wm + i * 16 + Mfma<T>::row(lane, e);
                const int gj = col0 + wn + j * 16 + (lane & 15);
                bool ok = gi < d.m && gj < d.n;
                if (fl & kCStoreUpper) ok = ok && gi <= gj;
                if (fl & kCStoreLower) ok = ok && gi >= gj;
                if (ok) {
                    T v = alpha * acc[i][j][e];
                    if (use_cin) v += beta * cin[i][j][e];
                    C[gi + (long long)gj * d.ldc] = v;
                }
            }
}

// C = alpha * (sum over the k-pieces in order) + beta * Cin, with the store masks.
template <class T>
__global__ void splitk_reduce_kernel(GemmDescT<T> d) {
    const int nout = d.reduce ? 1 : d.batch;
    const long long mn = (long long)d.m * d.n, total = mn * nout;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long ob = e / mn, r = e - ob * mn;
        const int gj = (int)(r / d.m), gi = (int)(r - (long long)gj * d.m);
        bool ok = true;
        if (d.flags & kCStoreUpper) ok = ok && gi <= gj;
        if (d.flags & kCStoreLower) ok = ok && gi >= gj;
        if (!ok) continue;
        T s = 0;
        for (int z = 0; z < d.splitk; ++z) s += d.work[((long long)z * nout + ob) * mn + r];
        T v = s;
        if (!d.prescaled) {
            v = (T)d.alpha * s;
            if (d.Cin && d.beta != 0.0) v += (T)d.beta * d.Cin[ob * d.strideCin + gi + (long long)gj * d.ldcin];
        }
        d.C[ob * d.strideC + gi + (long long)gj * d.ldc] = v;
    }
}

// With triangular operands or an upper-tile output the work per tile varies
// across the launch order (k-ranges that shrink with the tile row or column,
// tiles that exit at once), and equal tile counts per XCD leave the XCD with
// the long tiles running alone at the end: measured 1.8-2.6x slower than
// balanced on the triangular products of the Cholesky-type step.  The launch
// order is cut into 8 ranges of equal estimated work (k-slices, plus the
// epilogue), one per XCD; the grid holds 8 x the longest range and the
// surplus workgroups return at once.  Returns the grid's x extent.
// The cut depends only on the launch shape, so it is cached (a solve issues
// the same shapes again in every step).
struct BalanceKey {
    int m, n, k, bm, bn, nbatch;
    unsigned flags;
    bool cin;
    bool operator==(const BalanceKey& o) const {
        return m == o.m && n == o.n && k == o.k && bm == o.bm && bn == o.bn && nbatch == o.nbatch &&
               flags == o.flags && cin == o.cin;
    }
};
struct BalanceKeyHash {
    size_t operator()(const BalanceKey& x) const {
        size_t h = (size_t)x.m * 1000003u ^ (size_t)x.n * 999983u ^ (size_t)x.k * 998244353u;
        return h ^ ((size_t)x.flags << 40) ^ ((size_t)x.bm << 48) ^ ((size_t)x.bn << 52) ^
               ((size_t)x.nbatch << 56) ^ (size_t)x.cin;
    }
};
struct BalanceVal {
    int xsplit[9];
};
std::mutex g_balance_mu;
std::unordered_map<BalanceKey, BalanceVal, BalanceKeyHash> g_balance_cache;

template <class T, int BM, int BN>
int balance_xcds(GemmDescT<T>& d, int tiles_m, int tiles_n) {
    const unsigned fl = d.flags;
    const int ntile = tiles_m * tiles_n;
    d.xbal = 0;
    if (!(fl & (kCUpperTiles | kAUpper | kALower | kBUpper | kBLower)) || ntile < 4 * kNumXcd) return ntile;
    const BalanceKey key{d.m, d.n, d.k, BM, BN, d.reduce ? d.batch : 1, fl, d.Cin != nullptr && d.beta != 0.0};
    {
        std::lock_guard<std::mutex> lock(g_balance_mu);
        auto it = g_balance_cache.find(key);
        if (it != g_balance_cache.end()) {
            int longest = 0;
            for (int i = 0; i < kNumXcd; ++i) {
                d.xsplit[i] = it->second.xsplit[i];
                longest = std::max(longest, it->second.xsplit[i + 1] - it->second.xsplit[i]);
            }
            d.xsplit[kNumXcd] = it->second.xsplit[kNumXcd];
            d.xbal = 1;
            return kNumXcd * longest;
        }
    }
    const long long nbatch = d.reduce ? d.batch : 1;
    const long long c0 = 4 + ((d.Cin && d.beta != 0.0) ? 4 : 0);
    const int in_group = kTileGroup * tiles_n;
    auto cost = [&](int lin) -> long long {
        const int first_m = (lin / in_group) * kTileGroup;
        const int gsize = std::min(tiles_m - first_m, kTileGroup);
        const int tm = first_m + (lin % in_group) % gsize, tn = (lin % in_group) / gsize;
        const int row0 = tm * BM, col0 = tn * BN;
        if ((fl & kCUpperTiles) && row0 > col0 + BN - 1) return 1;
        int kb = 0, ke = d.k;
        if (fl & kAUpper) kb = std::max(kb, row0);
        if (fl & kBLower) kb = std::max(kb, col0);
        if (fl & kALower) ke = std::min(ke, row0 + BM);
        if (fl & kBUpper) ke = std::min(ke, col0 + BN);
        const long long nk = ke > kb ? (ke - kb + kBK - 1) / kBK : 0;
        return nk * nbatch + c0;
    };
    long long total = 0;
    for (int l = 0; l < ntile; ++l) total += cost(l);
    d.xsplit[0] = 0;
    long long acc = 0;
    int x = 1;
    for (int l = 0; l < ntile && x < kNumXcd; ++l) {
        while (x < kNumXcd && acc * kNumXcd >= total * x) d.xsplit[x++] = l;
        acc += cost(l);
    }
    while (x <= kNumXcd) d.xsplit[x++] = ntile;
    int longest = 0;
    for (int i = 0; i < kNumXcd; ++i) longest = std::max(longest, d.xsplit[i + 1] - d.xsplit[i]);
    d.xbal = 1;
    {
        std::lock_guard<std::mutex> lock(g_balance_mu);
        if (g_balance_cache.size() > 4096) g_balance_cache.clear();
        BalanceVal v;
        for (int i = 0; i <= kNumXcd; ++i) v.xsplit[i] = d.xsplit[i];
        g_balance_cache[key] = v;
    }
    return kNumXcd * longest;
}

template <class T, int BM, int BN>
hipError_t launch_bm_bn(const GemmDescT<T>& desc, hipStream_t s) {
    GemmDescT<T> d = desc;
    const int gx = balance_xcds<T, BM, BN>(d, (d.m + BM - 1) / BM, (d.n + BN - 1) / BN);
    dim3 grid(gx, d.reduce ? 1 : d.batch, d.splitk > 1 ? d.splitk : d.batch2);
    const int which = (d.transa ? 2 : 0) + (d.transb ? 1 : 0);
    char name[64];
    if (stats_on()) {
        snprintf(name, sizeof(name), "%cgemm_kernel<%d,%d,%c,%c>", sizeof(T) == 8 ? 'd' : 's', BM, BN,
                 d.transa ? 'T' : 'N', d.transb ? 'T' : 'N');
    } else {
        name[0] = 0;
    }
    StatScope sc(name, s, gemm_flops(d), gemm_bytes(d));
    if (which == 0) gemm_kernel<T, BM, BN, false, false><<<grid, 256, 0, s>>>(d);
    else if (which == 1) gemm_kernel<T, BM, BN, false, true><<<grid, 256, 0, s>>>(d);
    else if (which == 2) gemm_kernel<T, BM, BN, true, false><<<grid, 256, 0, s>>>(d);
    else gemm_kernel<T, BM, BN, true, true><<<grid, 256, 0, s>>>(d);
    if (d.splitk > 1) {
        const long long total = (long long)d.m * d.n * (d.reduce ? 1 : d.batch);
        long long g = (total + 255) / 256;
        if (g > 2048) g = 2048;
        splitk_reduce_kernel<T><<<(int)g, 256, 0, s>>>(d);
    }
    sc.end();
    return hipGetLastError();
}

// FP64 GEMM on the vector units.  On gfx950 the FP64 FMA pipes outrun the
// FP64 matrix cores (measured peaks 67 and 36-40 TFLOP/s; 61 TFLOP/s for
// this kernel's inner loop with operands from LDS), so large FP64 products
// run here.  128 x 128 tiles, 256 threads, 8 x 8 outputs per thread in
// registers, operands read from LDS as 16-byte pairs (8 reads per 64 FMAs).
// Thread (tx, ty) = (tid % 16, tid / 16) owns rows 32 q + 2 tx + {0, 1} and
// columns 32 q + 2 ty + {0, 1}, q = 0..3, so the 16 lanes of a row group
// read 256 contiguous bytes.  beta * Cin seeds the accumulators and
// alpha * alpha_b scales A as it is staged, so results are stored straight
// from the k-loop (in split-K mode piece 0 carries beta * Cin).  Staging,
// tile order, structure flags and split-K follow gemm_kernel.
typedef double dpair __attribute__((ext_vector_type(2)));
constexpr int kValuBK = 8;   // k-slice: 4 staged values per operand and thread

// acc[i][j] += a[i] b[j] for one k step (a, b as 4 pairs each).
__device__ inline void fma_8x8(double (&acc)[8][8], const dpair (&a)[4], const dpair (&b)[4]) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const double ai = (i & 1) ? a[i >> 1].y : a[i >> 1].x;
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = fma(ai, (j & 1) ? b[j >> 1].y : b[j >> 1].x, acc[i][j]);
    }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256, 2) void dgemm_valu_kernel(GemmDescT<double> d) {
    constexpr int BM = 128, BN = 128, BK = kValuBK;
    constexpr int APT = BM * BK / 256, BPT = BN * BK / 256;
    __shared__ double As[2][BK][BM + kPad];
    __shared__ double Bs[2][BK][BN + kPad];

    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int tiles_m = (d.m + BM - 1) / BM, tiles_n = (d.n + BN - 1) / BN;
    const int nblocks = tiles_m * tiles_n;
    int lin;
    if (d.xbal) {
        const int x = blockIdx.x % kNumXcd, idx = blockIdx.x / kNumXcd;
        lin = d.xsplit[x] + idx;
        if (lin >= d.xsplit[x + 1]) return;
    } else {
        lin = xcd_remap(blockIdx.x, nblocks);
    }
    const int in_group = kTileGroup * tiles_n;
    const int first_m = (lin / in_group) * kTileGroup;
    const int gsize = min(tiles_m - first_m, kTileGroup);
    const int tm = first_m + (lin % in_group) % gsize;
    const int tn = (lin % in_group) / gsize;
    const int row0 = tm * BM, col0 = tn * BN;
    if ((d.flags & kCUpperTiles) && row0 > col0 + BN - 1) return;

    const unsigned fl = d.flags;
    int kb = 0, ke = d.k;
    if (fl & kAUpper) kb = max(kb, row0);
    if (fl & kBLower) kb = max(kb, col0);
    if (fl & kALower) ke = min(ke, row0 + BM);
    if (fl & kBUpper) ke = min(ke, col0 + BN);
    const int nk = ke > kb ? (ke - kb + BK - 1) / BK : 0;
    const int nbatch = d.reduce ? d.batch : 1;
    const int bfirst = d.reduce ? 0 : blockIdx.y;
    const int ntiles = nk * nbatch;
    const bool split = d.splitk > 1;
    const int z2 = split ? 0 : blockIdx.z;
    const int t_begin = split ? (int)((long long)blockIdx.z * ntiles / d.splitk) : 0;
    const int t_end = split ? (int)((long long)(blockIdx.z + 1) * ntiles / d.splitk) : ntiles;
    const int nt = t_end - t_begin;

    const int ob = d.reduce ? 0 : blockIdx.y;
    double* __restrict__ C = d.C + (long long)ob * d.strideC + (long long)z2 * d.strideC2;
    const double* Cin = d.Cin ? d.Cin + (long long)ob * d.strideCin + (long long)z2 * d.strideCin2 : nullptr;

    double acc[8][8];
    if (Cin != nullptr && d.beta != 0.0 && (!split || blockIdx.z == 0)) {
        const double beta = d.beta;
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int gi = row0 + 32 * (i >> 1) + 2 * tx + (i & 1);
                const int gj = col0 + 32 * (j >> 1) + 2 * ty + (j & 1);
                const bool ok = gi < d.m && gj < d.n;
                const double v = Cin[ok ? gi + (long long)gj * d.ldcin : 0];
                acc[i][j] = ok ? beta * v : 0.0;
            }
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[i][j] = 0.0;
    }

    // Staging.  A slice that lies inside the matrices and off the diagonal
    // of a triangular operand (the common case) loads without masks from
    // per-thread offsets fixed for the whole k-loop, so the vector units
    // spend their cycles on FMAs; edge and diagonal slices take the masked
    // path.  Both decisions are uniform over the workgroup.
    double ra[APT], rb[BPT];
    unsigned amask = 0, bmask = 0;
    double al_cur = 1;
    bool fast_cur = false;
    // Thread tid stages elements e = tid + 256 s: their offsets differ by a
    // uniform step in s (2 k-rows or 32 rows/columns of the tile).
    const long long ka = TA ? 1 : d.lda, kbs = TB ? d.ldb : 1;   // offset step per k
    const long long offa0 = TA ? (long long)(row0 + tid / BK) * d.lda + tid % BK
                               : (row0 + tid % BM) + (long long)(tid / BM) * d.lda;
    const long long offb0 = TB ? (col0 + tid % BN) + (long long)(tid / BN) * d.ldb
                               : (long long)(col0 + tid / BK) * d.ldb + tid % BK;
    const long long sa = TA ? (256 / BK) * d.lda : (256 / BM) * d.lda;
    const long long sb = TB ? (256 / BN) * d.ldb : (256 / BK) * d.ldb;
    const bool rows_in = row0 + BM <= d.m, cols_in = col0 + BN <= d.n;
    auto gload = [&](int t) {
        const int bi = t / nk;
        const int k0 = kb + (t - bi * nk) * BK;
        const int b = bfirst + bi;
        const double* __restrict__ A = d.A + (long long)b * d.strideA + (long long)z2 * d.strideA2;
        const double* __restrict__ B = d.B + (long long)b * d.strideB + (long long)z2 * d.strideB2;
        al_cur = d.alpha * (d.nalpha > 0 ? d.alphas[b] : 1.0);
        bool fast = rows_in && cols_in && k0 + BK <= ke;
        if (fl & kAUpper) fast = fast && k0 >= row0 + BM - 1;
        if (fl & kALower) fast = fast && k0 + BK - 1 <= row0;
        if (fl & kBUpper) fast = fast && k0 + BK - 1 <= col0;
        if (fl & kBLower) fast = fast && k0 >= col0 + BN - 1;
        fast_cur = fast;
        if (fast) {
            const double* __restrict__ Ak = A + (long long)k0 * ka + offa0;
            const double* __restrict__ Bk = B + (long long)k0 * kbs + offb0;
#pragma unroll
            for (int s = 0; s < APT; ++s) ra[s] = Ak[s * sa];
#pragma unroll
            for (int s = 0; s < BPT; ++s) rb[s] = Bk[s * sb];
            return;
        }
        amask = 0;
        bmask = 0;
#pragma unroll
        for (int s = 0; s < APT; ++s) {
            const int e = tid + 256 * s;
            const int i = TA ? e / BK : e % BM;
            const int kk = TA ? e % BK : e / BM;
            const int gi = row0 + i, gk = k0 + kk;
            bool ok = gi < d.m && gk < ke;
            if (fl & kAUpper) ok = ok && gk >= gi;
            if (fl & kALower) ok = ok && gk <= gi;
            const long long off = TA ? gk + (long long)gi * d.lda : gi + (long long)gk * d.lda;
            ra[s] = A[ok ? off : 0];
            amask |= ok ? (1u << s) : 0u;
        }
#pragma unroll
        for (int s = 0; s < BPT; ++s) {
            const int e = tid + 256 * s;
            const int j = TB ? e % BN : e / BK;
            const int kk = TB ? e / BN : e % BK;
            const int gj = col0 + j, gk = k0 + kk;
            bool ok = gj < d.n && gk < ke;
            if (fl & kBUpper) ok = ok && gk <= gj;
            if (fl & kBLower) ok = ok && gk >= gj;
            const long long off = TB ? gj + (long long)gk * d.ldb : gk + (long long)gj * d.ldb;
            rb[s] = B[ok ? off : 0];
            bmask |= ok ? (1u << s) : 0u;
        }
    };
    auto lstore = [&](int buf) {
        if (fast_cur) {
#pragma unroll
            for (int s = 0; s < APT; ++s) {
                const int e = tid + 256 * s;
                As[buf][TA ? e % BK : e / BM][TA ? e / BK : e % BM] = ra[s] * al_cur;
            }
#pragma unroll
            for (int s = 0; s < BPT; ++s) {
                const int e = tid + 256 * s;
                Bs[buf][TB ? e / BN : e % BK][TB ? e % BN : e / BK] = rb[s];
            }
            return;
        }
#pragma unroll
        for (int s = 0; s < APT; ++s) {
            const int e = tid + 256 * s;
            const int i = TA ? e / BK : e % BM;
            const int kk = TA ? e % BK : e / BM;
            As[buf][kk][i] = (amask >> s) & 1u ? ra[s] * al_cur : 0.0;
        }
#pragma unroll
        for (int s = 0; s < BPT; ++s) {
            const int e = tid + 256 * s;
            const int j = TB ? e % BN : e / BK;
            const int kk = TB ? e / BN : e % BK;
            Bs[buf][kk][j] = (bmask >> s) & 1u ? rb[s] : 0.0;
        }
    };

    if (nt > 0) {
        gload(t_begin);
        lstore(0);
        __syncthreads();
        if (nt > 1) gload(t_begin + 1);
        for (int u = 0; u < nt; ++u) {
            const int cur = u & 1;
            // Operands of step k+1 are read into the other register set
            // while the FMAs of step k run (the loop is kept rolled so that
            // only two sets are live).
            const double* Ak = &As[cur][0][2 * tx];
            const double* Bk = &Bs[cur][0][2 * ty];
            dpair a0[4], b0[4], a1[4], b1[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a0[q] = *reinterpret_cast<const dpair*>(Ak + 32 * q);
                b0[q] = *reinterpret_cast<const dpair*>(Bk + 32 * q);
            }
#pragma unroll 1
            for (int k = 0; k < BK; k += 2) {
                const int k1 = (k + 1) * (BM + kPad), k2 = ((k + 2) % BK) * (BM + kPad);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    a1[q] = *reinterpret_cast<const dpair*>(Ak + k1 + 32 * q);
                    b1[q] = *reinterpret_cast<const dpair*>(Bk + k1 + 32 * q);
                }
                fma_8x8(acc, a0, b0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    a0[q] = *reinterpret_cast<const dpair*>(Ak + k2 + 32 * q);
                    b0[q] = *reinterpret_cast<const dpair*>(Bk + k2 + 32 * q);
                }
                fma_8x8(acc, a1, b1);
            }
            if (u + 1 < nt) {
                lstore(cur ^ 1);
                __syncthreads();
                if (u + 2 < nt) gload(t_begin + u + 2);
            }
        }
    }

    if (split) {
        const int nout = d.reduce ? 1 : d.batch;
        double* __restrict__ Wp = d.work + ((long long)blockIdx.z * nout + ob) * ((long long)d.m * d.n);
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int gi = row0 + 32 * (i >> 1) + 2 * tx + (i & 1);
                const int gj = col0 + 32 * (j >> 1) + 2 * ty + (j & 1);
                if (gi < d.m && gj < d.n) Wp[gi + (long long)gj * d.m] = acc[i][j];
            }
        return;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int gi = row0 + 32 * (i >> 1) + 2 * tx + (i & 1);
            const int gj = col0 + 32 * (j >> 1) + 2 * ty + (j & 1);
            bool ok = gi < d.m && gj < d.n;
            if (fl & kCStoreUpper) ok = ok && gi <= gj;
            if (fl & kCStoreLower) ok = ok && gi >= gj;
            if (ok) C[gi + (long long)gj * d.ldc] = acc[i][j];
        }
}

hipError_t launch_valu(const GemmDescT<double>& desc, hipStream_t s) {
    GemmDescT<double> d = desc;
    d.prescaled = 1;
    const int gx = balance_xcds<double, 128, 128>(d, (d.m + 127) / 128, (d.n + 127) / 128);
    dim3 grid(gx, d.reduce ? 1 : d.batch, d.splitk > 1 ? d.splitk : d.batch2);
    char name[64];
    if (stats_on()) {
        snprintf(name, sizeof(name), "dgemm_valu<128,128,%c,%c>", d.transa ? 'T' : 'N', d.transb ? 'T' : 'N');
    } else {
        name[0] = 0;
    }
    StatScope sc(name, s, gemm_flops(d), gemm_bytes(d));
    const int which = (d.transa ? 2 : 0) + (d.transb ? 1 : 0);
    if (which == 0) dgemm_valu_kernel<false, false><<<grid, 256, 0, s>>>(d);
    else if (which == 1) dgemm_valu_kernel<false, true><<<grid, 256, 0, s>>>(d);
    else if (which == 2) dgemm_valu_kernel<true, false><<<grid, 256, 0, s>>>(d);
    else dgemm_valu_kernel<true, true><<<grid, 256, 0, s>>>(d);
    if (d.splitk > 1) {
        const long long total = (long long)d.m * d.n * (d.reduce ? 1 : d.batch);
        long long g = (total + 255) / 256;
        if (g > 2048) g = 2048;
        splitk_reduce_kernel<double><<<(int)g, 256, 0, s>>>(d);
    }
    sc.end();
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pipelined FP64 MFMA GEMM.  Each k-slice (BK = 16) of both operands is
// loaded by 16-byte loads into registers, stored to one of two LDS stages
// after the previous slice's MFMAs have been issued, and multiplied from
// there; the loads of the slice after next are in flight meanwhile.  Within
// a slice the fragment reads of the next 4-deep step are issued ahead of the
// current step's MFMAs.  Measured at 8192^3 on gfx950: 68 TFLOP/s (the MFMA
// loop alone, without global loads, 75).  The same kernel with the slices
// copied global -> LDS directly (global_load_lds_dwordx4, three stages)
// reached 58: the copies and their waits left the MFMA pipe idle a quarter
// of the time (MFMA busy 0.75 against 0.93 for the vendor's FP64 GEMM, and
// 6.7x its wave-cycles waiting on memory or barriers).
//
// Layouts of one operand slice (R rows of op(A), or columns of op(B), by
// BK = 16), in 16-byte chunks of two elements adjacent in memory:
//   R-layout (memory contiguous along r: A as is, B transposed): chunk
//     (r/2, k) at k * R/2 + ((r/2) ^ 8 (k & 1));
//   K-layout (memory contiguous along k: A transposed, B as is): chunk
//     (r, k/2) at r * 8 + ((k/2) ^ (r & 7)).
// The XOR terms spread the 16 lanes of an MFMA fragment read over the LDS
// banks (2-way at most); the 64 lanes of a load instruction fill 64
// consecutive chunks, reading whole 128-byte lines in both layouts.
template <int R, bool KC>
struct Lay {
    static constexpr int kChunks = R * kBK / 2;
    static constexpr int kPerWave = kChunks / 64 / 4;   // load instructions per wave and slice
    __device__ static void coords(int slot, int& r, int& kk) {
        if constexpr (!KC) {
            kk = slot / (R / 2);
            r = 2 * ((slot % (R / 2)) ^ ((kk & 1) * 8));
        } else {
            r = slot / (kBK / 2);
            kk = 2 * ((slot % (kBK / 2)) ^ (r & 7));
        }
    }
    __device__ static int offset(int r, int kk) {   // bytes
        if constexpr (!KC) return ((kk * (R / 2) + ((r >> 1) ^ ((kk & 1) * 8))) << 4) + ((r & 1) << 3);
        else return ((r * (kBK / 2) + ((kk >> 1) ^ (r & 7))) << 4) + ((kk & 1) << 3);
    }
};

// PRE: load the Cin tile before the k-loop (short k-ranges, where its
// latency would not hide behind the loop); otherwise after it.
template <int BM, int BN, bool TA, bool TB, bool PRE>
__global__ __launch_bounds__(256, 2) void dgemm_pipe_kernel(GemmDescT<double> d) {
    constexpr int BK = kBK;
    constexpr int FM = BM / 32, FN = BN / 32;
    using LA = Lay<BM, TA>;
    using LB = Lay<BN, !TB>;
    constexpr int NA = LA::kChunks * 2, NB = LB::kChunks * 2;   // doubles per slice
    // Room for three slices of A and of B: the k-loop uses two stages of
    // each, and after it the same memory holds the output tile for the
    // coalesced epilogue (the 64 x 128 tile needs the third slice's room).
    __shared__ __align__(16) double lds[3 * (NA + NB)];
    // Stage s: A slice at lds + s NA, B slice at lds + 3 NA + s NB.
    // Output tile in LDS, column-major with a padded leading dimension.
    // A tile too large for them goes out in two passes of BN / 2 columns.
    constexpr int TLD = BM + 2;
    constexpr int EC = BN * TLD <= 3 * (NA + NB) ? BN : BN / 2;   // columns per epilogue pass
    static_assert(EC * TLD <= 3 * (NA + NB), "an epilogue pass fits in the stage buffers");
    static_assert(!PRE || EC == BN, "Cin loaded before the k-loop needs a one-pass epilogue");

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * (BN / 2);
    const int tiles_m = (d.m + BM - 1) / BM, tiles_n = (d.n + BN - 1) / BN;
    const int nblocks = tiles_m * tiles_n;
    int lin;
    if (d.xbal) {
        const int x = blockIdx.x % kNumXcd, idx = blockIdx.x / kNumXcd;
        lin = d.xsplit[x] + idx;
        if (lin >= d.xsplit[x + 1]) return;
    } else {
        lin = xcd_remap(blockIdx.x, nblocks);
    }
    const int in_group = kTileGroup * tiles_n;
    const int first_m = (lin / in_group) * kTileGroup;
    const int gsize = min(tiles_m - first_m, kTileGroup);
    const int tm = first_m + (lin % in_group) % gsize;
    const int tn = (lin % in_group) / gsize;
    const int row0 = tm * BM, col0 = tn * BN;
    if ((d.flags & kCUpperTiles) && row0 > col0 + BN - 1) return;

    const unsigned fl = d.flags;
    int kb = 0, ke = d.k;
    if (fl & kAUpper) kb = max(kb, row0);
    if (fl & kBLower) kb = max(kb, col0);
    if (fl & kALower) ke = min(ke, row0 + BM);
    if (fl & kBUpper) ke = min(ke, col0 + BN);
    const int nk = ke > kb ? (ke - kb + BK - 1) / BK : 0;
    const int nbatch = d.reduce ? d.batch : 1;
    const int bfirst = d.reduce ? 0 : blockIdx.y;
    const int ntiles = nk * nbatch;
    const bool split = d.splitk > 1;
    const int z2 = split ? 0 : blockIdx.z;
    const int t_begin = split ? (int)((long long)blockIdx.z * ntiles / d.splitk) : 0;
    const int t_end = split ? (int)((long long)(blockIdx.z + 1) * ntiles / d.splitk) : ntiles;

    d4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = d4{0, 0, 0, 0};

    const int ob = d.reduce ? 0 : blockIdx.y;
    double* __restrict__ C = d.C + (long long)ob * d.strideC + (long long)z2 * d.strideC2;
    const double* Cin = d.Cin ? d.Cin + (long long)ob * d.strideCin + (long long)z2 * d.strideCin2 : nullptr;
    const double alpha = d.alpha, beta = d.beta;
    const bool use_cin = !split && Cin != nullptr && d.beta != 0.0;
    // Cin in the coalesced layout of the epilogue: in a pass over columns
    // cb .. cb + EC - 1, wave w takes columns cb + w, cb + w + 4, ..., lane l
    // its rows l, l + 64, ...; each load instruction reads one column
    // segment of 64 rows.
    constexpr int CPW = EC / 4, RPL = BM / 64;
    double cin[CPW][RPL];
    auto load_cin = [&](int cb) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < CPW; ++q)
#pragma unroll
            for (int u = 0; u < RPL; ++u) {
                const int gi = row0 + lane + 64 * u;
                const int gj = col0 + cb + wv + 4 * q;
                const bool ok = gi < d.m && gj < d.n;
                cin[q][u] = Cin[ok ? gi + (long long)gj * d.ldcin : 0];
            }
    };
    if (PRE && use_cin) load_cin(0);

    // Each lane loads 16-byte chunks (two elements adjacent in memory) of
    // the slice into registers and later stores them to its slots of the
    // LDS layout.  The dispatcher only sends launches whose chunks are all
    // 16-byte aligned and never straddle an edge of op(A) or op(B) (even
    // extents along pairs, even leading dimensions and strides), so every
    // slice issues the same loads from in-bounds addresses: rows of op(A)
    // past m (columns of op(B) past n) are clamped to the last pair (they
    // only reach outputs that are never stored), a ragged last slice is
    // shifted back to end at ke (below), and elements outside the slice's
    // k-range or the triangle of a triangular operand are set to zero in
    // registers before the store.
    constexpr int KA = LA::kPerWave, KB = LB::kPerWave;
    const int a_last = TA ? d.m - 1 : d.m - 2, b_last = TB ? d.n - 2 : d.n - 1;
    const long long ka = TA ? 1 : d.lda, kbs = TB ? d.ldb : 1;   // offset step per k
    // Per chunk: element offset of its (clamped) row or column at its k
    // within the slice, relative to the slice's first element.
    long long dA[KA], dB[KB];
#pragma unroll
    for (int q = 0; q < KA; ++q) {
        int r, kk;
        LA::coords((wv * KA + q) * 64 + lane, r, kk);
        const int gi = max(min(row0 + r, a_last), 0);
        dA[q] = TA ? kk + (long long)gi * d.lda : gi + (long long)kk * d.lda;
    }
#pragma unroll
    for (int q = 0; q < KB; ++q) {
        int r, kk;
        LB::coords((wv * KB + q) * 64 + lane, r, kk);
        const int gj = max(min(col0 + r, b_last), 0);
        dB[q] = TB ? gj + (long long)kk * d.ldb : kk + (long long)gj * d.ldb;
    }
    // Slices with k0 >= kfull_lo and k0 + BK <= kfull_hi need no zeroing:
    // inside the k-range and clear of the diagonal of a triangular operand.
    int kfull_lo = kb, kfull_hi = ke;
    if (fl & kAUpper) kfull_lo = max(kfull_lo, row0 + BM - 1);
    if (fl & kBLower) kfull_lo = max(kfull_lo, col0 + BN - 1);
    if (fl & kALower) kfull_hi = min(kfull_hi, row0 + 1);
    if (fl & kBUpper) kfull_hi = min(kfull_hi, col0 + 1);

    // Odd k with an operand contiguous along k: the pairs of the ragged last
    // slice would straddle the end of k, so that slice is taken after the
    // loop with element-wise loads (the dispatcher sends such products only
    // in launches that do not sum over the batch, so the ragged slice ends
    // the sequence of the workgroup that has it).
    const bool peel = (TA || !TB) && (ke & 1) && t_end == ntiles;
    const int t_main = peel ? t_end - 1 : t_end;   // end of the pipelined slices

    // Load slice t of the (batch, k) sequence into registers.  A ragged
    // last slice loads the last BK values of k instead (ke >= BK here), the
    // part it shares with the slice before being zeroed at the store, so
    // every load stays in bounds with no per-chunk clamp.  Slices past the
    // range reload the last one (never stored): every trip of the loop
    // issues the same loads, and the compiler's wait counts let the newer
    // register set stay in flight while the older one is stored.
    auto gload = [&](int t, dpair (&ra)[KA], dpair (&rb)[KB]) __attribute__((always_inline)) {
        t = min(t, t_main - 1);
        const int bi = t / nk;
        const int k0 = min(kb + (t - bi * nk) * BK, ke - BK);
        const int b = bfirst + bi;
        const double* __restrict__ Ak = d.A + (long long)b * d.strideA + (long long)z2 * d.strideA2 + (long long)k0 * ka;
        const double* __restrict__ Bk = d.B + (long long)b * d.strideB + (long long)z2 * d.strideB2 + (long long)k0 * kbs;
#pragma unroll
        for (int q = 0; q < KA; ++q) ra[q] = *reinterpret_cast<const dpair*>(Ak + dA[q]);
#pragma unroll
        for (int q = 0; q < KB; ++q) rb[q] = *reinterpret_cast<const dpair*>(Bk + dB[q]);
    };
    // Zero the elements of slice t that lie outside [kq, ke) (kq: the
    // slice's first k; below it only for a shifted ragged slice) or outside
    // the triangle of a triangular operand (rare: the ragged last slice and
    // the diagonal blocks), then store the slice to an LDS stage.
    auto sstore = [&](int t, dpair (&ra)[KA], dpair (&rb)[KB], double* sa, double* sb) __attribute__((always_inline)) {
        const int kq = kb + (t % nk) * BK;
        const int k0 = min(kq, ke - BK);
        if (kq < kfull_lo || kq + BK > kfull_hi) {
#pragma unroll
            for (int q = 0; q < KA; ++q)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    int r, kk;
                    LA::coords((wv * KA + q) * 64 + lane, r, kk);
                    const int gi = row0 + r + (TA ? 0 : h), gk = k0 + kk + (TA ? h : 0);
                    bool ok = gk >= kq && gk < ke;
                    if (fl & kAUpper) ok = ok && gk >= gi;
                    if (fl & kALower) ok = ok && gk <= gi;
                    ra[q][h] = ok ? ra[q][h] : 0.0;
                }
#pragma unroll
            for (int q = 0; q < KB; ++q)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    int r, kk;
                    LB::coords((wv * KB + q) * 64 + lane, r, kk);
                    const int gj = col0 + r + (TB ? h : 0), gk = k0 + kk + (TB ? 0 : h);
                    bool ok = gk >= kq && gk < ke;
                    if (fl & kBUpper) ok = ok && gk <= gj;
                    if (fl & kBLower) ok = ok && gk >= gj;
                    rb[q][h] = ok ? rb[q][h] : 0.0;
                }
        }
#pragma unroll
        for (int q = 0; q < KA; ++q) *reinterpret_cast<dpair*>(sa + 2 * ((wv * KA + q) * 64 + lane)) = ra[q];
#pragma unroll
        for (int q = 0; q < KB; ++q) *reinterpret_cast<dpair*>(sb + 2 * ((wv * KB + q) * 64 + lane)) = rb[q];
    };

    // Per-lane byte offsets of the MFMA fragments at the first 4-deep step;
    // later steps add a constant (R-layout: 4 k-rows; K-layout: 2 chunk
    // columns, with the XOR applied to the low chunk bit only... see offset).
    const int ra0 = lane & 15, kl = lane >> 4;
    // SCALE: per-batch multipliers (batch-reduced products with alphas).
    auto compute_k = [&](const double* sa, const double* sb, int t, auto scale_) __attribute__((always_inline)) {
        constexpr bool SCALE = decltype(scale_)::value;
        const char* ca = reinterpret_cast<const char*>(sa);
        const char* cb = reinterpret_cast<const char*>(sb);
        double al = 1.0;
        if (SCALE) al = d.alphas[bfirst + t / nk];
        double af[2][FM], bf[2][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) af[0][i] = *reinterpret_cast<const double*>(ca + LA::offset(wm + i * 16 + ra0, kl));
#pragma unroll
        for (int j = 0; j < FN; ++j) bf[0][j] = *reinterpret_cast<const double*>(cb + LB::offset(wn + j * 16 + ra0, kl));
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int p = s4 & 1;
            if (s4 + 1 < 4) {
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    af[p ^ 1][i] = *reinterpret_cast<const double*>(ca + LA::offset(wm + i * 16 + ra0, 4 * (s4 + 1) + kl));
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    bf[p ^ 1][j] = *reinterpret_cast<const double*>(cb + LB::offset(wn + j * 16 + ra0, 4 * (s4 + 1) + kl));
            }
            // Keep the next step's fragment reads ahead of this step's MFMAs
            // (the scheduler otherwise sinks them below the MFMAs into the
            // registers those MFMAs read, and each step waits on its reads).
            __builtin_amdgcn_sched_barrier(0);
            if (SCALE) {
#pragma unroll
                for (int i = 0; i < FM; ++i) af[p][i] *= al;
            }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = mfma_f64_16x16x4(af[p][i], bf[p][j], acc[i][j]);
        }
    };

    // Two LDS stages and two register sets.  While slice u is multiplied
    // from LDS, slice u + 1 waits in registers and slice u + 2 is loaded
    // into the other set; slice u + 1 then goes to the stage slice u - 1
    // left (every wave finished reading it before the previous barrier).
    // The barrier waits for the LDS stores only: the loads in flight belong
    // to this wave's registers.  The loop body covers two slices so that
    // both register sets are named statically; it is instantiated once with
    // and once without the per-batch scale, since a run-time choice inside
    // it made the compiler keep a second set of accumulators and copy
    // between the two sets.
    auto barrier = [&]() __attribute__((always_inline)) {
        __builtin_amdgcn_s_waitcnt(0xC07F);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };
    double* const sA0 = lds;
    double* const sA1 = lds + NA;
    double* const sB0 = lds + 3 * NA;
    double* const sB1 = lds + 3 * NA + NB;
    auto kloop_main = [&](auto scale_, int nt) __attribute__((always_inline)) {
        if (nt <= 0) return;
        dpair ra0[KA], rb0[KB], ra1[KA], rb1[KB];
        gload(t_begin, ra0, rb0);
        sstore(t_begin, ra0, rb0, sA0, sB0);
        gload(t_begin + 1, ra1, rb1);
        barrier();
        int u = 0;
        for (; u + 1 < nt; u += 2) {
            gload(t_begin + u + 2, ra0, rb0);
            compute_k(sA0, sB0, t_begin + u, scale_);
            sstore(t_begin + u + 1, ra1, rb1, sA1, sB1);
            barrier();
            gload(t_begin + u + 3, ra1, rb1);
            compute_k(sA1, sB1, t_begin + u + 1, scale_);
            if (u + 2 < nt) sstore(t_begin + u + 2, ra0, rb0, sA0, sB0);
            barrier();
        }
        if (u < nt) compute_k(sA0, sB0, t_begin + u, scale_);
    };
    // The peeled slice: element-wise loads, zero outside [k0, ke) and the
    // triangle of a triangular operand, stored straight to LDS stage 0.
    auto peel_store = [&](int t) __attribute__((always_inline)) {
        const int bi = t / nk;
        const int k0 = kb + (t - bi * nk) * BK;
        const int b = bfirst + bi;
        const double* __restrict__ A = d.A + (long long)b * d.strideA + (long long)z2 * d.strideA2;
        const double* __restrict__ B = d.B + (long long)b * d.strideB + (long long)z2 * d.strideB2;
#pragma unroll 1
        for (int q = 0; q < KA; ++q) {
            int r, kk;
            LA::coords((wv * KA + q) * 64 + lane, r, kk);
            double v[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int gi = row0 + r + (TA ? 0 : h), gk = k0 + kk + (TA ? h : 0);
                bool ok = gi < d.m && gk < ke;
                if (fl & kAUpper) ok = ok && gk >= gi;
                if (fl & kALower) ok = ok && gk <= gi;
                const long long off = TA ? gk + (long long)gi * d.lda : gi + (long long)gk * d.lda;
                const double x = A[ok ? off : 0];
                v[h] = ok ? x : 0.0;
            }
            *reinterpret_cast<dpair*>(sA0 + 2 * ((wv * KA + q) * 64 + lane)) = dpair{v[0], v[1]};
        }
#pragma unroll 1
        for (int q = 0; q < KB; ++q) {
            int r, kk;
            LB::coords((wv * KB + q) * 64 + lane, r, kk);
            double v[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int gj = col0 + r + (TB ? h : 0), gk = k0 + kk + (TB ? 0 : h);
                bool ok = gj < d.n && gk < ke;
                if (fl & kBUpper) ok = ok && gk <= gj;
                if (fl & kBLower) ok = ok && gk >= gj;
                const long long off = TB ? gj + (long long)gk * d.ldb : gk + (long long)gj * d.ldb;
                const double x = B[ok ? off : 0];
                v[h] = ok ? x : 0.0;
            }
            *reinterpret_cast<dpair*>(sB0 + 2 * ((wv * KB + q) * 64 + lane)) = dpair{v[0], v[1]};
        }
    };
    auto kloop = [&](auto scale_) __attribute__((always_inline)) {
        kloop_main(scale_, t_main - t_begin);
        if (peel) {
            barrier();   // every wave is past its reads of stage 0
            peel_store(t_main);
            barrier();
            compute_k(sA0, sB0, t_main, scale_);
        }
    };
    if (d.nalpha > 0) kloop(std::true_type{});
    else kloop(std::false_type{});

    // Split-K pieces store their partial sums as they are (m x n, column-major)
    // through the same coalesced epilogue.
    double* __restrict__ Out = C;
    long long ldo = d.ldc;
    double alo = alpha;
    unsigned sfl = fl;
    if (split) {
        const int nout = d.reduce ? 1 : d.batch;
        Out = d.work + ((long long)blockIdx.z * nout + ob) * ((long long)d.m * d.n);
        ldo = d.m;
        alo = 1.0;
        sfl = 0;
    }
    // Each element's Cin value is loaded before that element is stored (Cin
    // and C may alias).  The accumulators go through LDS (the stage buffers,
    // once every wave has finished its last slice) so that each store
    // instruction writes one column segment of 64 rows instead of sixteen
    // 4-row pieces.
#pragma unroll
    for (int cb = 0; cb < BN; cb += EC) {
        if (!PRE && use_cin) load_cin(cb);
        __syncthreads();
        if (wn >= cb && wn < cb + EC) {
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int r = wm + i * 16 + Mfma<double>::row(lane, e);
                        const int c = wn - cb + j * 16 + (lane & 15);
                        lds[c * TLD + r] = acc[i][j][e];
                    }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < CPW; ++q)
#pragma unroll
            for (int u = 0; u < RPL; ++u) {
                const int r = lane + 64 * u, c = wv + 4 * q;
                const int gi = row0 + r, gj = col0 + cb + c;
                bool ok = gi < d.m && gj < d.n;
                if (sfl & kCStoreUpper) ok = ok && gi <= gj;
                if (sfl & kCStoreLower) ok = ok && gi >= gj;
                if (ok) {
                    double v = alo * lds[c * TLD + r];
                    if (use_cin) v += beta * cin[q][u];
                    Out[gi + (long long)gj * ldo] = v;
                }
            }
    }
}

template <int BM, int BN>
hipError_t launch_pipe(const GemmDescT<double>& desc, hipStream_t s) {
    GemmDescT<double> d = desc;
    const int gx = balance_xcds<double, BM, BN>(d, (d.m + BM - 1) / BM, (d.n + BN - 1) / BN);
    dim3 grid(gx, d.reduce ? 1 : d.batch, d.splitk > 1 ? d.splitk : d.batch2);
    char name[64];
    if (stats_on()) {
        snprintf(name, sizeof(name), "dgemm_pipe<%d,%d,%c,%c>", BM, BN, d.transa ? 'T' : 'N', d.transb ? 'T' : 'N');
    } else {
        name[0] = 0;
    }
    StatScope sc(name, s, gemm_flops(d), gemm_bytes(d));
    const bool pre = d.k <= 256 && BM * BN <= 64 * 64;
    const int which = (d.transa ? 2 : 0) + (d.transb ? 1 : 0) + (pre ? 4 : 0);
    switch (which) {
        case 0: dgemm_pipe_kernel<BM, BN, false, false, false><<<grid, 256, 0, s>>>(d); break;
        case 1: dgemm_pipe_kernel<BM, BN, false, true, false><<<grid, 256, 0, s>>>(d); break;
        case 2: dgemm_pipe_kernel<BM, BN, true, false, false><<<grid, 256, 0, s>>>(d); break;
        case 3: dgemm_pipe_kernel<BM, BN, true, true, false><<<grid, 256, 0, s>>>(d); break;
        default:
            if constexpr (BM * BN <= 64 * 64) {
                if (which == 4) dgemm_pipe_kernel<BM, BN, false, false, true><<<grid, 256, 0, s>>>(d);
                else if (which == 5) dgemm_pipe_kernel<BM, BN, false, true, true><<<grid, 256, 0, s>>>(d);
                else if (which == 6) dgemm_pipe_kernel<BM, BN, true, false, true><<<grid, 256, 0, s>>>(d);
                else dgemm_pipe_kernel<BM, BN, true, true, true><<<grid, 256, 0, s>>>(d);
            }
            break;
    }
    if (d.splitk > 1) {
        const long long total = (long long)d.m * d.n * (d.reduce ? 1 : d.batch);
        long long g = (total + 255) / 256;
        if (g > 2048) g = 2048;
        splitk_reduce_kernel<double><<<(int)g, 256, 0, s>>>(d);
    }
    sc.end();
    return hipGetLastError();
}

// Run-time tile choice for the pipelined FP64 MFMA kernel.  Its tile shapes
// give bit-identical results (each output sums the same products in the same
// k order; masked terms are exact zeros), so the first calls of a shape
// class rotate through the candidates on real work, time each with events
// that are read back only once complete (no synchronisation), and later
// calls use the fastest per flop.  Split-K launches keep the static choice
// (their piece boundaries depend on the tile).  Off unless ZOLO_AUTOTUNE=1
// or zolo_autotune_enable(1): the fixed rule is as fast on the Zolo-PD
// workloads, and keeps which kernel runs independent of timing noise.
constexpr int kTuneCand = 3;  // 64 x 128, 64 x 64, 128 x 64
struct TuneKey {
    int dev, ta, tb, reduce, lm, ln, lk;
    unsigned flags;
    bool cin;
    bool operator==(const TuneKey& o) const {
        return dev == o.dev && ta == o.ta && tb == o.tb && reduce == o.reduce && lm == o.lm && ln == o.ln &&
               lk == o.lk && flags == o.flags && cin == o.cin;
    }
};
struct TuneKeyHash {
    size_t operator()(const TuneKey& x) const {
        return ((size_t)x.lm << 0) ^ ((size_t)x.ln << 6) ^ ((size_t)x.lk << 12) ^ ((size_t)x.flags << 18) ^
               ((size_t)x.ta << 26) ^ ((size_t)x.tb << 27) ^ ((size_t)x.reduce << 28) ^ ((size_t)x.cin << 29) ^
               ((size_t)x.dev << 32);
    }
};
// Timed launches per class: each candidate twice, in the order 0 1 2 2 1 0,
// so that a steady drift of the problem size along a sequence of calls (the
// shrinking trailing matrix of a factorisation) weighs on every candidate
// alike.
constexpr int kTuneSlots = 2 * kTuneCand;
constexpr int kTuneOrder[kTuneSlots] = {0, 1, 2, 2, 1, 0};
// A candidate replaces the fixed rule's choice only when it is faster per
// flop by more than this fraction (the rule is right for most classes, and
// event timings of single launches vary by a few percent).
constexpr double kTuneMargin = 0.03;
struct TuneEntry {
    int chosen = -1, launched = 0;
    bool measured[kTuneSlots] = {};
    float ms[kTuneSlots] = {};
    double flops[kTuneSlots] = {};
    hipEvent_t ev[kTuneSlots][2] = {};
};
std::mutex g_tune_mu;
std::unordered_map<TuneKey, TuneEntry, TuneKeyHash> g_tune;

std::atomic<int> g_tune_set{-1};  // zolo_autotune_enable; -1: from the environment

bool autotune_on() {
    const int v = g_tune_set.load(std::memory_order_relaxed);
    if (v >= 0) return v != 0;
    static const bool env = [] {
        const char* e = getenv("ZOLO_AUTOTUNE");
        return e && atoi(e) != 0;
    }();
    return env;
}

int ilog2(long long x) {
    int l = 0;
    while (x > 1) {
        x >>= 1;
        ++l;
    }
    return l;
}

hipError_t launch_pipe_cand(int c, const GemmDescT<double>& d, hipStream_t s) {
    if (c == 0) return launch_pipe<64, 128>(d, s);
    if (c == 1) return launch_pipe<64, 64>(d, s);
    return launch_pipe<128, 64>(d, s);
}

hipError_t dispatch_pipe_tuned(const GemmDescT<double>& d, int static_choice, hipStream_t s) {
    if (!autotune_on() || d.splitk > 1) return launch_pipe_cand(static_choice, d, s);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return launch_pipe_cand(static_choice, d, s);
    const TuneKey key{dev, d.transa, d.transb, d.reduce ? 1 : 0, ilog2(d.m), ilog2(d.n), ilog2(d.k), d.flags,
                      d.Cin != nullptr && d.beta != 0.0};
    std::lock_guard<std::mutex> lock(g_tune_mu);
    TuneEntry& e = g_tune[key];
    if (e.chosen >= 0) return launch_pipe_cand(e.chosen, d, s);
    int done = 0;
    for (int q = 0; q < e.launched; ++q) {
        if (!e.measured[q] && hipEventQuery(e.ev[q][1]) == hipSuccess &&
            hipEventElapsedTime(&e.ms[q], e.ev[q][0], e.ev[q][1]) == hipSuccess)
            e.measured[q] = true;
        done += e.measured[q] ? 1 : 0;
    }
    if (done == kTuneSlots) {
        double ms[kTuneCand] = {}, fl[kTuneCand] = {};
        for (int q = 0; q < kTuneSlots; ++q) {
            ms[kTuneOrder[q]] += e.ms[q];
            fl[kTuneOrder[q]] += e.flops[q];
        }
        double score[kTuneCand];
        for (int c = 0; c < kTuneCand; ++c) score[c] = ms[c] / (fl[c] > 0 ? fl[c] : 1.0);
        int best = static_choice;
        for (int c = 0; c < kTuneCand; ++c)
            if (score[c] < score[best] && score[c] < (1.0 - kTuneMargin) * score[static_choice]) best = c;
        e.chosen = best;
        static const bool log = [] {
            const char* v = getenv("ZOLO_AUTOTUNE_LOG");
            return v && atoi(v) != 0;
        }();
        if (log) {
            fprintf(stderr, "[zolo autotune] %c%c m~2^%d n~2^%d k~2^%d flags %u reduce %d cin %d:", d.transa ? 'T' : 'N',
                    d.transb ? 'T' : 'N', key.lm, key.ln, key.lk, key.flags, key.reduce, (int)key.cin);
            for (int q = 0; q < kTuneSlots; ++q)
                fprintf(stderr, " %d:%.3fms/%.2fGF", kTuneOrder[q], e.ms[q], e.flops[q] * 1e-9);
            fprintf(stderr, " -> %d (fixed rule %d)\n", best, static_choice);
        }
        for (int q = 0; q < kTuneSlots; ++q)
            for (int h = 0; h < 2; ++h) (void)hipEventDestroy(e.ev[q][h]);
        return launch_pipe_cand(best, d, s);
    }
    if (e.launched < kTuneSlots) {
        const int q = e.launched, c = kTuneOrder[q];
        if (hipEventCreate(&e.ev[q][0]) != hipSuccess) return launch_pipe_cand(static_choice, d, s);
        if (hipEventCreate(&e.ev[q][1]) != hipSuccess) {
            (void)hipEventDestroy(e.ev[q][0]);
            return launch_pipe_cand(static_choice, d, s);
        }
        ++e.launched;
        e.flops[q] = gemm_flops(d);
        hipError_t err = hipEventRecord(e.ev[q][0], s);
        if (err == hipSuccess) err = launch_pipe_cand(c, d, s);
        if (err == hipSuccess) err = hipEventRecord(e.ev[q][1], s);
        return err;
    }
    return launch_pipe_cand(static_choice, d, s);
}

// Kernel and tile shape for a descriptor: 0/1 = MFMA gemm_kernel with
// 64 x 64 / 64 x 128 tiles, 4 = dgemm_valu_kernel (128 x 128),
// 5/6 = dgemm_pipe_kernel with 64 x 128 / 64 x 64 tiles.  Measured on gfx950
// (FP64, TFLOP/s; gemm_kernel / vector / the pipelined kernel's earlier form
// with direct global -> LDS copies):
//   8192^3 N,N                          39.7 / 46.0 / 56.9
//   8192^3 T,N upper tiles (Gram)       37.3 / 35.3 / 52.9
//   8192^3 x 8 N,T batch-reduced        38.5 / 43.3 / 51.2
//   128 x 8064 x 8320 x 8 T,N, split 4  18.6 / 18.2 / 25.6
//   4096^3 x 8 N,N triangular A         35.6 / 35.7 / 46.7
//   8320 x 8064 x 128 x 8 N,N (k=128)   14.2 / 16.0 / 15.9
//   7936^2 x 64 x 8 T,N upper (k=64)    18.6 / 20.8 / 18.9
//   8320 x 7936 x 256 x 8 N,N (k=256)   30.5 / 36.2 / 37.9 (64 x 64 tiles: 40.5)
// (counting the nonzeros of trapezoidal operands).  The pipelined kernel as
// it stands: 8192^3 N,N 68.3, T,N 68.5, N,T 63.5; 256 x 8192 x 8256 x 8 T,N
// 65.1; 8256 x 8192 x 256 x 8 N,N with C read 50.1.  Up to k = 256 it runs
// 64 x 64 tiles, three workgroups per CU, with Cin loaded before the k-loop;
// beyond, 64 x 128 tiles.  128 x 128 tiles (one workgroup per CU) were
// slower in both the earlier and the current form.  64-row MFMA tiles of
// gemm_kernel run two workgroups per CU and beat its 128 x 128 tiles on
// every shape (35 against 40 at 8192^3).
template <class T>
int pick_tile(const GemmDescT<T>& d) {
    const long long nb = (long long)(d.reduce ? 1 : d.batch) * d.batch2;
    const long long t1 = (long long)((d.m + 63) / 64) * ((d.n + 127) / 128) * nb;
    if constexpr (sizeof(T) == 8) {
        if (d.k <= 128) {
            if (d.m >= 256 && d.n >= 256) {
                const long long t128 = (long long)((d.m + 127) / 128) * ((d.n + 127) / 128) * nb;
                if (t128 >= 512) return 4;
            }
            return 0;
        }
        // dgemm_pipe_kernel loads 16-byte pairs: they must be aligned and
        // must not straddle an edge of op(A) or op(B); with odd k and an
        // operand contiguous along k it takes the ragged last slice apart,
        // which only works when that slice ends the sequence (no sum over
        // the batch).
        const bool even_edges = (d.transa || (d.m & 1) == 0) && (!d.transb || (d.n & 1) == 0) &&
                                ((!d.transa && d.transb) || (d.k & 1) == 0 || !(d.reduce && d.batch > 1));
        const bool even_ld = (d.lda & 1) == 0 && (d.ldb & 1) == 0;
        const bool aligned = ((reinterpret_cast<uintptr_t>(d.A) | reinterpret_cast<uintptr_t>(d.B)) & 15) == 0 &&
                             ((d.strideA | d.strideB | d.strideA2 | d.strideB2) & 1) == 0;
        if (even_edges && even_ld && aligned) return (d.k > 256 && d.m >= 128 && d.n >= 128 && t1 >= 256) ? 5 : 6;
    }
    if (d.k <= 128) return 0;
    if (d.m >= 128 && d.n >= 128 && t1 >= 256) return 1;
    return 0;
}

inline void tile_dims(int t, int& bm, int& bn) {
    bm = t == 4 ? 128 : 64;
    bn = (t == 1 || t == 4 || t == 5) ? 128 : 64;
}

template <class T>
hipError_t gemm_dispatch(const GemmDescT<T>& d, hipStream_t s) {
    if (d.m <= 0 || d.n <= 0) return hipSuccess;
    if (d.batch <= 0 || d.batch2 <= 0) return hipSuccess;
    if (d.nalpha > kMaxInlineAlpha || (d.nalpha > 0 && d.nalpha < d.batch)) return hipErrorInvalidValue;
    if (d.splitk > 1 && (d.batch2 != 1 || d.work == nullptr)) return hipErrorInvalidValue;
    const int t = pick_tile(d);
    if constexpr (sizeof(T) == 8) {
        if (t == 4) return launch_valu(d, s);
        if (t == 5) return dispatch_pipe_tuned(d, 0, s);
        if (t == 6) return dispatch_pipe_tuned(d, 1, s);
    }
    switch (t) {
        case 0: return launch_bm_bn<T, 64, 64>(d, s);
        case 1: return launch_bm_bn<T, 64, 128>(d, s);
        case 2: return launch_bm_bn<T, 128, 64>(d, s);
        default: return launch_bm_bn<T, 128, 128>(d, s);
    }
}

}  // namespace

hipError_t gemm(const GemmDesc& d, hipStream_t s) { return gemm_dispatch(d, s); }
hipError_t gemm(const SGemmDesc& d, hipStream_t s) { return gemm_dispatch(d, s); }

// Split-K for long-k products with few output tiles (the block-reflector
// products W = V^T C of the structured QR: 128 x n outputs, k = m + 128).
// Measured on gfx950 over 136-1008 tiles of 64 x 64 and 64 x 128 at
// k = 8320, batch 8: one piece per tile leaves the last round of workgroups
// (2 per CU) partly empty, up to 1.6x the balanced time; four pieces are the
// fastest or within 3% of it across the whole range (more pieces add the
// partial-sum traffic, fewer leave the rounds uneven).  Below 256 tiles the
// pieces are raised to about 1024 workgroups in all.
hipError_t gemm_split(GemmDesc d, double* work, size_t work_elems, hipStream_t s) {
    d.splitk = 1;
    if (work != nullptr && d.batch2 == 1 && d.k >= 1024 && d.m > 0 && d.n > 0 && d.batch > 0 &&
        !(d.flags & kCUpperTiles)) {
        int bm, bn;
        tile_dims(pick_tile(d), bm, bn);
        const long long tiles = (long long)((d.m + bm - 1) / bm) * ((d.n + bn - 1) / bn) * (d.reduce ? 1 : d.batch);
        if (tiles < 1024) {
            long long sk = std::max(4LL, (1024 + tiles - 1) / tiles);
            sk = std::min(sk, (long long)d.k / 512);             // at least 512 of k per piece
            sk = std::min(sk, 32LL);
            const long long per = (long long)d.m * d.n * (d.reduce ? 1 : d.batch);
            if (sk * per > (long long)work_elems) sk = (long long)work_elems / per;
            if (sk > 1) {
                d.splitk = (int)sk;
                d.work = work;
            }
        }
    }
    return gemm_dispatch(d, s);
}

}  // namespace zolo

extern "C" int zolo_autotune_enable(int on) {
    zolo::g_tune_set.store(on ? 1 : 0, std::memory_order_relaxed);
    return 0;
}

extern "C" int zolo_autotune_reset(void) {
    std::lock_guard<std::mutex> lock(zolo::g_tune_mu);
    for (auto& kv : zolo::g_tune)
        if (kv.second.chosen < 0)
            for (int q = 0; q < kv.second.launched; ++q)
                for (int h = 0; h < 2; ++h) (void)hipEventDestroy(kv.second.ev[q][h]);
    zolo::g_tune.clear();
    return 0;
}
