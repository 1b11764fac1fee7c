// Structured Householder QR of the stacked matrices M_b = [Y_b; p_b I]
// ((m + n) x n, the [X; sqrt(c_{2j-1}) I] of eq. (12)) for all b at once, and
// the plain Householder QR of an m x n matrix (no identity block), on gfx950.
//
// Structure (Section 3.1 of the paper).  Reflector k pivots on row k of the
// dense block; below the pivot it touches the dense rows k+1..m-1 and the
// identity-block rows m..m+k (the identity block fills in upper triangular as
// the factorisation proceeds).  With M stored as one column-major array, a
// block of NB = 64 reflectors starting at column p0 therefore lives on the
// contiguous rows [p0, m + p0 + NB): m + NB live rows instead of the m + n - p0
// of a dense QR.  The identity rows stay below the dense rows on purpose:
// pivoting on the small rows p I first (identity block on top) loses row-wise
// backward stability when p is tiny, e.g. 1e-10 backward error at kappa = 1e8.
//
// Panel: one launch per panel factors all b together (a cooperative launch
// when a matrix takes more than one workgroup).  Each matrix gets G
// workgroups, each owning a slab of the panel's live rows.  The panel's 64
// columns are factored in leaves of 16.  For column k a workgroup applies
// reflector k-1 to the leaf's columns on its rows and, in the same pass,
// accumulates the dot products of column k (below the pivot) with the
// leaf's columns and picks up the pivot row; one cross-workgroup reduction
// of these 32 numbers gives the norm, the update coefficients of the leaf's
// remaining columns and the next column of the leaf's T (compact WY,
// Q = I - V T V^T).  At the end of a leaf one MFMA reduction and one
// exchange give V_leaf^T times the other panel columns, from which the
// panel's T is extended and the rest of the panel takes the leaf's block
// reflector.  Every reduction sums partials in a fixed order; its barrier
// waits a bounded time.  On exit the panel's top block holds V explicitly
// (unit diagonal, zeros above) and the R diagonal block is saved apart.
//
// Trailing update and Q formation are GEMMs on the MFMA kernel over the live
// rows:  W = V^T C,  W2 = T^T W,  C -= V W2  (ORGQR: T instead of T^T, last
// to first, then a panel's own columns = [I; 0] - V (T V_top^T)).  Panels
// come in pairs (blocks) and pairs of blocks (superblocks): the second panel
// is updated by the first, the second block by the first, and the rest of
// the matrix by all four panels at once with the compact-WY factor of the
// product, merged pairwise as T = [T1, -T1 V1^T V2 T2; 0, T2], so each
// trailing element is read and written once per 256 columns (stored R
// entries that sit above a later panel's diagonal are masked out of V by the
// GEMM's triangular flags).
#include "misc.hpp"
#include "stats.hpp"

#include <cstdlib>
#include <algorithm>
#include <map>
#include <mutex>

namespace zolo {
namespace {

constexpr int kNB = kPanelNB;
constexpr int kLW = 16;                  // leaf width: columns factored one exchange at a time
constexpr int kNL = kNB / kLW;           // leaves per panel
constexpr int kOther = kNB - kLW;        // panel columns outside one leaf
constexpr int kPT = 512;                 // threads per panel workgroup
constexpr int kRG = kPT / 64;            // row groups: every wave owns the leaf's columns over its rows
// Exchanges of one panel: one per column and one at the end of each leaf.
constexpr int kPanelExchanges = kNB + kNL;
static_assert(kLW * kOther == kPanelSlot, "exchange slot sized for the leaf-end sums");
// Slab rows per lane loaded together in the column sweep: two when the
// slab stays in global memory (latency of L2), one from LDS.
template <bool InLds>
constexpr int kRowUnroll = InLds ? 1 : 2;
// Resident-leaf variant (one workgroup per matrix, slab in global memory):
// while a leaf's columns are factored the leaf stays on chip, a thread's
// rows first + 512 j in registers for j < kResJ and in LDS beyond, so that
// a column's sweep touches no global memory.  It takes panels of at most
// kResRows live rows (the LDS part then holds 1024 rows x 16 columns).
constexpr int kResJ = 3;
constexpr int kResRows = 2560;
// Rows per lane step of the leaf-end MFMA reduction (loads issued together).
template <bool InLds>
constexpr int kQuadUnroll = InLds ? 2 : 16;
// Cache-policy operand of a buffer load that makes it coherent at agent
// scope (sc1 on gfx950), and the fourth word of a raw buffer resource.
constexpr int kCoherentLoad = 16;
constexpr int kBufferRsrcWord3 = 0x00020000;
// s_waitcnt immediate (gfx9 encoding) that waits for vmcnt == 0 only:
// vmcnt bits [3:0],[15:14] = 0, expcnt [6:4] = 7, lgkmcnt [11:8] = 15.
constexpr int kWaitVmcnt0 = 0x0F70;

struct PanelArgs {
    int L, nb, G, rows_per_wg;
    double* P; long long ld, sp;         // panel top-left (row p0, column p0) of matrix 0
    double* T; long long st;             // T_b, kNB x kNB column-major
    double* Rd; long long srd;           // R diagonal block out, kNB x kNB
    double* partials;                    // [batch][2][G][kPanelSlot]
    unsigned* flags;                     // [batch][G]: last exchange each workgroup published
    unsigned seq;                        // exchange x of this panel is published as seq + x + 1
    int* error_flag;
    unsigned spin_limit;
    int lds_stride;                      // leading dimension of the slab (InLds) or of the leaf's rows (Res) in LDS
};

// The workgroup's slab (rows [r0, r1) of the panel) lives either in LDS
// (InLds: loaded once, written back at the end) or stays in global memory.
// Row r of the slab, column j, is X[(r - r0) + j * xld] with X = LDS or P + r0.
// One level of the transposing butterfly: lanes with bit OFF set keep the
// upper HALF of their values, the others the lower, each adding its
// partner's copy of the kept half (compile-time indices keep h in registers).
// A wave-uniform double moved to scalar registers.
__device__ inline double uniform(double x) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <int HALF, int OFF>
__device__ inline void butterfly_step(double (&h)[16], int lane) {
    const bool upper = (lane & OFF) != 0;
#pragma unroll
    for (int j = 0; j < HALF; ++j) {
        const double keep = upper ? h[j + HALF] : h[j];
        const double send = upper ? h[j] : h[j + HALF];
        h[j] = keep + __shfl_xor(send, OFF, 64);
    }
}

// Blocked panel.  The panel's columns are factored in leaves of kLW = 16.
// Inside a leaf, column k takes one sweep over the slab's rows that applies
// reflector k-1 to the leaf's later columns and accumulates the dot products
// of column k below its pivot with the leaf's 16 columns, then one exchange
// of those 16 sums and of the pivot row's 16 entries, which give the norm,
// the update coefficients of the leaf's later columns and the next column of
// the leaf's own compact-WY factor T_s.  At the end of a leaf, one MFMA
// reduction over the rows forms W = V_s^T [V_prev, C] (V_s: the leaf's
// reflectors; V_prev: the earlier leaves'; C: the later columns of the
// panel), one exchange sums it over the workgroups, the first workgroup
// merges T = [T1, -T1 (V_prev^T V_s) T_s; 0, T_s], and every workgroup
// applies the leaf's block reflector to C:  C -= V_s (T_s^T (V_s^T C)).
// Against one sweep of all 64 columns per column, this sweeps 16 columns per
// column and the whole panel twice per leaf.
template <bool InLds, bool Res = false>
__global__ __launch_bounds__(kPT) void panel_kernel(PanelArgs a) {
    static_assert(!(InLds && Res), "the resident leaf is for slabs in global memory");
    extern __shared__ double smem[];
    __shared__ double s_T[kNB * (kNB + 1) / 2];  // upper T packed by columns: T[i][l] at l (l + 1) / 2 + i
    // Leaf-end sums W[i][q] at i * kOther + q (i: leaf column, q: other
    // column, the earlier leaves' columns first).  While a leaf's columns
    // are factored, its first kRG * kLW entries hold each wave's column sums.
    __shared__ double s_W[kLW * kOther];
    __shared__ double s_coef[kLW], s_z[kLW];
    __shared__ double s_rfl[4];          // beta, tau, scale of the latest reflector
    __shared__ double s_prow[kLW];       // Res: the pivot row of the leaf after the sweep
    double* const s_wp = s_W;
    const int g = blockIdx.x % a.G, b = blockIdx.x / a.G;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const long long ld = a.ld;
    double* __restrict__ P = a.P + b * a.sp;
    const int r0 = g * a.rows_per_wg;
    const int r1 = min(a.L, r0 + a.rows_per_wg);
    const int nb = a.nb;
    const long long xld = InLds ? a.lds_stride : ld;
    double* __restrict__ X = InLds ? smem : P + r0;
    constexpr int S = 64 * kRG;          // row stride of a lane
    const int first = r0 + 64 * wv + lane;  // this thread's rows: first + S j
    const int ldl = a.lds_stride;        // Res: LDS rows of the leaf, row first + S (kResJ + j) at 64 w + lane + S j
    double xr[Res ? kResJ : 1][kLW];     // Res: the leaf on this thread's first kResJ rows
    if (InLds) {
        for (int e = tid; e < (r1 - r0) * nb; e += kPT) {
            const int rl = e % (r1 - r0), j = e / (r1 - r0);
            X[rl + j * xld] = P[(r0 + rl) + j * ld];
        }
    }
    __syncthreads();
    unsigned* flg = a.flags + (long long)b * a.G;
    unsigned ex = 0;  // exchanges done in this panel

    // Sums cnt values of src over the matrix's workgroups into dst (LDS;
    // src may be dst).  Thread t publishes src[t], which it wrote itself or
    // which a barrier made visible.  Partials, flags and polls are
    // device-coherent (agent-scope) relaxed atomics.  A workgroup barrier
    // does not wait for outstanding global stores, so every storing wave
    // waits for its partial stores to be acknowledged (vmcnt 0) before the
    // barrier after which thread 0 raises the workgroup's flag; without that
    // wait another workgroup can see the flag and read a stale partial.  No
    // release/acquire fences: those would write back or invalidate the whole
    // L2 on every exchange.  Each workgroup has a flag of its own, set to the
    // exchange's sequence number, and thread t polls the flag of workgroup t.
    // Slots alternate between two parities: a workgroup can only rewrite a
    // slot after every other workgroup has published the exchange after the
    // one that read it.  The sums are taken in workgroup order.
    auto exchange = [&](const double* src, double* dst, int cnt) __attribute__((always_inline)) {
        if (a.G == 1) {
            if (src != dst)
                for (int t = tid; t < cnt; t += kPT) dst[t] = src[t];
            __syncthreads();
            ++ex;
            return;
        }
        double* part = a.partials + (((long long)b * 2 + (ex & 1)) * a.G + g) * kPanelSlot;
        for (int t = tid; t < cnt; t += kPT)
            __hip_atomic_store(&part[t], src[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        __syncthreads();
        const unsigned target = a.seq + ex + 1u;
        if (tid == 0) __hip_atomic_store(&flg[g], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int t = tid; t < a.G; t += kPT) {
            if (t == g) continue;
            unsigned spins = 0;
            while (__hip_atomic_load(&flg[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (++spins > a.spin_limit) {
                    atomicOr(a.error_flag, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
        // The partials are read with plain buffer loads that carry the
        // agent-coherence cache policy (sc1, what an agent-scope relaxed
        // atomic load uses): the compiler keeps atomic loads in order and
        // interleaved their uses with them, one memory round trip per load;
        // plain loads of 32 partials are all issued before the first wait.
        // The barrier after the polls orders them after the flags were seen.
        const double* pb = a.partials + ((long long)b * 2 + (ex & 1)) * a.G * kPanelSlot;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void*)pb, (short)0, 0x7fffffff, kBufferRsrcWord3);
        for (int t = tid; t < cnt; t += kPT) {
            // Thirty-two loads in flight per round (clamped index, padded
            // with +0.0, which leaves the in-order sum unchanged).
            double sum = 0.0;
            for (int gg = 0; gg < a.G; gg += 32) {
                double v[32];
#pragma unroll
                for (int u = 0; u < 32; ++u) {
                    const int gi = min(gg + u, a.G - 1);
                    v[u] = __builtin_bit_cast(
                        double, __builtin_amdgcn_raw_buffer_load_b64(rs, (gi * kPanelSlot + t) * 8, 0, kCoherentLoad));
                }
#pragma unroll
                for (int u = 0; u < 32; ++u) sum += gg + u < a.G ? v[u] : 0.0;
            }
            dst[t] = sum;
        }
        __syncthreads();
        ++ex;
    };

    // The same exchange done by wave 0 alone, for at most 64 values held one
    // per lane (no workgroup barrier: the wave's own stores are acknowledged
    // before its lane 0 raises the flag).  Returns lane l's sum over the
    // matrix's workgroups (lanes >= cnt: 0).
    auto exchange_wave = [&](double val, int cnt) __attribute__((always_inline)) -> double {
        double* part = a.partials + (((long long)b * 2 + (ex & 1)) * a.G + g) * kPanelSlot;
        if (lane < cnt) __hip_atomic_store(&part[lane], val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        const unsigned target = a.seq + ex + 1u;
        if (lane == 0) __hip_atomic_store(&flg[g], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int t = lane; t < a.G; t += 64) {
            if (t == g) continue;
            unsigned spins = 0;
            while (__hip_atomic_load(&flg[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (++spins > a.spin_limit) {
                    atomicOr(a.error_flag, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        asm volatile("" ::: "memory");  // the partials are read after the polls
        const double* pb = a.partials + ((long long)b * 2 + (ex & 1)) * a.G * kPanelSlot;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void*)pb, (short)0, 0x7fffffff, kBufferRsrcWord3);
        double sum = 0.0;
        if (lane < cnt) {
            for (int gg = 0; gg < a.G; gg += 32) {
                double v[32];
#pragma unroll
                for (int u = 0; u < 32; ++u) {
                    const int gi = min(gg + u, a.G - 1);
                    v[u] = __builtin_bit_cast(
                        double, __builtin_amdgcn_raw_buffer_load_b64(rs, (gi * kPanelSlot + lane) * 8, 0, kCoherentLoad));
                }
#pragma unroll
                for (int u = 0; u < 32; ++u) sum += gg + u < a.G ? v[u] : 0.0;
            }
        }
        return sum;
    };

    for (int c0 = 0; c0 < nb; c0 += kLW) {
        const int lw = min(kLW, nb - c0);
        if constexpr (Res) {
            // The leaf onto the chip (each thread its own rows).
#pragma unroll
            for (int j = 0; j < kResJ; ++j) {
                const int row = first + S * j;
#pragma unroll
                for (int q = 0; q < kLW; ++q)
                    xr[j][q] = row < r1 ? X[row - r0 + (c0 + min(q, lw - 1)) * xld] : 0.0;
            }
            for (int row = first + S * kResJ; row < r1; row += S) {
                const int rr = row - r0 - S * kResJ;
#pragma unroll
                for (int q = 0; q < kLW; ++q) smem[rr + q * ldl] = X[row - r0 + (c0 + min(q, lw - 1)) * xld];
            }
        }
        for (int kk = 0; kk < lw; ++kk) {
            const int k = c0 + kk;
            // Sweep: reflector k-1 (inside this leaf) on the leaf's columns
            // > k-1 (rows >= k-1) and the dot products of column k below the
            // pivot with the leaf's columns.  Each thread owns the same rows
            // in every column (r0 + 64 w + lane + 64 kRG j for wave w), so
            // that it can write column k on its rows after the exchange
            // without a barrier; per-column conditions are uniform.
            double acc[kLW], cq[kLW];
#pragma unroll
            for (int q = 0; q < kLW; ++q) {
                const double c = s_coef[q];
                acc[q] = 0.0;
                // Res: column kk too (its coefficient is ck), so that the
                // sweep leaves reflector k-1 applied to column kk in place.
                cq[q] = (kk > 0 && (Res ? q >= kk : q > kk) && q < lw) ? c : 0.0;
                if constexpr (Res) cq[q] = uniform(cq[q]);  // wave-uniform: scalar registers
            }
            const double ck = kk > 0 ? s_coef[kk] : 0.0;
            const int lo = max(r0, kk > 0 ? k - 1 : k);
            constexpr int U = kRowUnroll<InLds>;
            // Rows are taken U at a time, all their loads first, then the
            // arithmetic and the stores row by row in increasing order, so
            // each lane accumulates its rows in the same order as one at a time.
            auto load_row = [&](int row, double (&val)[kLW], double& vraw, double& xraw)
                                __attribute__((always_inline)) {
                const int rl = row >= lo && row < r1 ? row - r0 : lo - r0;
#pragma unroll
                for (int q = 0; q < kLW; ++q) val[q] = X[rl + (c0 + min(q, lw - 1)) * xld];
                vraw = kk > 0 ? X[rl + (k - 1) * xld] : 0.0;
                xraw = X[rl + k * xld];
            };
            auto finish_row = [&](int row, double (&val)[kLW], double vraw, double xraw)
                                  __attribute__((always_inline)) {
                if (row < lo || row >= r1) return;
                const int rl = row - r0;
                const double vprev = kk > 0 ? (row == k - 1 ? 1.0 : vraw) : 0.0;
                const double xk = xraw - ck * vprev;
                const double xa = row > k ? xk : 0.0;  // column k below the pivot
#pragma unroll
                for (int q = 0; q < kLW; ++q) {
                    double v = val[q] - cq[q] * vprev;  // cq = 0 leaves columns <= k as they are
                    if (q == kk) v = xk;
                    val[q] = v;
                    acc[q] += xa * v;
                }
                if (kk > 0) {
#pragma unroll
                    for (int q = 0; q < kLW; ++q)
                        if (q > kk && q < lw) X[rl + (c0 + q) * xld] = val[q];
                }
            };
            if constexpr (Res) {
                // The same arithmetic on the resident leaf, with column kk
                // updated in place; the thread that owns the pivot row
                // (always a register row) publishes it.
#pragma unroll
                for (int j = 0; j < kResJ; ++j) {
                    const int row = first + S * j;
                    if (row >= lo && row < r1) {
                        double vprev = 0.0;
                        if (kk > 0) {
                            double vr = 0.0;
#pragma unroll
                            for (int q = 0; q < kLW; ++q)
                                if (q + 1 == kk) vr = xr[j][q];
                            vprev = row == k - 1 ? 1.0 : vr;
                        }
#pragma unroll
                        for (int q = 0; q < kLW; ++q) xr[j][q] = xr[j][q] - cq[q] * vprev;
                        double xk = 0.0;
#pragma unroll
                        for (int q = 0; q < kLW; ++q)
                            if (q == kk) xk = xr[j][q];
                        const double xa = row > k ? xk : 0.0;  // column k below the pivot
#pragma unroll
                        for (int q = 0; q < kLW; ++q) acc[q] += xa * xr[j][q];
                        if (row == k) {
#pragma unroll
                            for (int q = 0; q < kLW; ++q) s_prow[q] = xr[j][q];
                        }
                    }
                }
                for (int row = first + S * kResJ; row < r1; row += S) {
                    if (row < lo) continue;
                    // LDS rows column by column (no row copy in registers).
                    const int rr = row - r0 - S * kResJ;
                    const double vprev = kk > 0 ? (row == k - 1 ? 1.0 : smem[rr + (kk - 1) * ldl]) : 0.0;
                    const double xk = smem[rr + kk * ldl] - ck * vprev;
                    const double xa = row > k ? xk : 0.0;
#pragma unroll
                    for (int q = 0; q < kLW; ++q) {
                        const double v = smem[rr + q * ldl] - cq[q] * vprev;
                        acc[q] += xa * v;
                        if (kk > 0 && q >= kk && q < lw) smem[rr + q * ldl] = v;
                    }
                }
            } else {
                for (int row = first; row < r1; row += S * U) {
                    double val[U][kLW], vraw[U], xraw[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) load_row(row + S * u, val[u], vraw[u], xraw[u]);
#pragma unroll
                    for (int u = 0; u < U; ++u) finish_row(row + S * u, val[u], vraw[u], xraw[u]);
                }
            }
            {
                // The 16 column sums of the wave in one transposing butterfly:
                // at offsets 32, 16, 8, 4 each lane keeps half of its values and
                // adds the partner's copy of that half (17 shuffles instead of
                // 16 x 6); then lane l holds value (l >> 2) & 15 summed over the
                // 16 lanes that differ in bits 2-5, and offsets 2, 1 finish it.
                static_assert(kLW == 16, "butterfly written for 16 columns per wave");
                double h[kLW];
#pragma unroll
                for (int q = 0; q < kLW; ++q) h[q] = acc[q];
                butterfly_step<8, 32>(h, lane);
                butterfly_step<4, 16>(h, lane);
                butterfly_step<2, 8>(h, lane);
                butterfly_step<1, 4>(h, lane);
                double t = h[0];
                t += __shfl_xor(t, 2, 64);
                t += __shfl_xor(t, 1, 64);
                if ((lane & 3) == 0) s_wp[wv * kLW + ((lane >> 2) & 15)] = t;
            }
            __syncthreads();
            if (wv == 0) {
                // Wave 0 alone does the column's exchange: lanes 0..15 add
                // the waves' sums in a fixed order, lanes 16..31 read back the
                // pivot row after the update if this slab holds it (zero
                // elsewhere: columns > k were stored above, columns < k are
                // unchanged and column k is recomputed).
                double val = 0.0;
                if (lane < kLW) {
                    val = s_wp[lane];
#pragma unroll
                    for (int q = 1; q < kRG; ++q) val += s_wp[q * kLW + lane];
                } else if (lane < 2 * kLW && k >= r0 && k < r1) {
                    const int q = lane - kLW, rl = k - r0;
                    double v;
                    if constexpr (Res) {
                        v = s_prow[q];
                    } else {
                        v = X[rl + (c0 + min(q, lw - 1)) * xld];
                        if (q == kk) v -= ck * (kk > 0 ? X[rl + (k - 1) * xld] : 0.0);
                    }
                    val = q < lw ? v : 0.0;
                }
                double sum = val;
                if (a.G > 1) sum = exchange_wave(val, 2 * kLW);
                // Reflector k on x = [alpha; below], beta = -sign(alpha) |x|,
                // v = [1; below / (alpha - beta)]  (no cancellation in alpha - beta).
                const double s2 = __shfl(sum, kk, 64), alpha = __shfl(sum, kLW + kk, 64);
                double beta, tau, scale;
                if (s2 == 0.0) {
                    beta = alpha;
                    tau = 0.0;
                    scale = 0.0;
                } else {
                    const double nrm = sqrt(alpha * alpha + s2);
                    beta = alpha >= 0.0 ? -nrm : nrm;
                    tau = (beta - alpha) / beta;
                    scale = 1.0 / (alpha - beta);
                }
                // v_k^T col (lane > kk) or v_lane^T v_k (lane < kk)
                const double w = __shfl(sum, kLW + (lane & (kLW - 1)), 64) + scale * sum;
                if (lane < lw && lane > kk) s_coef[lane] = tau * w;
                if (lane < kk) s_z[lane] = w;
                if (lane == 0) {
                    s_rfl[0] = beta;
                    s_rfl[1] = tau;
                    s_rfl[2] = scale;
                }
            }
            ++ex;
            __syncthreads();
            const double beta = s_rfl[0], tau = s_rfl[1], scale = s_rfl[2];
            // Column k on this thread's rows: R entry on row k-1, beta on the
            // pivot, v below (column k was not stored by the sweep; column
            // k-1 on these rows was written by this thread).
            if constexpr (Res) {
                // Column kk already holds reflector k-1's result (the sweep).
#pragma unroll
                for (int j = 0; j < kResJ; ++j) {
                    const int row = first + S * j;
                    if (row >= lo && row < r1) {
                        double x = 0.0;
#pragma unroll
                        for (int q = 0; q < kLW; ++q)
                            if (q == kk) x = xr[j][q];
                        const double nv = row == k ? beta : (row > k ? scale * x : x);
#pragma unroll
                        for (int q = 0; q < kLW; ++q)
                            if (q == kk) xr[j][q] = nv;
                    }
                }
                for (int row = first + S * kResJ; row < r1; row += S) {
                    if (row < lo) continue;
                    const int rr = row - r0 - S * kResJ;
                    const double x = smem[rr + kk * ldl];
                    smem[rr + kk * ldl] = row == k ? beta : (row > k ? scale * x : x);
                }
            } else {
                for (int row = first; row < r1; row += S) {
                    if (row < lo) continue;
                    const int rl = row - r0;
                    const double vprev = kk > 0 ? (row == k - 1 ? 1.0 : X[rl + (k - 1) * xld]) : 0.0;
                    const double x = X[rl + k * xld] - ck * vprev;
                    X[rl + k * xld] = row == k ? beta : (row > k ? scale * x : x);
                }
            }
            // Column kk of the leaf's T_s (every workgroup keeps T_s):
            // T[c0+j][k] = -tau sum_l T[c0+j][c0+l] z_l, T[k][k] = tau.
            // Thread 64 + j forms row j of T_s in every column, so it only
            // reads entries it wrote itself.
            if (tid >= 64 && tid <= 64 + kk) {
                const int j = tid - 64;
                const int base = k * (k + 1) / 2 + c0;
                if (j < kk) {
                    double s0 = 0.0, s1 = 0.0;
                    int l = j;
                    for (; l + 1 < kk; l += 2) {
                        s0 += s_T[(c0 + l) * (c0 + l + 1) / 2 + c0 + j] * s_z[l];
                        s1 += s_T[(c0 + l + 1) * (c0 + l + 2) / 2 + c0 + j] * s_z[l + 1];
                    }
                    for (; l < kk; ++l) s0 += s_T[(c0 + l) * (c0 + l + 1) / 2 + c0 + j] * s_z[l];
                    s_T[base + j] = -tau * (s0 + s1);
                } else {
                    s_T[base + kk] = tau;
                }
            }
        }
        if constexpr (Res) {
            // The leaf back to global memory (each thread its own rows).
#pragma unroll
            for (int j = 0; j < kResJ; ++j) {
                const int row = first + S * j;
                if (row < r1) {
#pragma unroll
                    for (int q = 0; q < kLW; ++q)
                        if (q < lw) X[row - r0 + (c0 + q) * xld] = xr[j][q];
                }
            }
            for (int row = first + S * kResJ; row < r1; row += S) {
                const int rr = row - r0 - S * kResJ;
#pragma unroll
                for (int q = 0; q < kLW; ++q)
                    if (q < lw) X[row - r0 + (c0 + q) * xld] = smem[rr + q * ldl];
            }
        }
        __syncthreads();  // the leaf's columns and T_s are complete

        // Leaf end: W = V_s^T [V_prev, C] over rows >= c0 (V_s is zero above
        // row c0, 1 on its diagonal).  Wave w forms the 16 x 16 block of
        // other columns 16 w .. 16 w + 15 with 16 x 16 x 4 MFMAs: lane l
        // holds V_s[row][c0 + l % 16] and Y[row][l % 16] for row = base + l / 16.
        const int nother = nb - lw;
        if (nother == 0) break;
        const int nblk = (nother + 15) / 16;
        const int rs = max(r0, c0);
        // Wave w takes block w % nblk over every nparts-th group of rows
        // (part w / nblk); the parts' blocks are added in part order.
        const int nparts = kRG / nblk;
        const int part = wv / nblk;
        d4 w4 = d4{0, 0, 0, 0};
        const int q0 = (wv % nblk) * 16;
        const int i = lane & 15;
        if (part < nparts) {
            const int cb = q0 < c0 ? q0 : q0 + lw;  // first column of the block (blocks do not straddle the leaf)
            const int ci = c0 + i, cj = cb + i;
            const bool iok = i < lw, jok = cj < nb && (q0 + i) < nother;
            constexpr int UQ = kQuadUnroll<InLds>;
            for (int base = rs + 4 * UQ * part; base < r1; base += 4 * UQ * nparts) {
                double av[UQ], bv[UQ];
#pragma unroll
                for (int u = 0; u < UQ; ++u) {
                    const int r = base + 4 * u + (lane >> 4);
                    const bool rok = r < r1;
                    const int rl = rok ? r - r0 : 0;
                    const double xa = X[rl + (iok ? ci : c0) * xld];
                    const double xb = X[rl + (jok ? cj : c0) * xld];
                    av[u] = (rok && iok && r >= ci) ? (r == ci ? 1.0 : xa) : 0.0;
                    bv[u] = (rok && jok) ? xb : 0.0;
                }
#pragma unroll
                for (int u = 0; u < UQ; ++u) w4 = mfma_f64_16x16x4(av[u], bv[u], w4);
            }
        }
        for (int pp = 0; pp < nparts; ++pp) {
            if (part == pp) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int ii = Mfma<double>::row(lane, e);
                    double& d = s_W[ii * kOther + q0 + i];
                    d = pp == 0 ? w4[e] : d + w4[e];
                }
            }
            __syncthreads();
        }
        exchange(s_W, s_W, lw * kOther);

        if (g == 0 && c0 > 0) {
            // T[0:c0, c0:c0+lw] = -T1 (V_prev^T V_s) T_s, first M = (V_prev^T V_s) T_s.
            double m[2] = {0.0, 0.0};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int t = tid + h * kPT;
                if (t < c0 * lw) {
                    const int j = t / lw, i = t % lw;
                    double s = 0.0;
                    for (int l = 0; l <= i; ++l)
                        s += s_W[l * kOther + j] * s_T[(c0 + i) * (c0 + i + 1) / 2 + c0 + l];
                    m[h] = s;
                }
            }
            __syncthreads();
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int t = tid + h * kPT;
                if (t < c0 * lw) s_W[(t % lw) * kOther + t / lw] = m[h];
            }
            __syncthreads();
            for (int t = tid; t < c0 * lw; t += kPT) {
                const int jj = t / lw, i = t % lw;
                double s = 0.0;
                for (int j = jj; j < c0; ++j) s += s_T[j * (j + 1) / 2 + jj] * s_W[i * kOther + j];
                s_T[(c0 + i) * (c0 + i + 1) / 2 + jj] = -s;
            }
        }
        const int nc = nb - c0 - lw;  // later columns of the panel
        if (nc > 0) {
            // W2 = T_s^T (V_s^T C) in place of V_s^T C, then C -= V_s W2.
            double m[2] = {0.0, 0.0};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int t = tid + h * kPT;
                if (t < lw * nc) {
                    const int i = t / nc, q = c0 + t % nc;
                    double s = 0.0;
                    for (int l = 0; l <= i; ++l)
                        s += s_T[(c0 + i) * (c0 + i + 1) / 2 + c0 + l] * s_W[l * kOther + q];
                    m[h] = s;
                }
            }
            __syncthreads();
            // W2 goes back transposed, W2[i][q] at q * kLW + i (q: column of
            // C), so that a column's 16 entries are contiguous.
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int t = tid + h * kPT;
                if (t < lw * nc) s_W[(t % nc) * kLW + t / nc] = m[h];
            }
            __syncthreads();
            for (int r = rs + tid; r < r1; r += kPT) {
                const int rl = r - r0;
                double v[kLW];
#pragma unroll
                for (int i = 0; i < kLW; ++i) {
                    const int ci = c0 + i;
                    const double x = X[rl + min(ci, nb - 1) * xld];
                    v[i] = (i < lw && r >= ci) ? (r == ci ? 1.0 : x) : 0.0;
                }
                // Sixteen columns' loads issued together.
#pragma unroll 1
                for (int q0 = 0; q0 < nc; q0 += 16) {
                    double cv[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) cv[u] = q0 + u < nc ? X[rl + (c0 + lw + q0 + u) * xld] : 0.0;
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        if (q0 + u < nc) {
                            double s = 0.0;
#pragma unroll
                            for (int i = 0; i < kLW; ++i) s += v[i] * s_W[(q0 + u) * kLW + i];
                            X[rl + (c0 + lw + q0 + u) * xld] = cv[u] - s;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    // Save the R diagonal block; make V's top block explicit (1 on the
    // diagonal, 0 above) so the GEMMs can use the stored panel as V.
    double* Rd = a.Rd + b * a.srd;
    for (int e = tid; e < kNB * kNB; e += kPT) {
        const int i = e % kNB, j = e / kNB;
        if ((i >= r0 && i < r1) || (g == 0 && i >= a.L)) {
            const bool in = i < nb && j < nb && i < a.L;
            const double v = in ? X[(i - r0) + j * xld] : 0.0;
            Rd[e] = (in && i <= j) ? v : 0.0;
            if (in && i <= j) X[(i - r0) + j * xld] = (i == j) ? 1.0 : 0.0;
        }
    }
    if (InLds) {
        __syncthreads();
        for (int e = tid; e < (r1 - r0) * nb; e += kPT) {
            const int rl = e % (r1 - r0), j = e / (r1 - r0);
            P[(r0 + rl) + j * ld] = X[rl + j * xld];
        }
    }
    if (g == 0 && tid < kNB) {
        double* Tb = a.T + b * a.st;
        for (int l = 0; l < kNB; ++l) Tb[tid + l * kNB] = (tid <= l && l < nb) ? s_T[l * (l + 1) / 2 + tid] : 0.0;
    }
}

// ORGQR panel fix-up: rows above the panel become 0 and the top block gets +I.
__global__ void orgqr_fix_kernel(int p0, int nb, double* M, long long ld, long long sm) {
    const int b = blockIdx.y;
    double* Mb = M + b * sm;
    const int total = (p0 + nb) * nb;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int i = e % (p0 + nb), j = e / (p0 + nb);
        double* p = Mb + i + (long long)(p0 + j) * ld;
        if (i < p0) *p = 0.0;
        else if (i - p0 == j) *p += 1.0;
    }
}

// M_b[0:m] = X (skipped when X is null), M_b[m:m+n] = p_b I.
__global__ void stack_init_kernel(int m, int n, const double* __restrict__ X, long long ldx,
                                  double* __restrict__ M, long long ld, long long sm, ShiftArgs piv) {
    const long long rows = (long long)m + n;
    const long long total = rows * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long j = e / rows, i = e - j * rows;
        if (i < m && X == nullptr) continue;  // dense block already in place
        const double x = i < m ? X[i + j * ldx] : 0.0;
        for (int b = 0; b < piv.batch; ++b)
            M[b * sm + i + j * ld] = i < m ? x : (i - m == j ? piv.shift[b] : 0.0);
    }
}

// R_b (n x n) from the factored M_b: off-diagonal blocks from M's upper part,
// diagonal blocks from the saved Rd, zeros below the diagonal.
__global__ void assemble_r_kernel(int n, const double* __restrict__ M, long long ld, long long sm,
                                  const double* __restrict__ Rd, long long srd_b, double* __restrict__ R,
                                  long long ldr, long long sr) {
    const int b = blockIdx.y;
    const long long total = (long long)n * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long j = e / n, i = e - j * n;
        double v = 0.0;
        if (i <= j) {
            const long long pi = i / kNB, pj = j / kNB;
            v = pi == pj ? Rd[b * srd_b + pi * kNB * kNB + (i % kNB) + (j % kNB) * kNB] : M[b * sm + i + j * ld];
        }
        R[b * sr + i + j * ldr] = v;
    }
}

struct Geometry {
    int G, rows;
    bool lds;
};

// Rows each workgroup owns when the slab stays in global memory.
constexpr int kPanelRowsTarget = 256;

// Panels of the solves of zolo_pd_batched with at most this many live rows
// take one workgroup per matrix: an ordinary launch on the solve's own
// stream, instead of a cooperative launch on the panel stream that all
// concurrent solves share.  Slower per column, but the panels of different
// solves overlap; measured on gfx950 over 512 matrices with
// n in [64, 1024], m in [n, 2n] (live rows up to 2112), 4 solves at once:
// 3.34 s with cooperative panels, 2.81 s with single-workgroup panels.
constexpr int kSinglePanelRows = 2304;

constexpr int kStaticLds = (kNB * (kNB + 1) / 2 + kLW * kOther + 5 * kLW) * 8 + 256;

int lds_limit() {
    static int v = [] {
        int dev = 0, bytes = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 0;
        if (hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
        if (hipFuncSetAttribute((const void*)panel_kernel<false, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                bytes - kStaticLds) != hipSuccess)
            return 0;
        if (hipFuncSetAttribute((const void*)panel_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                bytes - kStaticLds) != hipSuccess)
            return 0;
        return bytes;
    }();
    return v;
}

int cu_count() {
    static int v = [] {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        return cus;
    }();
    return v;
}

// Co-resident workgroups of the LDS panel kernel with an R-row slab.
int lds_coresident(int R) {
    static std::map<int, int> cache;
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(R);
    if (it != cache.end()) return it->second;
    int per_cu = 0;
    const size_t dyn = (size_t)R * kNB * sizeof(double);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)panel_kernel<true>, kPT, dyn) !=
        hipSuccess)
        per_cu = 0;
    return cache[R] = per_cu * cu_count();
}

// Co-resident workgroups of the global-memory panel kernel.
int global_coresident() {
    static int v = [] {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)panel_kernel<false>, kPT, 0) !=
            hipSuccess)
            return 0;
        return per_cu * cu_count();
    }();
    return v;
}

// At most this many workgroups share one matrix's panel: every column's
// exchange polls and sums one partial per workgroup, so beyond this the
// exchange costs more than the shorter sweep saves.  Measured on gfx950 for
// one 8256-row panel per launch (QR-type steps of degree 1 at n = 8192):
// 129 workgroups (the co-residency limit) 0.80 ms per 64-column panel, 64
// workgroups 0.61 ms, 32 workgroups 0.53 ms, 16 (global-memory slabs)
// 0.86 ms; eight panels per launch already take 31 workgroups each.
constexpr int kPanelMaxG = 32;

Geometry panel_geometry(int L, int batch) {
    // Slab in LDS when every workgroup of the launch can be resident with it.
    const int limit = lds_limit();
    if (limit > 0) {
        const int max_rows = (limit - kStaticLds) / (kNB * (int)sizeof(double));
        // Taller slabs than the LDS holds fall back to the most rows it does.
        const int rmin = std::max(64, std::min(((L + kPanelMaxG - 1) / kPanelMaxG + 15) / 16 * 16, max_rows / 16 * 16));
        for (int R = rmin; R <= max_rows; R += 16) {
            const int G = (L + R - 1) / R;
            if (G * batch <= lds_coresident(R)) {
                const int rows = (L + G - 1) / G;
                return {G, rows, true};
            }
        }
    }
    const int target = kPanelRowsTarget;
    int G = (L + target - 1) / target;
    if (G < 1) G = 1;
    int cap = global_coresident() / batch;
    if (cap < 1) cap = 1;
    if (G > cap) G = cap;
    int rows = (L + G - 1) / G;
    if (rows < 64) rows = 64;
    G = (L + rows - 1) / rows;
    return {G, rows, false};
}

inline int live_rows(int m, int e, int p0, int nb) {
    const int end = m + p0 + nb < m + e ? m + p0 + nb : m + e;
    return end - p0;
}

}  // namespace

// The most panel workgroups one launch of either variant can use (the LDS
// variant with its smallest slab packs the most per CU); sizes the buffers
// of per-workgroup partial sums and flags.
int panel_max_coresident() {
    int v = global_coresident();
    if (lds_limit() > 0) v = std::max(v, lds_coresident(64));
    return v;
}

hipError_t stack_init(int m, int n, const double* X, long long ldx, double* M, long long ld, long long sm,
                      const double* pivots, int batch, hipStream_t st) {
    if (batch > kMaxInlineAlpha) return hipErrorInvalidValue;
    ShiftArgs piv;
    piv.batch = batch;
    for (int b = 0; b < batch; ++b) piv.shift[b] = pivots[b];
    const long long total = ((long long)m + n) * n;
    long long grid = (total + 255) / 256;
    if (grid > 8192) grid = 8192;
    stack_init_kernel<<<(int)grid, 256, 0, st>>>(m, n, X, ldx, M, ld, sm, piv);
    return hipGetLastError();
}

hipError_t assemble_r(int n, const double* M, long long ld, long long sm, int batch, const QrWork& w, double* R,
                      long long ldr, long long sr, hipStream_t st) {
    const int npanels = (n + kNB - 1) / kNB;
    long long grid = ((long long)n * n + 255) / 256;
    if (grid > 4096) grid = 4096;
    assemble_r_kernel<<<dim3((int)grid, batch), 256, 0, st>>>(n, M, ld, sm, w.Rd, (long long)npanels * kNB * kNB,
                                                             R, ldr, sr);
    return hipGetLastError();
}

namespace {

// Cooperative launch of the panel kernel for panel p (columns p0 .. p0+nb-1).
hipError_t run_panel(int m, int e, int p, int nb, double* M, long long ld, long long sm, int batch, const QrWork& w,
                     long long stT, hipStream_t st) {
    const int p0 = p * kNB;
    const int L = live_rows(m, e, p0, nb);
    Geometry geo = panel_geometry(L, batch);
    if (geo.G > 1 && w.single_panels && L <= kSinglePanelRows) {
        const int limit = lds_limit();
        const int max_rows = limit > 0 ? (limit - kStaticLds) / (kNB * (int)sizeof(double)) : 0;
        geo = {1, L, L <= max_rows};
    }
    // The partial-sum and flag buffers hold max_coresident workgroups.
    if ((long long)geo.G * batch > w.max_coresident && geo.G > 1) return hipErrorInvalidValue;
    PanelArgs pa;
    pa.L = L; pa.nb = nb; pa.G = geo.G; pa.rows_per_wg = geo.rows;
    pa.P = M + p0 + (long long)p0 * ld; pa.ld = ld; pa.sp = sm;
    pa.T = w.T + (long long)p * kNB * kNB; pa.st = stT;
    pa.Rd = w.Rd + (long long)p * kNB * kNB; pa.srd = stT;
    pa.partials = w.partials;
    pa.flags = w.flags;
    pa.seq = (unsigned)p * kPanelExchanges;
    pa.error_flag = w.error_flag;
    pa.spin_limit = 1u << 24;
    pa.lds_stride = geo.rows;
    void* args[] = {&pa};
    hipError_t err;
    if (geo.G == 1) {
        // One workgroup per matrix needs no co-residency: an ordinary launch
        // on the solve's own stream, free to overlap other solves.  A slab
        // that the LDS does not hold keeps each leaf on chip while it is
        // factored when it has at most kResRows rows.
        const bool res = !geo.lds && L <= kResRows && lds_limit() > 0;
        const int res_rows = std::max(L - kPT * kResJ, 0);
        if (res) pa.lds_stride = std::max(res_rows, 1);
        StatScope sc(geo.lds ? "panel_kernel<lds>" : (res ? "panel_kernel<resident>" : "panel_kernel<global>"), st,
                     4.0 * L * (double)nb * nb * batch, 16.0 * L * (double)nb * batch);
        if (geo.lds)
            panel_kernel<true><<<batch, kPT, (size_t)geo.rows * kNB * sizeof(double), st>>>(pa);
        else if (res)
            panel_kernel<false, true><<<batch, kPT, (size_t)res_rows * kLW * sizeof(double), st>>>(pa);
        else
            panel_kernel<false><<<batch, kPT, 0, st>>>(pa);
        sc.end();
        return hipGetLastError();
    }
    // Several solves at once (zolo_pd_batched): every cooperative panel goes
    // to one shared stream, so two panels never wait for each other's
    // workgroups to become resident; events order it against this solve.
    hipStream_t ps = st;
    if (w.panel_stream && w.panel_stream != st) {
        ps = w.panel_stream;
        if ((err = hipEventRecord(w.ev_ready, st)) != hipSuccess) return err;
        if ((err = hipStreamWaitEvent(ps, w.ev_ready, 0)) != hipSuccess) return err;
    }
    StatScope sc(geo.lds ? "panel_kernel<lds>" : "panel_kernel<global>", ps, 4.0 * L * (double)nb * nb * batch,
                 16.0 * L * (double)nb * batch);
    if (geo.lds)
        err = hipLaunchCooperativeKernel((const void*)panel_kernel<true>, dim3(pa.G * batch), dim3(kPT), args,
                                         (size_t)geo.rows * kNB * sizeof(double), ps);
    else
        err = hipLaunchCooperativeKernel((const void*)panel_kernel<false>, dim3(pa.G * batch), dim3(kPT), args, 0, ps);
    sc.end();
    if (err == hipSuccess && ps != st) {
        if ((err = hipEventRecord(w.ev_done, ps)) != hipSuccess) return err;
        err = hipStreamWaitEvent(st, w.ev_done, 0);
    }
    return err;
}

// Applies the block reflector I - V T V^T (forward: its transpose, as in the
// factorisation; backward: itself, as in forming Q) of the nbv columns of V
// starting at column c0 to `trail` columns C starting at column c0 + nbv, over
// the live rows [c0, c0 + L).  T (ld ldt, batch stride stt) is upper
// triangular.  V's zeros above its unit diagonal, including an R block stored
// there by an earlier panel of the same block, are masked by the GEMM's
// triangular flags.  col_off skips that many columns of C first.
hipError_t apply_block(int L, int c0, int nbv, int trail, const double* Tm, long long ldt, long long stt,
                       bool transpose_t, double* M, long long ld, long long sm, int batch, const QrWork& w,
                       hipStream_t st, int col_off = 0) {
    if (trail <= 0) return hipSuccess;
    const double* V = M + c0 + (long long)c0 * ld;
    double* C = M + c0 + (long long)(c0 + nbv + col_off) * ld;
    const long long sw = (long long)kQrSuper * trail;
    GemmDesc g1;  // W = V^T C
    g1.m = nbv; g1.n = trail; g1.k = L; g1.transa = 1;
    g1.A = V; g1.lda = ld; g1.strideA = sm;
    g1.B = C; g1.ldb = ld; g1.strideB = sm;
    g1.C = w.W; g1.ldc = kQrSuper; g1.strideC = sw;
    g1.batch = batch; g1.flags = kAUpper;
    hipError_t err = gemm_split(g1, w.splitk, w.splitk_elems, st);
    if (err != hipSuccess) return err;
    GemmDesc g2;  // W2 = T^T W (forward) or T W (backward)
    g2.m = nbv; g2.n = trail; g2.k = nbv; g2.transa = transpose_t ? 1 : 0;
    g2.A = Tm; g2.lda = ldt; g2.strideA = stt;
    g2.B = w.W; g2.ldb = kQrSuper; g2.strideB = sw;
    g2.C = w.W2; g2.ldc = kQrSuper; g2.strideC = sw;
    g2.batch = batch; g2.flags = transpose_t ? kALower : kAUpper;
    if ((err = gemm(g2, st)) != hipSuccess) return err;
    GemmDesc g3;  // C -= V W2
    g3.m = L; g3.n = trail; g3.k = nbv;
    g3.A = V; g3.lda = ld; g3.strideA = sm;
    g3.B = w.W2; g3.ldb = kQrSuper; g3.strideB = sw;
    g3.Cin = C; g3.ldcin = ld; g3.strideCin = sm;
    g3.C = C; g3.ldc = ld; g3.strideC = sm;
    g3.alpha = -1.0; g3.beta = 1.0; g3.batch = batch; g3.flags = kALower;
    return gemm(g3, st);
}

// To = [T1, -T1 (V1^T V2) T2; 0, T2]: the compact-WY factor of the product
// of the block reflectors of columns [c1, c1 + n1) (factor T1) and
// [c2, c2 + n2), c2 = c1 + n1 (factor T2).  The T12 block is written by the
// GEMMs before this kernel; the rest is copied or zeroed here.
__global__ void assemble_wy_kernel(int n1, int n2, const double* __restrict__ T1, long long ld1, long long st1,
                                   const double* __restrict__ T2, long long ld2, long long st2,
                                   double* __restrict__ To, long long ldo, long long sto) {
    const int b = blockIdx.y, nt = n1 + n2;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nt * nt; e += gridDim.x * blockDim.x) {
        const int i = e % nt, j = e / nt;
        if (i < n1 && j >= n1) continue;  // T12
        double v = 0.0;
        if (i < n1 && j < n1) v = T1[b * st1 + i + (long long)j * ld1];
        else if (i >= n1 && j >= n1) v = T2[b * st2 + (i - n1) + (long long)(j - n1) * ld2];
        To[b * sto + i + (long long)j * ldo] = v;
    }
}

hipError_t merge_wy(int m, int e, int c1, int n1, const double* T1, long long ld1, long long st1, int n2,
                    const double* T2, long long ld2, long long st2, double* M, long long ld, long long sm, int batch,
                    const QrWork& w, double* To, long long ldo, long long sto, hipStream_t st) {
    const int c2 = c1 + n1;
    const int k = live_rows(m, e, c1, n1) - n1;  // rows [c2, end of V1's live rows): V1 is zero below
    const long long ss = (long long)kQrBlock * kQrBlock;
    double* P = w.S;
    double* Y = w.S + (long long)batch * ss;
    GemmDesc g;  // P = V1^T V2 (n1 x n2); V2's part above its diagonal (zeros, or R of an
                 // earlier panel of its block) is masked
    g.m = n1; g.n = n2; g.k = k; g.transa = 1;
    g.A = M + c2 + (long long)c1 * ld; g.lda = ld; g.strideA = sm;
    g.B = M + c2 + (long long)c2 * ld; g.ldb = ld; g.strideB = sm;
    g.C = P; g.ldc = kQrBlock; g.strideC = ss;
    g.batch = batch; g.flags = kBLower;
    hipError_t err = gemm_split(g, w.splitk, w.splitk_elems, st);
    if (err != hipSuccess) return err;
    GemmDesc y;  // Y = P T2 (T2 upper)
    y.m = n1; y.n = n2; y.k = n2;
    y.A = P; y.lda = kQrBlock; y.strideA = ss;
    y.B = T2; y.ldb = ld2; y.strideB = st2;
    y.C = Y; y.ldc = kQrBlock; y.strideC = ss;
    y.batch = batch; y.flags = kBUpper;
    if ((err = gemm(y, st)) != hipSuccess) return err;
    GemmDesc t;  // T12 = -T1 Y (T1 upper) into To[0:n1, n1:n1+n2]
    t.m = n1; t.n = n2; t.k = n1;
    t.A = T1; t.lda = ld1; t.strideA = st1;
    t.B = Y; t.ldb = kQrBlock; t.strideB = ss;
    t.C = To + (long long)n1 * ldo; t.ldc = ldo; t.strideC = sto;
    t.alpha = -1.0; t.batch = batch; t.flags = kAUpper;
    if ((err = gemm(t, st)) != hipSuccess) return err;
    assemble_wy_kernel<<<dim3(16, batch), 256, 0, st>>>(n1, n2, T1, ld1, st1, T2, ld2, st2, To, ldo, sto);
    return hipGetLastError();
}

}  // namespace

// Panels of 64 columns, paired into 128-column blocks (factor Tb), paired
// into 256-column superblocks (factor Ts).  Inside a superblock each block's
// reflectors update the superblock's remaining columns; the rest of the
// matrix takes one rank-256 block-reflector update per superblock, so the
// trailing matrix is read and written once per 256 columns.  That update
// is done in two parts: the next superblock's 256 columns first, then the
// far columns.  With one matrix per launch (whose panels leave most of the
// GPU idle) and a second stream, the far part runs there while the next
// superblock's panels and inner updates proceed on the caller's stream
// (look-ahead); the next superblock's own trailing update waits for it.
// Both orders compute the same products in the same way (the same two
// column ranges), so the results do not depend on the stream.
hipError_t structured_geqrf(int m, int e, int n, double* M, long long ld, long long sm, int batch, const QrWork& w,
                            hipStream_t st) {
    if (batch > kMaxInlineAlpha || batch < 1) return hipErrorInvalidValue;
    const int npanels = (n + kNB - 1) / kNB;
    const int nblocks = (n + kQrBlock - 1) / kQrBlock;
    const int nsuper = (n + kQrSuper - 1) / kQrSuper;
    const long long stT = (long long)npanels * kNB * kNB;
    const long long stb = (long long)nblocks * kQrBlock * kQrBlock;
    const long long sts = (long long)nsuper * kQrSuper * kQrSuper;
    hipError_t err = zero_ints(reinterpret_cast<int*>(w.flags), (int)w.flag_elems, st);
    if (err != hipSuccess) return err;
    const bool lookahead = batch == 1 && !w.single_panels && w.side_stream && w.side_stream != st &&
                           w.ev_side_ready && w.ev_side_done && w.W_side && w.W2_side && w.splitk_side &&
                           (size_t)kQrSuper * n <= qr_w_elems(n, 1);
    bool side_pending = false;
    for (int Q = 0; Q < nsuper; ++Q) {
        const int s0 = Q * kQrSuper;
        const int nsq = n - s0 < kQrSuper ? n - s0 : kQrSuper, send = s0 + nsq;
        const int trail_s = n - send;
        for (int q = 2 * Q; q < 2 * Q + 2 && q < nblocks; ++q) {
            const int p0 = q * kQrBlock, p = 2 * q;
            const int nbq = n - p0 < kQrBlock ? n - p0 : kQrBlock;
            const int nb1 = nbq < kNB ? nbq : kNB, nb2 = nbq - nb1;
            const int trail_in = send - p0 - nbq;  // columns to the right inside the superblock
            const double* T1 = w.T + (long long)p * kNB * kNB;
            if ((err = run_panel(m, e, p, nb1, M, ld, sm, batch, w, stT, st)) != hipSuccess) return err;
            if (nb2 == 0) {
                err = apply_block(live_rows(m, e, p0, nb1), p0, nb1, trail_in, T1, kNB, stT, true, M, ld, sm, batch,
                                  w, st);
                if (err != hipSuccess) return err;
                continue;
            }
            err = apply_block(live_rows(m, e, p0, nb1), p0, nb1, nb2, T1, kNB, stT, true, M, ld, sm, batch, w, st);
            if (err != hipSuccess) return err;
            if ((err = run_panel(m, e, p + 1, nb2, M, ld, sm, batch, w, stT, st)) != hipSuccess) return err;
            if (trail_in <= 0 && trail_s <= 0) continue;  // no later update needs Tb
            double* Tb = w.Tb + (long long)q * kQrBlock * kQrBlock;
            err = merge_wy(m, e, p0, kNB, T1, kNB, stT, nb2, T1 + kNB * kNB, kNB, stT, M, ld, sm, batch, w, Tb,
                           kQrBlock, stb, st);
            if (err != hipSuccess) return err;
            err = apply_block(live_rows(m, e, p0, nbq), p0, nbq, trail_in, Tb, kQrBlock, stb, true, M, ld, sm, batch,
                              w, st);
            if (err != hipSuccess) return err;
        }
        if (trail_s <= 0) continue;
        // The superblock (two full blocks when anything follows it) on the rest.
        const int nB = nsq - kQrBlock;
        const double* TA = w.Tb + (long long)(2 * Q) * kQrBlock * kQrBlock;
        const double* TB = nB > kNB ? w.Tb + (long long)(2 * Q + 1) * kQrBlock * kQrBlock
                                    : w.T + (long long)(4 * Q + 2) * kNB * kNB;
        const long long ldB = nB > kNB ? kQrBlock : kNB, stB = nB > kNB ? stb : stT;
        double* Ts = w.Ts + (long long)Q * kQrSuper * kQrSuper;
        err = merge_wy(m, e, s0, kQrBlock, TA, kQrBlock, stb, nB, TB, ldB, stB, M, ld, sm, batch, w, Ts, kQrSuper, sts,
                       st);
        if (err != hipSuccess) return err;
        // Columns the far part of the previous superblock's update wrote are
        // read from here on.
        if (side_pending) {
            if ((err = hipStreamWaitEvent(st, w.ev_side_done, 0)) != hipSuccess) return err;
            side_pending = false;
        }
        const int L = live_rows(m, e, s0, nsq);
        const int ahead = trail_s < kQrSuper ? trail_s : kQrSuper;
        err = apply_block(L, s0, nsq, ahead, Ts, kQrSuper, sts, true, M, ld, sm, batch, w, st);
        if (err != hipSuccess) return err;
        const int far = trail_s - ahead;
        if (far <= 0) continue;
        // One matrix: the far part runs on the side buffers (batch 1 sizes)
        // on either stream, since its split-K depends on the buffer size.
        QrWork ws = w;
        if (batch == 1 && w.W_side && w.W2_side && w.splitk_side) {
            ws.W = w.W_side;
            ws.W2 = w.W2_side;
            ws.splitk = w.splitk_side;
            ws.splitk_elems = w.splitk_side_elems;
        }
        if (lookahead) {
            if ((err = hipEventRecord(w.ev_side_ready, st)) != hipSuccess) return err;
            if ((err = hipStreamWaitEvent(w.side_stream, w.ev_side_ready, 0)) != hipSuccess) return err;
            err = apply_block(L, s0, nsq, far, Ts, kQrSuper, sts, true, M, ld, sm, batch, ws, w.side_stream, ahead);
            if (err != hipSuccess) return err;
            if ((err = hipEventRecord(w.ev_side_done, w.side_stream)) != hipSuccess) return err;
            side_pending = true;
        } else {
            err = apply_block(L, s0, nsq, far, Ts, kQrSuper, sts, true, M, ld, sm, batch, ws, st, ahead);
            if (err != hipSuccess) return err;
        }
    }
    if (side_pending) return hipStreamWaitEvent(st, w.ev_side_done, 0);
    return hipSuccess;
}

hipError_t structured_orgqr(int m, int e, int n, double* M, long long ld, long long sm, int batch, const QrWork& w,
                            hipStream_t st) {
    const int npanels = (n + kNB - 1) / kNB;
    const int nblocks = (n + kQrBlock - 1) / kQrBlock;
    const int nsuper = (n + kQrSuper - 1) / kQrSuper;
    const long long stT = (long long)npanels * kNB * kNB;
    const long long stb = (long long)nblocks * kQrBlock * kQrBlock;
    const long long sts = (long long)nsuper * kQrSuper * kQrSuper;
    hipError_t err;
    for (int Q = nsuper - 1; Q >= 0; --Q) {
        const int s0 = Q * kQrSuper;
        const int nsq = n - s0 < kQrSuper ? n - s0 : kQrSuper, send = s0 + nsq;
        // The superblock's reflectors on the columns already formed to its right
        // (a superblock that is followed by columns holds two full blocks).
        if (n - send > 0) {
            err = apply_block(live_rows(m, e, s0, nsq), s0, nsq, n - send, w.Ts + (long long)Q * kQrSuper * kQrSuper,
                              kQrSuper, sts, false, M, ld, sm, batch, w, st);
            if (err != hipSuccess) return err;
        }
        for (int q = (2 * Q + 1 < nblocks ? 2 * Q + 1 : 2 * Q); q >= 2 * Q; --q) {
            const int p0 = q * kQrBlock;
            const int nbq = n - p0 < kQrBlock ? n - p0 : kQrBlock;
            const int trail = send - p0 - nbq;
            // The block's reflectors on the superblock's columns to its right.
            if (trail > 0) {
                if (nbq > kNB)
                    err = apply_block(live_rows(m, e, p0, nbq), p0, nbq, trail,
                                      w.Tb + (long long)q * kQrBlock * kQrBlock, kQrBlock, stb, false, M, ld, sm, batch,
                                      w, st);
                else
                    err = apply_block(live_rows(m, e, p0, nbq), p0, nbq, trail, w.T + (long long)(2 * q) * kNB * kNB,
                                      kNB, stT, false, M, ld, sm, batch, w, st);
                if (err != hipSuccess) return err;
            }
            // The block's own columns, panel by panel from the last.
            for (int p = (nbq > kNB ? 2 * q + 1 : 2 * q); p >= 2 * q; --p) {
                const int pp0 = p * kNB;
                const int nb = n - pp0 < kNB ? n - pp0 : kNB;
                const int L = live_rows(m, e, pp0, nb);
                const double* Tp = w.T + (long long)p * kNB * kNB;
                double* V = M + pp0 + (long long)pp0 * ld;
                const int inblock = p0 + nbq - pp0 - nb;
                if ((err = apply_block(L, pp0, nb, inblock, Tp, kNB, stT, false, M, ld, sm, batch, w, st)) !=
                    hipSuccess)
                    return err;
                // Panel columns: S = T V_top^T, then Q[rows, panel] = -V S (in place:
                // one tile column covers the nb <= 64 columns), then +I and zeros above.
                GemmDesc s;
                s.m = nb; s.n = nb; s.k = nb; s.transb = 1;
                s.A = Tp; s.lda = kNB; s.strideA = stT;
                s.B = V; s.ldb = ld; s.strideB = sm;
                s.C = w.S; s.ldc = kNB; s.strideC = (long long)kNB * kNB;
                s.batch = batch; s.flags = kAUpper | kBUpper;
                if ((err = gemm(s, st)) != hipSuccess) return err;
                GemmDesc qd;
                qd.m = L; qd.n = nb; qd.k = nb;
                qd.A = V; qd.lda = ld; qd.strideA = sm;
                qd.B = w.S; qd.ldb = kNB; qd.strideB = (long long)kNB * kNB;
                qd.C = V; qd.ldc = ld; qd.strideC = sm;
                qd.alpha = -1.0; qd.batch = batch;
                if ((err = gemm(qd, st)) != hipSuccess) return err;
                const int total = (pp0 + nb) * nb;
                int grid = (total + 255) / 256;
                if (grid > 1024) grid = 1024;
                orgqr_fix_kernel<<<dim3(grid, batch), 256, 0, st>>>(pp0, nb, M, ld, sm);
                if ((err = hipGetLastError()) != hipSuccess) return err;
            }
        }
    }
    return hipSuccess;
}

}  // namespace zolo
