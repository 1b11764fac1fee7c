// Plain FP64 symmetric eigensolver of Zolo-SVD (Algorithm 2: H = V diag(S) V^T
// once A = Qp H), on gfx950.  Three stages, as in the eigensolvers the paper
// builds on (Section 2.3):
//
//  1. Householder tridiagonalisation Q^T H Q = T, blocked: panels of kTB
//     columns, each column's reflector from a matrix-vector product with the
//     trailing matrix corrected by the panel's earlier reflectors (the
//     trailing matrix itself is updated once per panel by a rank-2 kTB
//     product on the matrix cores).  The matrix-vector product reads the
//     trailing matrix once per column: this stage is bound by HBM bandwidth.
//  2. Divide and conquer on T (Cuppen's method): T splits into 1 x 1 blocks
//     by removing every off-diagonal coupling (a rank-one term each); blocks
//     are merged pairwise, bottom up, each merge solving the eigenproblem of
//     D + rho z z^T: deflation, the secular equation by bisection (one
//     thread per root), Gu-Eisenstat eigenvectors, and the product of the
//     merged block's eigenvectors with that solution (matrix cores).
//  3. Back-transformation V = Q V_T with the reflectors of stage 1 in
//     blocks of kBT, on the matrix cores.
// The eigenvalues come back in descending order with matching columns.
#include "eig_dc.hpp"
#include "misc.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace zolo {
namespace {

constexpr int kTB = 32;       // tridiagonalisation panel width
constexpr int kBT = 128;      // reflectors per block of the back-transformation
constexpr int kET = 256;      // threads per workgroup
constexpr int kMaxG = 512;    // workgroups of the row-parallel kernels (partial sums)

__device__ inline double block_sum256(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Sum of the first g partials in a fixed order (every workgroup gets the same value).
__device__ inline double sum_partials(const double* p, int g, double* sh) {
    double s = 0.0;
    for (int i = threadIdx.x; i < g; i += blockDim.x) s += p[i];
    // fixed-order reduction: per-thread strided sums, then the block tree
    return block_sum256(s, sh);
}

// ---------------------------------------------------------------------------
// Stage 1.  Panel starting at column j0; column j = j0 + c.  V's columns are
// the reflectors v_{j0..j-1}, stored in A below their explicit unit (row
// j' + 1 of column j'); W holds w'_c (before the alpha_c v_c term, which
// consumers add on the fly: w_c = w'_c + alpha_c v_c).
// ---------------------------------------------------------------------------
struct TrdArgs {
    int n, j, j0, c;
    double* A; long long lda;
    double* W; long long ldw;      // n x kTB, w'_c
    double* alpha;                 // kTB: alpha_c
    double* tau;                   // n: tau_j
    double* d; double* e;          // n: diagonal, off-diagonal of T
    double* sc;                    // n: 1 / (a - beta) of each column
    double* y;                     // n: A22 v
    double* pq;                    // 2 kTB: V^T v, W'^T v
    double* partA; double* partW;  // kMaxG each
    int gA, gW;                    // partial counts written by the producers
};

// A[j:n, j] -= V[j:n, 0:c] W[j, 0:c]^T + W[j:n, 0:c] V[j, 0:c]^T, then the
// partial sums of a[j+2:n, j]^2.  First alpha_{c-1} = -tau_{c-1} (w'_{c-1}^T v_{c-1}) / 2.
__global__ __launch_bounds__(kET) void trd_update_col(TrdArgs a) {
    __shared__ double sh[4];
    __shared__ double wj[kTB], vj[kTB], al[kTB];
    const int n = a.n, j = a.j, c = a.c, j0 = a.j0;
    if (c > 0) {
        const double s = sum_partials(a.partW, a.gW, sh);
        if (threadIdx.x == 0) {
            const double t = a.tau[j - 1];
            al[c - 1] = -0.5 * t * s;
            if (blockIdx.x == 0) a.alpha[c - 1] = al[c - 1];
        }
    }
    if ((int)threadIdx.x < c - 1) al[threadIdx.x] = a.alpha[threadIdx.x];
    __syncthreads();
    if ((int)threadIdx.x < c) {
        const int q = threadIdx.x;
        const double v = a.A[j + (long long)(j0 + q) * a.lda];      // V[j, q] (1 for q = c - 1)
        vj[q] = v;
        wj[q] = a.W[j + (long long)q * a.ldw] + al[q] * v;         // W[j, q]
    }
    __syncthreads();
    double part = 0.0;
    for (int row = j + blockIdx.x * kET + threadIdx.x; row < n; row += gridDim.x * kET) {
        double x = a.A[row + (long long)j * a.lda];
        for (int q = 0; q < c; ++q) {
            const double vr = a.A[row + (long long)(j0 + q) * a.lda];
            const double wr = a.W[row + (long long)q * a.ldw] + al[q] * vr;
            x -= vr * wj[q] + wr * vj[q];
        }
        a.A[row + (long long)j * a.lda] = x;
        if (row >= j + 2) part += x * x;
    }
    part = block_sum256(part, sh);
    if (threadIdx.x == 0) a.partA[blockIdx.x] = part;
}

// The reflector of column j (beta, tau, v = [1; a[j+2:n, j] / (alpha - beta)]),
// then y_i = A[j+1:n, i]^T v for the trailing columns i > j and the 2c dots
// V^T v, W'^T v.  One wave per column; v is formed on the fly from column j.
__global__ __launch_bounds__(kET) void trd_symv(TrdArgs a) {
    __shared__ double sh[4];
    __shared__ double s_scale;
    const int n = a.n, j = a.j, c = a.c;
    const double s2 = sum_partials(a.partA, a.gA, sh);
    if (threadIdx.x == 0) {
        const double al = a.A[(j + 1) + (long long)j * a.lda];
        double beta = al, t = 0.0, scale = 0.0;
        if (s2 > 0.0) {
            const double nrm = sqrt(al * al + s2);
            beta = al >= 0.0 ? -nrm : nrm;
            t = (beta - al) / beta;
            scale = 1.0 / (al - beta);
        }
        s_scale = scale;
        if (blockIdx.x == 0) {
            a.d[j] = a.A[j + (long long)j * a.lda];
            a.e[j] = beta;
            a.tau[j] = t;
            a.sc[j] = scale;
        }
    }
    __syncthreads();
    const double scale = s_scale;
    const int lane = threadIdx.x & 63;
    const int nw = gridDim.x * (kET / 64);
    const int items = (n - j - 1) + 2 * c;
    const double* colj = a.A + (long long)j * a.lda;
    for (int it = blockIdx.x * (kET / 64) + (threadIdx.x >> 6); it < items; it += nw) {
        const double* col;
        if (it < n - j - 1) col = a.A + (long long)(j + 1 + it) * a.lda;
        else if (it - (n - j - 1) < c) col = a.A + (long long)(a.j0 + it - (n - j - 1)) * a.lda;
        else col = a.W + (long long)(it - (n - j - 1) - c) * a.ldw;
        double s = 0.0;
        for (int row = j + 1 + lane; row < n; row += 64) {
            const double v = row == j + 1 ? 1.0 : scale * colj[row];
            s += col[row] * v;
        }
        s = wave_sum(s);
        if (lane == 0) {
            if (it < n - j - 1) a.y[j + 1 + it] = s;
            else a.pq[it - (n - j - 1)] = s;
        }
    }
}

// w'_c = tau (y - V (W^T v) - W (V^T v)) on rows j+1..n-1 (W = W' + alpha V),
// v stored into A[j+1:n, j] (explicit unit), partial sums of w'^T v.
__global__ __launch_bounds__(kET) void trd_w(TrdArgs a) {
    __shared__ double sh[4];
    __shared__ double p[kTB], q[kTB], al[kTB];
    const int n = a.n, j = a.j, c = a.c, j0 = a.j0;
    if ((int)threadIdx.x < c) {
        const int t = threadIdx.x;
        al[t] = a.alpha[t];
        p[t] = a.pq[t];                              // V^T v
        q[t] = a.pq[c + t] + a.alpha[t] * a.pq[t];   // W^T v
    }
    __syncthreads();
    const double t = a.tau[j], scale = a.sc[j];
    double part = 0.0;
    for (int row = j + 1 + blockIdx.x * kET + threadIdx.x; row < n; row += gridDim.x * kET) {
        const double v = row == j + 1 ? 1.0 : scale * a.A[row + (long long)j * a.lda];
        double x = a.y[row];
        for (int k = 0; k < c; ++k) {
            const double vr = a.A[row + (long long)(j0 + k) * a.lda];
            const double wr = a.W[row + (long long)k * a.ldw] + al[k] * vr;
            x -= vr * q[k] + wr * p[k];
        }
        x *= t;
        a.W[row + (long long)c * a.ldw] = x;
        a.A[row + (long long)j * a.lda] = v;
        part += x * v;
    }
    part = block_sum256(part, sh);
    if (threadIdx.x == 0) a.partW[blockIdx.x] = part;
}

// End of a panel: alpha of its last column, then W = W' + alpha V on the
// trailing rows r0..n-1 (the operands of the rank-2 kTB update).
__global__ __launch_bounds__(kET) void trd_finish_panel(TrdArgs a, int jb, int r0) {
    __shared__ double sh[4];
    __shared__ double al[kTB];
    const double s = sum_partials(a.partW, a.gW, sh);
    if (threadIdx.x == 0) {
        al[jb - 1] = -0.5 * a.tau[a.j0 + jb - 1] * s;
        if (blockIdx.x == 0) a.alpha[jb - 1] = al[jb - 1];
    }
    if ((int)threadIdx.x < jb - 1) al[threadIdx.x] = a.alpha[threadIdx.x];
    __syncthreads();
    const long long rows = a.n - r0;
    for (long long e = blockIdx.x * (long long)kET + threadIdx.x; e < rows * jb; e += (long long)gridDim.x * kET) {
        const int q = (int)(e / rows);
        const int row = r0 + (int)(e - q * rows);
        a.W[row + (long long)q * a.ldw] += al[q] * a.A[row + (long long)(a.j0 + q) * a.lda];
    }
}

// After the reduction: d[n-1], and zeros on and above the diagonal of A so
// that the reflector blocks read as unit lower trapezoidal matrices.
__global__ void trd_cleanup(int n, double* A, long long lda, double* d) {
    if (blockIdx.x == 0 && threadIdx.x == 0) d[n - 1] = A[(n - 1) + (long long)(n - 1) * lda];
    __syncthreads();
    const long long total = (long long)n * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long col = e / n, row = e - col * n;
        if (row <= col && !(row == n - 1 && col == n - 1)) A[row + col * lda] = 0.0;
    }
}

// T factor of the reflector block starting at column j0 (nb columns):
// T[c][c] = tau_c, T[0:c, c] = -tau_c T[0:c, 0:c] S[0:c, c], S = V^T V.
__global__ void form_t(int nb, const double* S, long long lds, const double* tau, double* T, long long ldt) {
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) T[(e % nb) + (long long)(e / nb) * ldt] = 0.0;
    __syncthreads();
    for (int c = 0; c < nb; ++c) {
        const double t = tau[c];
        const int i = threadIdx.x;
        double s = 0.0;
        if (i < c)
            for (int k = i; k < c; ++k) s += T[i + (long long)k * ldt] * S[k + (long long)c * lds];
        __syncthreads();
        if (i < c) T[i + (long long)c * ldt] = -t * s;
        if (i == c) T[c + (long long)c * ldt] = t;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Stage 2.  Divide and conquer.  Level with half-width s: group g covers
// [A0, A0 + k), A0 = 2 s g, k = min(2 s, n - A0); it is a merge when
// A0 + s < n, else the block is carried unchanged.  Every block keeps its
// eigenvalues in ascending order (and its eigenvector columns to match), so
// the poles of a merge come in order by merging two sorted lists.  Per-group
// arrays live at offset A0 of length-n arrays.
// ---------------------------------------------------------------------------
struct DcArgs {
    int n, s;
    const double* e;                 // couplings
    double* D;                       // eigenvalues of the current blocks (ascending per block)
    double* Qa; double* Qb; double* U; long long ld;
    double *ds, *zs, *pole, *zp, *dval, *rc, *rs, *tau, *zh, *vals, *rho;
    int *colsrc, *src, *ri, *rj, *org, *inv, *K, *nrot;
};

__global__ void dc_init(int n, const double* d, const double* e, double* D) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) D[i] = d[i] - (i > 0 ? fabs(e[i - 1]) : 0.0) - (i + 1 < n ? fabs(e[i]) : 0.0);
}

constexpr int kScanChunk = 1024;

// One workgroup per group: the merged poles in ascending order with their z
// (from the facing rows of the two blocks), normalisation, and the
// deflation scan (thread 0, over chunks staged in LDS).
__global__ __launch_bounds__(kET) void dc_prepare(DcArgs a) {
    __shared__ double sh[4];
    __shared__ double cd[kScanChunk], cz[kScanChunk];
    const int g = blockIdx.x, s = a.s, n = a.n, A0 = 2 * s * g, k = min(2 * s, n - A0);
    if (A0 + s >= n) {
        if (threadIdx.x == 0) a.K[g] = -1;
        return;
    }
    const double beta = a.e[A0 + s - 1], sg = beta >= 0.0 ? 1.0 : -1.0;
    const double* D = a.D + A0;
    for (int c = threadIdx.x; c < k; c += kET) {
        const double x = D[c];
        int lo, hi;
        if (c < s) {             // count of the second block's values < x
            lo = s; hi = k;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (D[mid] < x) lo = mid + 1;
                else hi = mid;
            }
            lo -= s;
        } else {                 // count of the first block's values <= x
            lo = 0; hi = s;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (D[mid] <= x) lo = mid + 1;
                else hi = mid;
            }
        }
        const int pos = (c < s ? c : c - s) + lo;
        const long long col = (long long)(A0 + c) * a.ld;
        a.ds[A0 + pos] = x;
        a.zs[A0 + pos] = c < s ? a.Qa[(A0 + s - 1) + col] : sg * a.Qa[(A0 + s) + col];
        a.colsrc[A0 + pos] = c;
    }
    __syncthreads();
    double zz = 0.0, dm = 0.0;
    for (int t = threadIdx.x; t < k; t += kET) {
        const double z = a.zs[A0 + t];
        zz += z * z;
        dm = fmax(dm, fabs(a.ds[A0 + t]));
    }
    zz = block_sum256(zz, sh);
    // max over the workgroup
    for (int off = 32; off > 0; off >>= 1) dm = fmax(dm, __shfl_xor(dm, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = dm;
    __syncthreads();
    dm = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    const double zn = sqrt(zz);
    double zm = 0.0;
    for (int t = threadIdx.x; t < k; t += kET) {
        const double z = zn > 0.0 ? a.zs[A0 + t] / zn : 0.0;
        a.zs[A0 + t] = z;
        zm = fmax(zm, fabs(z));
    }
    for (int off = 32; off > 0; off >>= 1) zm = fmax(zm, __shfl_xor(zm, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = zm;
    __syncthreads();
    zm = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    const double r = fabs(beta) * zn * zn;
    dc::DeflateScan sc;
    sc.pole = a.pole + A0; sc.zp = a.zp + A0; sc.dval = a.dval + A0; sc.rc = a.rc + A0; sc.rs = a.rs + A0;
    sc.src = a.src + A0; sc.ri = a.ri + A0; sc.rj = a.rj + A0;
    sc.begin(k, r, 8.0 * dc::kEps * fmax(dm, r * zm));
    for (int c0 = 0; c0 < k; c0 += kScanChunk) {
        const int cn = min(kScanChunk, k - c0);
        __syncthreads();
        for (int t = threadIdx.x; t < cn; t += kET) {
            cd[t] = a.ds[A0 + c0 + t];
            cz[t] = a.zs[A0 + c0 + t];
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int t = 0; t < cn; ++t) sc.step(c0 + t, cd[t], cz[t]);
    }
    if (threadIdx.x == 0) {
        a.K[g] = sc.finish();
        a.nrot[g] = sc.nrot;
        a.rho[g] = r;
    }
}

// The deflating rotations on the block columns of each merge (row-parallel;
// rotation indices are sorted positions, mapped to block columns).
__global__ void dc_rotate(DcArgs a) {
    const int g = blockIdx.y, s = a.s, A0 = 2 * s * g;
    if (a.K[g] < 0) return;
    const int k = min(2 * s, a.n - A0), nr = a.nrot[g];
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < k; r += gridDim.x * blockDim.x) {
        double* row = a.Qa + (A0 + r);
        for (int t = 0; t < nr; ++t) {
            const long long ci = (long long)(A0 + a.colsrc[A0 + a.ri[A0 + t]]) * a.ld;
            const long long cj = (long long)(A0 + a.colsrc[A0 + a.rj[A0 + t]]) * a.ld;
            const double x = row[ci], y = row[cj], c = a.rc[A0 + t], sn = a.rs[A0 + t];
            row[ci] = c * x + sn * y;
            row[cj] = c * y - sn * x;
        }
    }
}

// One thread per root: bisection of the secular equation.
__global__ void dc_secular(DcArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const int g = p / (2 * a.s), A0 = 2 * a.s * g, t = p - A0, K = a.K[g];
    if (K < 0 || t >= K) return;
    int o;
    double tau;
    dc::secular_root(K, a.pole + A0, a.zp + A0, a.rho[g], t, &o, &tau);
    a.org[A0 + t] = o;
    a.tau[A0 + t] = tau;
}

// Gu-Eisenstat z and the new eigenvalues (roots, then deflated values).
__global__ void dc_lowner(DcArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const int g = p / (2 * a.s), A0 = 2 * a.s * g, t = p - A0, K = a.K[g];
    if (K < 0) {
        a.vals[p] = a.D[p];
        return;
    }
    if (t < K) {
        a.zh[p] = dc::lowner_z(K, a.pole + A0, a.zp + A0, a.rho[g], a.org + A0, a.tau + A0, t);
        a.vals[p] = a.pole[A0 + a.org[p]] + a.tau[p];
    } else {
        a.vals[p] = a.dval[p];
    }
}

// Ascending order of the new eigenvalues of each group: inv[A0 + rank] = t.
__global__ void dc_rank(DcArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const int g = p / (2 * a.s), A0 = 2 * a.s * g, t = p - A0, K = a.K[g];
    if (K < 0) {
        a.inv[p] = t;
        return;
    }
    const int k = min(2 * a.s, a.n - A0);
    const double x = a.vals[p];
    int rank = 0;
    for (int u = 0; u < k; ++u) {
        const double y = a.vals[A0 + u];
        rank += (y < x || (y == x && u < t)) ? 1 : 0;
    }
    a.inv[A0 + rank] = t;
}

// One workgroup per output column p of the group's k x k block of U, and the
// eigenvalue D[p].  Carried blocks get identity columns.
__global__ __launch_bounds__(kET) void dc_vectors(DcArgs a) {
    __shared__ double sh[4];
    const int p = blockIdx.x;
    const int g = p / (2 * a.s), A0 = 2 * a.s * g, K = a.K[g];
    const int k = min(2 * a.s, a.n - A0);
    const int t = a.inv[p];
    double* col = a.U + A0 + (long long)p * a.ld;
    for (int r = threadIdx.x; r < k; r += kET) col[r] = 0.0;
    __syncthreads();
    if (K < 0) {
        if (threadIdx.x == 0) col[t] = 1.0;
        return;
    }
    if (threadIdx.x == 0) a.D[p] = a.vals[A0 + t];
    if (t >= K) {
        if (threadIdx.x == 0) col[a.colsrc[A0 + a.src[A0 + t]]] = 1.0;
        return;
    }
    const double* pole = a.pole + A0;
    const int o = a.org[A0 + t];
    const double tau = a.tau[A0 + t];
    double sum = 0.0;
    for (int j = threadIdx.x; j < K; j += kET) {
        const double u = a.zh[A0 + j] / dc::pole_minus_root(pole, j, o, tau);
        sum += u * u;
    }
    sum = block_sum256(sum, sh);
    const double inv = 1.0 / sqrt(sum);
    for (int j = threadIdx.x; j < K; j += kET)
        col[a.colsrc[A0 + a.src[A0 + j]]] = a.zh[A0 + j] / dc::pole_minus_root(pole, j, o, tau) * inv;
}

// Qb block = Qa block * U block for groups of at most 64 columns (one
// workgroup per group; the matrix cores take the larger ones).
__global__ __launch_bounds__(kET) void dc_small_product(DcArgs a, int ngroups) {
    const int g = blockIdx.x;
    if (g >= ngroups) return;
    const int A0 = 2 * a.s * g, k = min(2 * a.s, a.n - A0);
    for (int e = threadIdx.x; e < k * k; e += kET) {
        const int r = e % k, c = e / k;
        double acc = 0.0;
        for (int q = 0; q < k; ++q)
            acc += a.Qa[(A0 + r) + (long long)(A0 + q) * a.ld] * a.U[(A0 + q) + (long long)(A0 + c) * a.ld];
        a.Qb[(A0 + r) + (long long)(A0 + c) * a.ld] = acc;
    }
}

// Vs[:, k] = V[:, perm[k]] (n x n).
__global__ void gather_columns(int n, const double* V, long long ldv, const int* perm, double* Vs, long long lds) {
    const int k = blockIdx.y;
    const int src = perm[k];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        Vs[i + (long long)k * lds] = V[i + (long long)src * ldv];
}

template <class T>
T* carve(char*& p, size_t count) {
    T* r = reinterpret_cast<T*>(p);
    p += ((count * sizeof(T) + 255) / 256) * 256;
    return r;
}

}  // namespace

size_t syevd_work_bytes(int n) {
    const size_t nn = (size_t)n * n, N = (size_t)n + 64;
    return 3 * (nn * 8 + 256) + (size_t)n * kTB * 8 + 256 + (size_t)kBT * kBT * 8 * 2 + 512 +
           20 * (N * 8 + 256) + 10 * (N * 4 + 256) + 4 * (kMaxG * 8 + 256) + 4096;
}

// Eigen-decomposition of the symmetric n x n matrix A (lower triangle used;
// A is overwritten).  w_host: eigenvalues, descending; Z (ldz): the matching
// orthonormal eigenvectors.  work: syevd_work_bytes(n) bytes of device memory.
// host: pinned buffer of at least n doubles.  Synchronises the stream.
hipError_t syevd(int n, double* A, long long lda, double* w_host, double* Z, long long ldz, char* work,
                 double* host, hipStream_t st) {
    if (n < 1) return hipErrorInvalidValue;
    char* p = work;
    const long long ld = n;
    double* Qa = carve<double>(p, (size_t)n * n);
    double* Qb = carve<double>(p, (size_t)n * n);
    double* U = carve<double>(p, (size_t)n * n);
    double* W = carve<double>(p, (size_t)n * kTB);
    double* S = carve<double>(p, (size_t)kBT * kBT);
    double* Tf = carve<double>(p, (size_t)kBT * kBT);
    const size_t N = (size_t)n + 64;
    double *d = carve<double>(p, N), *e = carve<double>(p, N), *tau = carve<double>(p, N), *sc = carve<double>(p, N);
    double *y = carve<double>(p, N), *pq = carve<double>(p, N), *alpha = carve<double>(p, N);
    double *D = carve<double>(p, N), *ds = carve<double>(p, N), *zs = carve<double>(p, N);
    double *pole = carve<double>(p, N), *zp = carve<double>(p, N), *dval = carve<double>(p, N);
    double *rc = carve<double>(p, N), *rs = carve<double>(p, N), *dtau = carve<double>(p, N);
    double *zh = carve<double>(p, N), *vals = carve<double>(p, N), *rho = carve<double>(p, N);
    int *colsrc = carve<int>(p, N), *src = carve<int>(p, N), *ri = carve<int>(p, N), *rj = carve<int>(p, N);
    int *org = carve<int>(p, N), *inv = carve<int>(p, N), *Kc = carve<int>(p, N), *nrot = carve<int>(p, N);
    int* perm = carve<int>(p, N);
    double* partA = carve<double>(p, kMaxG);
    double* partW = carve<double>(p, kMaxG);
    hipError_t err;

    // --- Stage 1: tridiagonalisation ----------------------------------------
    TrdArgs ta;
    ta.n = n; ta.A = A; ta.lda = lda; ta.W = W; ta.ldw = n; ta.alpha = alpha; ta.tau = tau;
    ta.d = d; ta.e = e; ta.sc = sc; ta.y = y; ta.pq = pq; ta.partA = partA; ta.partW = partW;
    for (int j0 = 0; j0 < n - 1; j0 += kTB) {
        const int jb = std::min(kTB, n - 1 - j0);
        ta.j0 = j0;
        for (int c = 0; c < jb; ++c) {
            const int j = j0 + c;
            ta.j = j; ta.c = c;
            const int rows = n - j;
            const int gA = std::max(1, std::min(kMaxG, (rows + kET - 1) / kET));
            ta.gA = gA;
            trd_update_col<<<gA, kET, 0, st>>>(ta);
            const int items = (n - j - 1) + 2 * c;
            const int gB = std::max(1, std::min(2048, (items + 3) / 4));
            trd_symv<<<gB, kET, 0, st>>>(ta);
            const int gW = std::max(1, std::min(kMaxG, (rows - 1 + kET - 1) / kET));
            trd_w<<<gW, kET, 0, st>>>(ta);
            ta.gW = gW;
        }
        const int r0 = j0 + jb;
        const int nt = n - r0;
        {
            const long long tot = (long long)nt * jb;
            const int g = (int)std::max(1LL, std::min<long long>(1024, (tot + kET - 1) / kET));
            trd_finish_panel<<<g, kET, 0, st>>>(ta, jb, r0);
        }
        if (nt > 0) {
            GemmDesc g1;  // A22 -= V W^T
            g1.m = nt; g1.n = nt; g1.k = jb; g1.transb = 1;
            g1.A = A + r0 + (long long)j0 * lda; g1.lda = lda;
            g1.B = W + r0; g1.ldb = n;
            g1.Cin = A + r0 + (long long)r0 * lda; g1.ldcin = lda; g1.beta = 1.0; g1.alpha = -1.0;
            g1.C = A + r0 + (long long)r0 * lda; g1.ldc = lda;
            if ((err = gemm(g1, st)) != hipSuccess) return err;
            GemmDesc g2 = g1;  // A22 -= W V^T
            g2.A = W + r0; g2.lda = n;
            g2.B = A + r0 + (long long)j0 * lda; g2.ldb = lda;
            if ((err = gemm(g2, st)) != hipSuccess) return err;
        }
    }
    trd_cleanup<<<std::max(1, std::min(2048, (int)(((long long)n * n + kET - 1) / kET))), kET, 0, st>>>(n, A, lda, d);
    if ((err = hipGetLastError()) != hipSuccess) return err;

    // --- Stage 2: divide and conquer on T ------------------------------------
    dc_init<<<(n + kET - 1) / kET, kET, 0, st>>>(n, d, e, D);
    if ((err = fill_matrix<double>(n, n, Qa, ld, 0, 1, 1.0, 0.0, st)) != hipSuccess) return err;
    DcArgs da;
    da.n = n; da.e = e; da.D = D; da.ld = ld; da.ds = ds; da.zs = zs; da.pole = pole; da.zp = zp;
    da.dval = dval; da.rc = rc; da.rs = rs; da.tau = dtau; da.zh = zh; da.vals = vals; da.rho = rho;
    da.colsrc = colsrc; da.src = src; da.ri = ri; da.rj = rj; da.org = org; da.inv = inv; da.K = Kc;
    da.nrot = nrot;
    for (int s = 1; s < n; s *= 2) {
        const int ngroups = (n + 2 * s - 1) / (2 * s);
        da.s = s; da.Qa = Qa; da.Qb = Qb; da.U = U;
        dc_prepare<<<ngroups, kET, 0, st>>>(da);
        {
            const int k = std::min(2 * s, n);
            dc_rotate<<<dim3(std::max(1, std::min(64, (k + kET - 1) / kET)), ngroups), kET, 0, st>>>(da);
        }
        dc_secular<<<(n + 63) / 64, 64, 0, st>>>(da);
        dc_lowner<<<(n + 63) / 64, 64, 0, st>>>(da);
        dc_rank<<<(n + 63) / 64, 64, 0, st>>>(da);
        dc_vectors<<<n, kET, 0, st>>>(da);
        if ((err = fill_matrix<double>(n, n, Qb, ld, 0, 1, 0.0, 0.0, st)) != hipSuccess) return err;
        if (2 * s <= 64) {
            dc_small_product<<<ngroups, kET, 0, st>>>(da, ngroups);
        } else {
            const int full = n / (2 * s), k2 = 2 * s;
            const long long stride = (long long)k2 * (ld + 1);
            if (full > 0) {
                GemmDesc g;
                g.m = k2; g.n = k2; g.k = k2;
                g.A = Qa; g.lda = ld; g.strideA = stride;
                g.B = U; g.ldb = ld; g.strideB = stride;
                g.C = Qb; g.ldc = ld; g.strideC = stride;
                g.batch = full;
                if ((err = gemm(g, st)) != hipSuccess) return err;
            }
            const int tail = n - full * k2;
            if (tail > 0) {
                const long long off = (long long)full * stride;
                GemmDesc g;
                g.m = tail; g.n = tail; g.k = tail;
                g.A = Qa + off; g.lda = ld; g.B = U + off; g.ldb = ld; g.C = Qb + off; g.ldc = ld;
                if ((err = gemm(g, st)) != hipSuccess) return err;
            }
        }
        if ((err = hipGetLastError()) != hipSuccess) return err;
        std::swap(Qa, Qb);
    }

    // Eigenvalues to the host, descending order; matching columns.
    if ((err = hipMemcpyAsync(host, D, sizeof(double) * n, hipMemcpyDeviceToHost, st)) != hipSuccess) return err;
    if ((err = hipStreamSynchronize(st)) != hipSuccess) return err;
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y2) { return host[x] > host[y2]; });
    for (int i = 0; i < n; ++i) w_host[i] = host[order[i]];
    int* hperm = reinterpret_cast<int*>(host);
    for (int i = 0; i < n; ++i) hperm[i] = order[i];
    if ((err = hipMemcpyAsync(perm, hperm, sizeof(int) * n, hipMemcpyHostToDevice, st)) != hipSuccess) return err;
    gather_columns<<<dim3(std::max(1, std::min(64, (n + kET - 1) / kET)), n), kET, 0, st>>>(n, Qa, ld, perm, Z, ldz);

    // --- Stage 3: Z <- Q Z with the reflectors of stage 1 --------------------
    const int nref = n - 1;
    const long long ldt = std::min(kBT, n);   // scratch U, Qb hold nb x n with nb <= ldt
    for (int b0 = ((nref - 1) / kBT) * kBT; nref > 0 && b0 >= 0; b0 -= kBT) {
        const int nb = std::min(kBT, nref - b0);
        const int rows = n - b0 - 1;
        const double* V = A + (b0 + 1) + (long long)b0 * lda;
        GemmDesc s;  // S = V^T V
        s.m = nb; s.n = nb; s.k = rows; s.transa = 1;
        s.A = V; s.lda = lda; s.B = V; s.ldb = lda; s.C = S; s.ldc = kBT;
        s.flags = kAUpper | kBLower;
        if ((err = gemm(s, st)) != hipSuccess) return err;
        form_t<<<1, kBT, 0, st>>>(nb, S, kBT, tau + b0, Tf, kBT);
        GemmDesc w1;  // U = V^T Z[b0+1:, :]   (nb x n, in U)
        w1.m = nb; w1.n = n; w1.k = rows; w1.transa = 1;
        w1.A = V; w1.lda = lda; w1.B = Z + (b0 + 1); w1.ldb = ldz; w1.C = U; w1.ldc = ldt;
        w1.flags = kAUpper;
        if ((err = gemm(w1, st)) != hipSuccess) return err;
        GemmDesc w2;  // Qb = T U
        w2.m = nb; w2.n = n; w2.k = nb;
        w2.A = Tf; w2.lda = kBT; w2.B = U; w2.ldb = ldt; w2.C = Qb; w2.ldc = ldt;
        w2.flags = kAUpper;
        if ((err = gemm(w2, st)) != hipSuccess) return err;
        GemmDesc w3;  // Z[b0+1:, :] -= V Qb
        w3.m = rows; w3.n = n; w3.k = nb;
        w3.A = V; w3.lda = lda; w3.B = Qb; w3.ldb = ldt;
        w3.Cin = Z + (b0 + 1); w3.ldcin = ldz; w3.beta = 1.0; w3.alpha = -1.0;
        w3.C = Z + (b0 + 1); w3.ldc = ldz;
        w3.flags = kALower;
        if ((err = gemm(w3, st)) != hipSuccess) return err;
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    return hipStreamSynchronize(st);
}

}  // namespace zolo
