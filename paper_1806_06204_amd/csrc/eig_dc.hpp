// Scalar pieces of the tridiagonal divide-and-conquer eigensolver (Cuppen's
// method with deflation and Gu-Eisenstat eigenvectors), written once for the
// device kernels of eig.hip.  Every function is plain sequential code over
// arrays, so the same definitions can be compiled for the host.
//
// One merge joins two blocks whose eigendecompositions are known:
//   T = diag(T1, T2) + rho u u^T,  rho = |beta| >= 0,
// where beta couples the last row of T1 and the first row of T2 and
// u = e_last + sign(beta) e_first (T1, T2 had |beta| taken off their facing
// diagonal entries).  With T1 = Q1 D1 Q1^T, T2 = Q2 D2 Q2^T this is
//   diag(Q1, Q2) (D + rho z z^T) diag(Q1, Q2)^T,  z = [Q1^T e_last; sign(beta) Q2^T e_first],
// and the eigenproblem of D + rho z z^T is solved here.
#pragma once

#ifndef ZOLO_HD
#define ZOLO_HD __host__ __device__
#endif

#include <cmath>

namespace zolo {
namespace dc {

constexpr double kEps = 1.1102230246251565e-16;   // unit roundoff 2^-53

// Deflation (the rules of Cuppen's method as refined by Dongarra and
// Sorensen), as a scan over the merged poles in ascending order.  The caller
// normalises z (||z|| = 1, rho -> rho ||z||^2) and sets
//   tol = 8 eps max(max |d|, rho max |z|),
// then calls step() for t = 0..k-1 with the t-th smallest pole and its z,
// and finish() once.  Outputs (positions t are sorted positions):
//   pole[u], zp[u], src[u] for u < K: remaining poles, strictly ascending,
//     with their z and sorted position;
//   src[u], dval[u] for K <= u < k: deflated eigenvalues and positions;
//   ri, rj, rc, rs [0..nrot): rotations of the columns at sorted positions
//     (q_i, q_j) <- (c q_i + s q_j, c q_j - s q_i), to apply in order.
struct DeflateScan {
    double rho, tol;
    int k, K, ndef, nrot, prev;
    double dprev, zprev;
    double *pole, *zp, *dval, *rc, *rs;
    int *src, *ri, *rj;

    ZOLO_HD void begin(int k_, double rho_, double tol_) {
        k = k_;
        rho = rho_;
        tol = tol_;
        K = ndef = nrot = 0;
        prev = -1;
        dprev = zprev = 0.0;
    }
    // A rotation moves a pole by at most tol, so a kept pole can land on or
    // below its predecessor; it is then moved just above it (an eigenvalue
    // change below tol), which keeps the poles strictly ascending.
    ZOLO_HD void keep(int t, double d, double z) {
        if (K > 0 && !(d > pole[K - 1])) d = nextafter(pole[K - 1], INFINITY);
        pole[K] = d;
        zp[K] = z;
        src[K] = t;
        ++K;
    }
    ZOLO_HD void drop(int t, double d) {
        src[k - 1 - ndef] = t;
        dval[k - 1 - ndef] = d;
        ++ndef;
    }
    ZOLO_HD void step(int t, double dc, double zc) {
        if (rho * fabs(zc) <= tol) {          // negligible coupling: eigenpair as is
            drop(t, dc);
            return;
        }
        if (prev >= 0) {
            // Two close poles: a rotation of their columns zeroes z_prev.
            const double h = hypot(zprev, zc);
            const double cs = zc / h, sn = -zprev / h;
            if (fabs((dc - dprev) * cs * sn) <= tol) {
                ri[nrot] = prev;
                rj[nrot] = t;
                rc[nrot] = cs;
                rs[nrot] = sn;
                ++nrot;
                drop(prev, dprev * cs * cs + dc * sn * sn);
                dc = dprev * sn * sn + dc * cs * cs;
                zc = h;
            } else {
                keep(prev, dprev, zprev);
            }
        }
        prev = t;
        dprev = dc;
        zprev = zc;
    }
    // Flushes the last candidate; returns K.
    ZOLO_HD int finish() {
        if (prev >= 0) keep(prev, dprev, zprev);
        return K;
    }
};

// Root t (0 <= t < K) of the secular equation 1 + rho sum_j zp_j^2 / (pole_j - lambda) = 0
// with poles strictly increasing and rho > 0: lambda_t lies in (pole_t, pole_{t+1})
// (the last in (pole_{K-1}, pole_{K-1} + rho)).  lambda is returned as
// pole[*org] + *tau with the origin the nearer pole, so that the distances
// pole_j - lambda = (pole_j - pole_org) - tau keep their relative accuracy.
// Bisection on tau to the last bit.
ZOLO_HD inline void secular_root(int K, const double* pole, const double* zp, double rho, int t, int* org,
                                 double* tau) {
    const double left = pole[t];
    const double right = t + 1 < K ? pole[t + 1] : pole[t] + rho;
    int o = t;
    double lo = 0.0, hi = right - left;
    if (t + 1 < K) {
        // g at the midpoint, relative to the left pole, picks the origin.
        const double mid = 0.5 * (right - left);
        double g = 1.0 / rho;
        for (int j = 0; j < K; ++j) g += zp[j] * zp[j] / ((pole[j] - left) - mid);
        if (g < 0.0) {          // root in the right half: measure from pole_{t+1}
            o = t + 1;
            lo = -mid;
            hi = 0.0;
        } else {
            hi = mid;
        }
    }
    const double po = pole[o];
    for (int it = 0; it < 400; ++it) {
        const double m = 0.5 * (lo + hi);
        if (!(m > lo && m < hi)) break;
        double g = 1.0 / rho;
        for (int j = 0; j < K; ++j) g += zp[j] * zp[j] / ((pole[j] - po) - m);
        if (g > 0.0) hi = m;
        else lo = m;
    }
    *org = o;
    *tau = 0.5 * (lo + hi);
}

// pole_i - lambda_j for the root stored as (org_j, tau_j).
ZOLO_HD inline double pole_minus_root(const double* pole, int i, int org_j, double tau_j) {
    return (pole[i] - pole[org_j]) - tau_j;
}

// Gu-Eisenstat: the z that makes the computed roots the exact eigenvalues
// of diag(pole) + rho zh zh^T,
//   zh_i^2 = (lambda_{K-1} - pole_i) / rho * prod_{j<i} (lambda_j - pole_i)/(pole_j - pole_i)
//                                       * prod_{i<j<K} (lambda_{j-1} - pole_i)/(pole_j - pole_i),
// every factor positive by interlacing; the sign of zp_i.
ZOLO_HD inline double lowner_z(int K, const double* pole, const double* zp, double rho, const int* org,
                               const double* tau, int i) {
    double p = -pole_minus_root(pole, i, org[K - 1], tau[K - 1]) / rho;
    for (int j = 0; j < i; ++j) p *= pole_minus_root(pole, i, org[j], tau[j]) / (pole[i] - pole[j]);
    for (int j = i + 1; j < K; ++j) p *= pole_minus_root(pole, i, org[j - 1], tau[j - 1]) / (pole[i] - pole[j]);
    const double v = sqrt(fmax(p, 0.0));
    return zp[i] >= 0.0 ? v : -v;
}

}  // namespace dc
}  // namespace zolo
