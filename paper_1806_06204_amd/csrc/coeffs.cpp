// Zolotarev coefficients on the host, FP64 (Section 2.2 of the paper).
//
//   c_i = l^2 sn^2(i K'/(2r+1); l') / cn^2(i K'/(2r+1); l'),  i = 1..2r   (eq. (7))
//   Mhat = prod_j (1 + c_{2j-1}) / (1 + c_{2j})                           (eq. (8))
//   a_j  = -prod_k (c_{2j-1} - c_{2k}) / prod_{k!=j} (c_{2j-1} - c_{2k-1})  (eq. (10),
//          read as the quotient: the residue of prod(t+c_{2k})/(t+c_{2k-1})
//          at t = -c_{2j-1}, which is what makes eq. (9) an identity)
//   l_next = Zhat(l; l) = Mhat l prod_j (l^2 + c_{2j}) / (l^2 + c_{2j-1})
//          (Algorithm 1 step 4(c) with l^2 + c_{2j}, i.e. Zhat at x = l)
//
// sn/cn at modulus l' are never evaluated directly (l' rounds to 1 when l is
// tiny).  For l <= 1/sqrt(2) the Jacobi imaginary transformation turns sc(u;l')
// into sn(iu; l), written with theta functions of nome q = exp(-pi K'/K):
//     c_i = 4 l sqrt(q) (S/C)^2,  S = sum (-1)^n q^{n(n+1)} sinh((2n+1) y),
//     C = 1 + 2 sum_{n>=1} (-1)^n q^{n^2} cosh(2 n y),  y = pi u / (2K).
// For l > 1/sqrt(2) the nome of l' itself, q' = exp(-pi K/K'), is small and
//     c_i = l (S'/C')^2,  S' = sum (-1)^n q'^{n(n+1)} sin((2n+1) v),
//     C' = sum q'^{n(n+1)} cos((2n+1) v),  v = i pi / (2(2r+1)).
// K = K(l), K' = K(l') from the arithmetic-geometric mean.  c_{r+1..2r} come
// from the reflection c_i c_{2r+1-i} = l^2.
//
// Near convergence 1 - l_next is evaluated without cancellation: a Zolo-PD
// step maps the complementary nome q' to q'^(2r+1) (degree-(2r+1) modular
// transformation), so l'_next = (theta2/theta3)^2 at that nome and
// 1 - l_next = l'_next^2 / (1 + l_next).
#include "coeffs.hpp"

#include <cmath>

namespace zolo {

namespace {

constexpr double kPi = 3.14159265358979323846;

double agm(double a, double b) {
    for (int it = 0; it < 80 && std::fabs(a - b) > 1e-16 * a; ++it) {
        const double an = 0.5 * (a + b);
        b = std::sqrt(a * b);
        a = an;
    }
    return 0.5 * (a + b);
}

double comp(double x) { return std::sqrt((1.0 - x) * (1.0 + x)); }

}  // namespace

double one_minus_l_next(double l, int r) {
    const double lp = comp(l);
    if (lp == 0.0) return 0.0;
    const double K = kPi / (2.0 * agm(1.0, lp));
    const double Kp = kPi / (2.0 * agm(1.0, l));
    const double lnq1 = -(2.0 * r + 1.0) * kPi * K / Kp;
    double s2 = 0.0, s3 = 1.0;
    for (int n = 0; n < 40; ++n) s2 += std::exp(lnq1 * n * (n + 1.0));
    for (int n = 1; n < 40; ++n) s3 += 2.0 * std::exp(lnq1 * n * (double)n);
    const double th2 = 2.0 * std::exp(0.25 * lnq1) * s2;
    const double lp1 = (th2 / s3) * (th2 / s3);
    const double l1 = comp(lp1);
    return lp1 * lp1 / (1.0 + l1);
}

int compute_coeffs(double l, int r, Coeffs* out) {
    if (!(l > 0.0) || !(l <= 1.0)) return -1;
    if (r < 1 || r > kMaxR) return -2;
    if (l < kLMin) l = kLMin;
    out->r = r;
    out->l = l;
    const double lp = comp(l);
    const double Kp = kPi / (2.0 * agm(1.0, l));            // K(l')
    const bool kinf = lp == 0.0;
    const double K = kinf ? HUGE_VAL : kPi / (2.0 * agm(1.0, lp));  // K(l)
    for (int i = 1; i <= r; ++i) {
        double ci;
        if (l <= 1.0 / std::sqrt(2.0)) {
            const double lnq = -kPi * Kp / K;
            const double y = kPi * (i * Kp / (2 * r + 1)) / (2.0 * K);
            double S = 0.0, C = 1.0;
            for (int n = 0; n < 12; ++n) {
                const double w = std::exp(lnq * n * (n + 1.0));
                S += ((n & 1) ? -w : w) * std::sinh((2 * n + 1) * y);
            }
            for (int n = 1; n < 12; ++n) {
                const double w = 2.0 * std::exp(lnq * n * (double)n);
                C += ((n & 1) ? -w : w) * std::cosh(2.0 * n * y);
            }
            ci = 4.0 * l * std::exp(0.5 * lnq) * (S / C) * (S / C);
        } else {
            const double v = i * kPi / (2.0 * (2 * r + 1));
            double S = std::sin(v), C = std::cos(v);
            if (!kinf) {
                const double lnq = -kPi * K / Kp;
                for (int n = 1; n < 12; ++n) {
                    const double w = std::exp(lnq * n * (n + 1.0));
                    S += ((n & 1) ? -w : w) * std::sin((2 * n + 1) * v);
                    C += w * std::cos((2 * n + 1) * v);
                }
            }
            ci = l * (S / C) * (S / C);
        }
        out->c[i - 1] = ci;
    }
    for (int i = r + 1; i <= 2 * r; ++i) out->c[i - 1] = l * l / out->c[2 * r - i];
    // Mhat, a_j
    double mh = 1.0;
    for (int j = 0; j < r; ++j) mh *= (1.0 + out->c[2 * j]) / (1.0 + out->c[2 * j + 1]);
    out->mhat = mh;
    for (int j = 0; j < r; ++j) {
        const double co = out->c[2 * j];
        double aj = out->c[2 * j + 1] - co;  // -(c_{2j-1} - c_{2j})
        for (int k = 0; k < r; ++k)
            if (k != j) aj *= (co - out->c[2 * k + 1]) / (co - out->c[2 * k]);
        out->a[j] = aj;
    }
    double z = mh * l;
    for (int j = 0; j < r; ++j) z *= (l * l + out->c[2 * j + 1]) / (l * l + out->c[2 * j]);
    if (1.0 - z < 1e-3) z = 1.0 - one_minus_l_next(l, r);
    out->l_next = z > 1.0 ? 1.0 : z;
    out->kappa_z = (1.0 + out->c[0]) / (l * l + out->c[0]);
    return 0;
}

int iterations_to_converge(double l0, int r, int max_iter) {
    double l = l0;
    int k = 0;
    Coeffs co;
    while (l < kConverged && k < max_iter) {
        if (compute_coeffs(l, r, &co) != 0) return max_iter;
        l = co.l_next;
        ++k;
    }
    return k;
}

int choose_r(double l) {
    for (int r = 1; r <= kMaxR; ++r)
        if (iterations_to_converge(l, r, 3) <= 2) return r;
    return kMaxR;
}

int predict_kinds(double l, int r, double chol_switch, char* kinds, int max_steps) {
    Coeffs co;
    int k = 0;
    while (k < max_steps) {
        if (compute_coeffs(l, r, &co) != 0) break;
        kinds[k++] = co.kappa_z > chol_switch ? 'Q' : 'C';
        l = co.l_next;
        if (l >= kConverged) break;
    }
    kinds[k] = 0;
    return k;
}

// Cost model of one solve on one MI355X, fitted to solves of this library
// (n = 8192: the QR-type step of degree 8 takes 596 ms of which the
// 64-column panels take 75 ms, a Cholesky-type step 144 ms; the sweep over
// r of the same matrix sets the panel and small-r terms).  The matrix-core
// products run at kRate once they fill the chip; below kFill flops per
// launch the rate falls in proportion (launch latency and too few tiles).
namespace {
constexpr double kRate = 42.0e9;          // flops per ms of the products of a step
constexpr double kRateBig = 52.0e9;       // flops per ms of X^T X and Qp^T A
constexpr double kFill = 2.0e10;          // flops of a product that fills the chip
constexpr double kPanel0 = 0.30;          // ms per 64-column panel, fixed part
constexpr double kPanelRow = 0.036 / 8256; // ms per panel per live row and matrix
constexpr double kLaunch = 0.012;         // ms per dependent launch

double gemm_ms(double flops, double rate, double launches) {
    const double eff = flops / (flops + kFill / 8.0);
    return flops / (rate * eff) + launches * kLaunch;
}
}  // namespace

double predict_ms(double l, int r, int m, int n, double chol_switch, char* kinds) {
    char buf[64];
    char* kk = kinds ? kinds : buf;
    const int steps = predict_kinds(l, r, chol_switch, kk, 16);
    const double M = m, N = n, panels = (n + 63) / 64;
    double ms = 0.0;
    for (int s = 0; s < steps; ++s) {
        if (kk[s] == 'Q') {
            // GEQRF + ORGQR (2 M N^2 each) and the combination (M N^2) per j;
            // 128 panels of m + 64 live rows each way, about 12 launches per
            // 256-column superblock.
            ms += gemm_ms(5.0 * r * M * N * N, kRate, 12.0 * panels / 4.0);
            ms += panels * (kPanel0 + kPanelRow * r * (M + 64.0));
        } else {
            // X^T X, r POTRF/TRTRI (N^3 / 3 each) and the F accumulation
            // (N^3 / 3 per j), X F; about 6 launches per 64 columns.
            ms += gemm_ms(3.0 * M * N * N + r * N * N * N, kRate, 6.0 * panels);
        }
    }
    ms += gemm_ms(M * N * N, kRateBig, 2.0);        // the verified check
    ms += gemm_ms(2.0 * M * N * N, kRateBig, 2.0);  // H
    return ms;
}

int choose_r_time(double l, int m, int n, double chol_switch) {
    int best = 1;
    double best_ms = 0.0;
    for (int r = 1; r <= kMaxR; ++r) {
        const double t = predict_ms(l, r, m, n, chol_switch, nullptr);
        if (r == 1 || t < best_ms) {
            best = r;
            best_ms = t;
        }
    }
    return best;
}

}  // namespace zolo
