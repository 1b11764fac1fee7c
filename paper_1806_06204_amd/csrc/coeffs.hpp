// Host FP64 Zolotarev coefficients (Section 2.2, eqs. (7)-(10), Table 1).
#pragma once

namespace zolo {

constexpr int kMaxR = 8;
constexpr double kLMin = 1e-20;
constexpr double kConverged = 1.0 - 1e-15;  // Table 1 criterion on l_k

struct Coeffs {
    int r = 0;
    double l = 0.0;             // l after clamping to >= kLMin
    double c[2 * kMaxR] = {};   // c_1..c_2r
    double a[kMaxR] = {};       // a_1..a_r
    double mhat = 0.0;
    double l_next = 0.0;        // Zhat(l; l)
    double kappa_z = 0.0;       // (1 + c_1) / (l^2 + c_1) = max_j kappa(X^T X + c_{2j-1} I)
};

// 0 on success, -1 for l outside (0, 1], -2 for r outside [1, 8].
int compute_coeffs(double l, int r, Coeffs* out);
// 1 - Zhat(l; l) via the modular transformation of the nome.
double one_minus_l_next(double l, int r);
// Iterations k of the scalar recursion until l_k >= 1 - 1e-15 (Table 1).
int iterations_to_converge(double l0, int r, int max_iter);
// Smallest r <= 8 converging in at most two iterations from l.
int choose_r(double l);

// Step kinds ('Q'/'C', NUL-terminated, at most max_steps) the solve takes
// from l with degree r, assuming the verified check passes once l reaches
// 1 - 1e-15.  Returns the number of steps.
int predict_kinds(double l, int r, double chol_switch, char* kinds, int max_steps);
// Predicted milliseconds of a solve of m x n with degree r from l on one
// MI355X (cost model of the library's kernels; see coeffs.cpp).
double predict_ms(double l, int r, int m, int n, double chol_switch, char* kinds);
// r in [1, 8] with the least predicted_ms (ties: the smaller r).
int choose_r_time(double l, int m, int n, double chol_switch);

}  // namespace zolo
