"""Zolo-PD and Zolo-SVD in plain FP64 (oracle; test infrastructure only).

Follows Algorithm 1 (Zolo-PD) and Algorithm 3 steps 1-4 of Li, Liu & Du,
arXiv 1806.06204, with each QR-type step in the inverse-free form of
eq. (12) (Theorem 2.2) and each Cholesky-type step in the form of
Algorithm 1 step 4(d); Algorithm 2 for the SVD.

Readings taken where the paper is silent or garbled (each is listed with its
reason in the design notes of the repository):

R1  alpha, when not given: 1.01 x a power-iteration estimate of ||A||_2
    (the paper assumes the bound is known, Section 3.2).
R2  l, when not given: l = 1 / (sqrt(n) ||R^{-1}||_1) from a Householder QR
    X0 = Q R; since ||R^{-1}||_2 <= sqrt(n) ||R^{-1}||_1 this is a lower bound
    on sigma_min(X0) (the paper assumes it known).
R3  r, when not given: the smallest r <= 8 whose scalar recursion meets the
    Table 1 criterion within two iterations (Section 2.2).
R4  Algorithm 1 step 3 "X1 = A": X1 is X0 = A / alpha; the Cholesky step is
    taken directly.  The step rule R6 does this by itself when kappa < 2.
R5  coefficients: theta-series evaluation of eq. (7), a_j as the quotient,
    l <- Zhat(l; l) with l^2 + c_{2j} (see oracle.coeffs).
R6  step kind: QR-type when (1 + c_1)/(l^2 + c_1) > 100, else Cholesky-type.
    The bound is max_j kappa(X^T X + c_{2j-1} I) for sigma(X) in [l, 1]; it is
    the Zolo analogue of the switch at c_k <= 100 used for QDWH (Section 2.1).
    A Cholesky breakdown redoes the step as QR-type.
R7  "L = Chol(Z)" is the upper factor R with R^T R = Z, so that
    X L^{-1} L^{-*} = X Z^{-1}.
R8  stop rule.  Paper mode: ||X_new - X_old||_F / ||X_new||_F <= eps^(1/(2r+1))
    with eps = 2^-52 (Algorithm 1 step 4(d), Algorithm 3 step 4(e)).
    Verified mode (default): once the predicted l reaches 1 - 1e-15 compute
    d = ||X^T X - I||_F / sqrt(n); stop if d <= tau, else continue with
    l = sqrt(1 - sqrt(n) d) (a lower bound on sigma_min when sqrt(n) d < 1).
    When sqrt(n) d >= 1 that bound is void (l was above sigma_min, so some
    singular values are still far from 1) and l is re-estimated by R2 on the
    current X, which is a bound again.
R9  "return to Step 1 with A <- X2": continue the loop with X and l updated,
    as Algorithm 3 step 4(e) states.
"""

import math

import numpy as np

from . import coeffs as zc
from . import dense

EPS = 2.0 ** -52


def frob(M):
    return math.sqrt(float(np.sum(np.asarray(M) * np.asarray(M))))


def estimate_alpha(A, max_steps=100, rtol=1e-10):
    """R1: 1.01 x power-iteration estimate of sigma_max(A) (on A^T A)."""
    n = A.shape[1]
    v = np.ones(n) / math.sqrt(n)
    lam = 0.0
    for it in range(max_steps):
        w = A.T @ (A @ v)
        lam_new = float(v @ w)
        nw = frob(w)
        if nw == 0.0:
            return 0.0
        v = w / nw
        if it >= 1 and abs(lam_new - lam) <= rtol * lam_new:
            lam = lam_new
            break
        lam = lam_new
    return 1.01 * math.sqrt(lam)


def estimate_l(X0):
    """R2: l = 1 / (sqrt(n) ||R^{-1}||_1) from X0 = Q R."""
    n = X0.shape[1]
    _, R = dense.householder_qr(X0)
    if np.any(np.diag(R) == 0.0):
        return zc.L_MIN
    rinv = dense.invert_upper(R)
    norm1 = float(np.max(np.sum(np.abs(rinv), axis=0)))
    return 1.0 / (math.sqrt(n) * norm1)


def step_kind(l, c, chol_switch=100.0):
    """R6: 'Q' when max_j kappa(Z_j) > chol_switch, else 'C'."""
    return "Q" if zc.z_condition_bound(l, c) > chol_switch else "C"


def qr_step(X, co):
    """One QR-type step, eq. (12): for each j a Householder QR of the stacked
    [X; sqrt(c_{2j-1}) I] = [Q_j1; Q_j2] R_j, then
    X_new = Mhat (X + sum_j a_j / sqrt(c_{2j-1}) Q_j1 Q_j2^T)."""
    m, n = X.shape
    c, a, mhat = co["c"], co["a"], co["mhat"]
    acc = X.copy()
    for j in range(len(a)):
        s = math.sqrt(c[2 * j])
        M = np.vstack([X, s * np.eye(n)])
        Q, _ = dense.householder_qr(M)
        acc += (a[j] / s) * (Q[:m] @ Q[m:].T)
    return mhat * acc


def chol_step(X, co):
    """One Cholesky-type step, Algorithm 1 step 4(d):
    Z_j = X^T X + c_{2j-1} I = R_j^T R_j,
    X_new = Mhat (X + sum_j a_j (X R_j^{-1}) R_j^{-T}).
    Raises dense.CholeskyBreakdown if some Z_j is not numerically SPD."""
    n = X.shape[1]
    c, a, mhat = co["c"], co["a"], co["mhat"]
    G = X.T @ X
    acc = X.copy()
    for j in range(len(a)):
        R = dense.cholesky_upper(G + c[2 * j] * np.eye(n))
        Y = dense.solve_right_upper_transpose(dense.solve_right_upper(X, R), R)
        acc += a[j] * Y
    return mhat * acc


def orthogonality(Q):
    """||Q^T Q - I||_F / sqrt(n)."""
    n = Q.shape[1]
    return frob(Q.T @ Q - np.eye(n)) / math.sqrt(n)


def backward_error(A, Qp, H):
    """||A - Qp H||_F / ||A||_F."""
    return frob(A - Qp @ H) / frob(A)


def zolo_pd(A, alpha=None, l=None, r=None, *, stop="verified", tau=5e-14,
            chol_switch=100.0, max_iter=10, record=False):
    """Polar decomposition A = Qp H by Zolo-PD (Algorithm 1).

    Returns (Qp, H, info).  info holds: status (0 converged, 1 not converged
    within max_iter), iters, kinds (one 'Q'/'C' per step), ls (l before each
    step), r, alpha, l0, chol_fallbacks, l_reestimates (R8) and, if record,
    the iterates X_k (X_0 = A / alpha first)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        raise ValueError("zolo_pd needs m >= n")
    if not np.all(np.isfinite(A)):
        raise ValueError("A has non-finite entries")
    if alpha is None:
        alpha = estimate_alpha(A)
    if not alpha > 0.0:
        raise ValueError("alpha must be positive (A = 0?)")
    X = A / alpha
    if l is None:
        l = estimate_l(X)
    l = min(max(float(l), zc.L_MIN), 1.0)
    l0 = l
    if r is None:
        r = zc.choose_r(l)
    info = {"status": 1, "iters": 0, "kinds": [], "ls": [], "r": int(r),
            "alpha": float(alpha), "l0": l0, "chol_fallbacks": 0, "l_reestimates": 0,
            "iterates": [X.copy()] if record else None, "orth_checks": [], "check_iters": []}
    for _ in range(max_iter):
        co = zc.coefficients(l, r)
        kind = step_kind(l, co["c"], chol_switch)
        info["ls"].append(l)
        if kind == "C":
            try:
                X_new = chol_step(X, co)
            except dense.CholeskyBreakdown:
                info["chol_fallbacks"] += 1
                kind = "Q"
        if kind == "Q":
            X_new = qr_step(X, co)
        info["kinds"].append(kind)
        info["iters"] += 1
        l_pred = co["l_next"]
        X_old, X = X, X_new
        if record:
            info["iterates"].append(X.copy())
        if stop == "paper":
            rel = frob(X - X_old) / frob(X)
            l = l_pred
            if rel <= EPS ** (1.0 / (2 * r + 1)):
                info["status"] = 0
                break
        else:
            if l_pred >= zc.CONVERGED:
                d = orthogonality(X)
                info["orth_checks"].append(d)
                info["check_iters"].append(info["iters"] - 1)
                if d <= tau:
                    info["status"] = 0
                    break
                b = math.sqrt(n) * d
                if b < 1.0:
                    l = math.sqrt(max(zc.L_MIN ** 2, 1.0 - b))
                else:
                    l = min(max(estimate_l(X), zc.L_MIN), 1.0)
                    info["l_reestimates"] += 1
            else:
                l = l_pred
    Qp = X
    C = Qp.T @ A
    H = 0.5 * (C + C.T)
    return Qp, H, info


def zolo_svd(A, alpha=None, l=None, r=None, **kw):
    """Zolo-SVD, Algorithm 2: A = Qp H, H = V Sigma V^T, U = Qp V.

    Returns (U, S, V, info) with S descending."""
    Qp, H, info = zolo_pd(A, alpha, l, r, **kw)
    S, V = dense.jacobi_eigh(H)
    U = Qp @ V
    return U, S, V, info


def svd_residual_paper(A, U, S, V):
    """Res of eq. (13): ||A - U Sigma V^T||_F / ||A||_2, with ||A||_2 = max S."""
    return frob(A - (U * S) @ V.T) / float(np.max(np.abs(S)))


def orth_paper(U):
    """OrthL / OrthR of Section 4.1: ||I - U^T U||_F / n."""
    n = U.shape[1]
    return frob(np.eye(n) - U.T @ U) / n
