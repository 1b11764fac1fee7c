"""Plain FP64 dense factorisations for the oracle (test infrastructure only).

Textbook, unblocked algorithms, one column at a time, written for clarity:
Householder QR with an explicitly formed thin Q, upper Cholesky (R^T R = Z),
triangular solves from the right, and the cyclic Jacobi eigenvalue method.
NumPy provides storage and vector/matrix products; no LAPACK factorisation is
called.  None of this shares code with the HIP library.
"""

import numpy as np


class CholeskyBreakdown(ArithmeticError):
    """A non-positive pivot appeared in the Cholesky factorisation."""


def householder_vector(x):
    """Reflector H = I - tau v v^T with v[0] = 1 and H x = beta e_1.

    beta has the opposite sign of x[0] so that x[0] - beta never cancels."""
    alpha = x[0]
    sigma = float(x[1:] @ x[1:])
    v = x.astype(np.float64).copy()
    if sigma == 0.0 and alpha >= 0.0:
        v[:] = 0.0
        v[0] = 1.0
        return v, 0.0, alpha
    norm = np.sqrt(alpha * alpha + sigma)
    beta = -norm if alpha >= 0.0 else norm
    v[1:] = x[1:] / (alpha - beta)
    v[0] = 1.0
    tau = (beta - alpha) / beta
    return v, tau, beta


def householder_qr(M):
    """Unblocked Householder QR of an m x n matrix (m >= n).

    Returns (Q, R): Q is m x n with orthonormal columns (thin Q formed by
    applying the reflectors, last to first, to the first n columns of I) and R
    is n x n upper triangular with M = Q R."""
    A = np.array(M, dtype=np.float64, copy=True)
    m, n = A.shape
    if m < n:
        raise ValueError("householder_qr needs m >= n")
    vs = []
    taus = []
    for k in range(n):
        v, tau, beta = householder_vector(A[k:, k])
        if k + 1 < n:
            w = v @ A[k:, k + 1:]
            A[k:, k + 1:] -= tau * np.outer(v, w)
        A[k, k] = beta
        A[k + 1:, k] = 0.0
        vs.append(v)
        taus.append(tau)
    R = np.triu(A[:n, :n])
    Q = np.zeros((m, n))
    Q[:n, :n] = np.eye(n)
    for k in range(n - 1, -1, -1):
        v = vs[k]
        w = v @ Q[k:, k:]
        Q[k:, k:] -= taus[k] * np.outer(v, w)
    return Q, R


def cholesky_upper(Z):
    """Upper-triangular R with R^T R = Z (Z symmetric positive definite).

    Raises CholeskyBreakdown on a non-positive (or non-finite) pivot."""
    Z = np.array(Z, dtype=np.float64, copy=True)
    n = Z.shape[0]
    R = np.zeros((n, n))
    for k in range(n):
        d = Z[k, k] - float(R[:k, k] @ R[:k, k])
        if not (d > 0.0) or not np.isfinite(d):
            raise CholeskyBreakdown(f"non-positive pivot {d!r} at column {k}")
        R[k, k] = np.sqrt(d)
        if k + 1 < n:
            R[k, k + 1:] = (Z[k, k + 1:] - R[:k, k] @ R[:k, k + 1:]) / R[k, k]
    return R


def solve_right_upper(X, R):
    """Y = X R^{-1} for upper-triangular R (column by column, Y R = X)."""
    X = np.asarray(X, dtype=np.float64)
    n = R.shape[0]
    Y = np.zeros_like(X)
    for k in range(n):
        Y[:, k] = (X[:, k] - Y[:, :k] @ R[:k, k]) / R[k, k]
    return Y


def solve_right_upper_transpose(X, R):
    """Y = X R^{-T} for upper-triangular R (Y R^T = X, R^T lower triangular)."""
    X = np.asarray(X, dtype=np.float64)
    n = R.shape[0]
    Y = np.zeros_like(X)
    for k in range(n - 1, -1, -1):
        Y[:, k] = (X[:, k] - Y[:, k + 1:] @ R[k, k + 1:]) / R[k, k]
    return Y


def invert_upper(R):
    """R^{-1} for upper-triangular R, by back substitution on the identity."""
    n = R.shape[0]
    return solve_right_upper(np.eye(n), R)


def jacobi_eigh(S, tol=1e-15, max_sweeps=60):
    """Eigen-decomposition of a symmetric matrix by the cyclic Jacobi method.

    Returns (w, V) with S V = V diag(w), eigenvalues in descending order.
    Each rotation annihilates one off-diagonal pair (classical two-sided
    Jacobi); sweeps stop when the off-diagonal mass is below tol * ||S||_F."""
    A = np.array(S, dtype=np.float64, copy=True)
    n = A.shape[0]
    V = np.eye(n)
    scale = np.linalg.norm(A)  # Frobenius norm (a plain sum of squares)
    for _ in range(max_sweeps):
        # Off-diagonal mass summed directly: ||A||^2 - ||diag A||^2 would cancel
        # to zero long before the rotations have converged.
        off = np.sqrt(float(np.sum((A - np.diag(np.diag(A))) ** 2)))
        if off <= tol * scale:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = A[p, q]
                if abs(apq) <= 1e-300 or abs(apq) <= 1e-18 * abs(A[q, q] - A[p, p]):
                    # Negligible against the diagonal gap: the rotation angle
                    # is below rounding, so the pair is already decoupled.
                    continue
                theta = (A[q, q] - A[p, p]) / (2.0 * apq)
                if theta == 0.0:
                    t = 1.0
                else:
                    t = np.sign(theta) / (abs(theta) + np.sqrt(theta * theta + 1.0))
                c = 1.0 / np.sqrt(t * t + 1.0)
                s = t * c
                ap = A[:, p].copy()
                aq = A[:, q].copy()
                A[:, p] = c * ap - s * aq
                A[:, q] = s * ap + c * aq
                ap = A[p, :].copy()
                aq = A[q, :].copy()
                A[p, :] = c * ap - s * aq
                A[q, :] = s * ap + c * aq
                A[p, q] = 0.0
                A[q, p] = 0.0
                vp = V[:, p].copy()
                vq = V[:, q].copy()
                V[:, p] = c * vp - s * vq
                V[:, q] = s * vp + c * vq
    w = np.diag(A).copy()
    order = np.argsort(-w)
    return w[order], V[:, order]
