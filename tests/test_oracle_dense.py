"""Pins for the oracle's own dense factorisations.

Each routine is checked against its defining invariants (orthonormality,
reconstruction, triangularity) and against an independent LAPACK routine from
NumPy, which the oracle itself never calls.
"""

import numpy as np
import pytest

from oracle import dense


@pytest.mark.parametrize("m,n", [(7, 7), (40, 13), (96, 64)])
def test_householder_qr(m, n):
    rng = np.random.default_rng(m * 100 + n)
    M = rng.standard_normal((m, n))
    Q, R = dense.householder_qr(M)
    assert np.allclose(np.triu(R), R)
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) < 1e-14 * n
    assert np.linalg.norm(Q @ R - M) < 1e-14 * np.linalg.norm(M) * n
    _, R_ref = np.linalg.qr(M)
    # R is unique up to the sign of each row.
    s = np.sign(np.diag(R)) * np.sign(np.diag(R_ref))
    assert np.allclose(R * s[:, None], R_ref, rtol=1e-11, atol=1e-12)


def test_householder_qr_stacked_identity():
    # The structure of eq. (12): [X; sqrt(c) I].
    rng = np.random.default_rng(5)
    X = rng.standard_normal((30, 12))
    M = np.vstack([X, 0.3 * np.eye(12)])
    Q, R = dense.householder_qr(M)
    assert np.linalg.norm(Q @ R - M) < 1e-13
    # The bottom block of Q is sqrt(c) R^{-1}: upper triangular.
    assert np.allclose(np.tril(Q[30:], -1), 0.0, atol=1e-14)


def test_cholesky_and_breakdown():
    rng = np.random.default_rng(1)
    B = rng.standard_normal((50, 20))
    Z = B.T @ B + 0.1 * np.eye(20)
    R = dense.cholesky_upper(Z)
    assert np.allclose(np.triu(R), R)
    assert np.allclose(R, np.linalg.cholesky(Z).T, rtol=1e-12, atol=1e-13)
    Zbad = Z.copy()
    Zbad[5, 5] = -1.0
    with pytest.raises(dense.CholeskyBreakdown):
        dense.cholesky_upper(Zbad)


def test_triangular_solves():
    rng = np.random.default_rng(2)
    R = np.triu(rng.standard_normal((25, 25))) + 5 * np.eye(25)
    X = rng.standard_normal((40, 25))
    Y1 = dense.solve_right_upper(X, R)
    Y2 = dense.solve_right_upper_transpose(X, R)
    assert np.allclose(Y1, np.linalg.solve(R.T, X.T).T, rtol=1e-12, atol=1e-13)
    assert np.allclose(Y2, np.linalg.solve(R, X.T).T, rtol=1e-12, atol=1e-13)
    assert np.allclose(dense.invert_upper(R) @ R, np.eye(25), atol=1e-13)


def test_jacobi_eigh():
    rng = np.random.default_rng(3)
    B = rng.standard_normal((30, 30))
    S = B + B.T
    w, V = dense.jacobi_eigh(S)
    assert np.all(np.diff(w) <= 0)
    assert np.allclose(w, np.sort(np.linalg.eigvalsh(S))[::-1], rtol=1e-12, atol=1e-12)
    assert np.linalg.norm(V.T @ V - np.eye(30)) < 1e-13
    assert np.linalg.norm(S @ V - V * w) < 1e-12 * np.linalg.norm(S)
