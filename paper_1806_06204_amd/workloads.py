"""Seeded synthetic inputs for Zolo-PD (shared by tests, bench and the oracle checks).

This module holds none of the method's arithmetic: it only builds matrices of
known singular structure, with the shapes and spectra of the paper's
workloads, so that the HIP library and the CPU oracle can be fed the same
inputs.

* Haar-distributed orthonormal factors: QR of a seeded Gaussian matrix with
  the columns multiplied by sign(diag R) (sign(0) = +1).
* A = U diag(sigma) V^T with sigma log-spaced from 1 down to 1/kappa, so
  alpha = sigma_max = 1 and l = sigma_min / sigma_max = 1/kappa are known.
* A banded-plus-sparse pattern matrix standing in for the paper's sparse
  test matrices (Section 4, Table 3 and Table 8), which are not available:
  N(0,1) entries on |i - j| <= bandwidth plus each off-band entry present
  with probability p, stored dense.
"""

import numpy as np


def haar(m, k, seed):
    """m x k matrix with orthonormal columns, Haar distributed (seeded): the
    Gaussian matrix from NumPy's seeded generator, its QR by NumPy's LAPACK."""
    g = np.random.default_rng(seed).standard_normal((m, k))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def logspaced_sigma(n, kappa):
    """sigma_i = kappa^(-(i-1)/(n-1)), i = 1..n (sigma_1 = 1, sigma_n = 1/kappa)."""
    if n == 1:
        return np.ones(1)
    return np.power(float(kappa), -np.arange(n) / (n - 1.0))


def svd_matrix(m, n, kappa, seed_u, seed_v, sigma=None):
    """A = U diag(sigma) V^T with Haar U (m x n), V (n x n).

    Returns (A, U, sigma, V); the exact polar factors are U V^T and
    V diag(sigma) V^T."""
    if sigma is None:
        sigma = logspaced_sigma(n, kappa)
    U = haar(m, n, seed_u)
    V = haar(n, n, seed_v)
    A = (U * sigma) @ V.T
    return np.asfortranarray(A), U, np.asarray(sigma, dtype=np.float64), V


def config_small(index=0, m=256, n=128, kappa=1e8):
    """The 256 x 128, kappa = 1e8 case (seeds 1000+i, 2000+i); r = 3, l = 1/kappa."""
    A, U, s, V = svd_matrix(m, n, kappa, 1000 + index, 2000 + index)
    return {"A": A, "U": U, "sigma": s, "V": V, "alpha": 1.0, "l": 1.0 / kappa, "r": 3}


def config_large(n=8192, kappa=1e16, index=1):
    """Square n x n, kappa = 1e16 log-spaced spectrum, r = 8, l = 1/kappa."""
    A, U, s, V = svd_matrix(n, n, kappa, 1000 + index, 2000 + index)
    return {"A": A, "U": U, "sigma": s, "V": V, "alpha": 1.0, "l": 1.0 / kappa, "r": 8}


def sparse_pattern(n=4096, bandwidth=64, p=0.01, seed=3000):
    """Banded (|i-j| <= bandwidth) N(0,1) entries plus each off-band entry
    present with probability p (N(0,1) value); returned dense, column-major."""
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n))
    i, j = np.indices((n, n))
    band = np.abs(i - j) <= bandwidth
    off = (~band) & (rng.random((n, n)) < p)
    mask = band | off
    A[mask] = rng.standard_normal(int(mask.sum()))
    return np.asfortranarray(A)


def batch_specs(count=512, seed=4000, nmin=64, nmax=1024, kmin=2.0, kmax=12.0):
    """Shapes and condition numbers of a batch of uneven matrices:
    n ~ U{nmin..nmax}, m ~ U{n..2n}, log10 kappa ~ U[kmin, kmax]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        m = int(rng.integers(n, 2 * n + 1))
        kappa = float(10.0 ** rng.uniform(kmin, kmax))
        out.append({"m": m, "n": n, "kappa": kappa, "seed_u": seed + 10 * i + 1,
                    "seed_v": seed + 10 * i + 2})
    return out


def training_spectra(count, seed, nmin=128, nmax=2048, kmin=1.0, kmax=16.0):
    """Spectra for training the learned l/r estimator: n ~ U{nmin..nmax},
    m ~ U{n..2n}, log10 kappa ~ U[kmin, kmax]; half log-spaced from 1 to
    1/kappa, half clustered: 2-4 clusters at log-uniform positions in
    [1/kappa, 1] that always include 1 and 1/kappa, each value jittered by a
    factor in [0.95, 1.05] (then 1 and 1/kappa restored as the extremes).
    Returns (ms, ns, kappas, sigmas, families) with sigmas a list of
    descending arrays and families 0 (log-spaced) or 1 (clustered)."""
    rng = np.random.default_rng(seed)
    ms, ns, ks, sig, fam = [], [], [], [], []
    for _ in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        m = int(rng.integers(n, 2 * n + 1))
        kappa = float(10.0 ** rng.uniform(kmin, kmax))
        clustered = rng.random() >= 0.5
        if not clustered:
            s = logspaced_sigma(n, kappa)
        else:
            nc = int(rng.integers(2, 5))
            centres = np.concatenate([[0.0, -np.log10(kappa)],
                                      -np.log10(kappa) * rng.random(nc - 2)])
            which = rng.integers(0, nc, size=n)
            which[0], which[-1] = 0, 1
            s = 10.0 ** centres[which] * rng.uniform(0.95, 1.05, size=n)
            s = np.sort(np.clip(s, 1.0 / kappa, 1.0))[::-1]
            s[0], s[-1] = 1.0, 1.0 / kappa
        ms.append(m)
        ns.append(n)
        ks.append(kappa)
        sig.append(np.asarray(s, dtype=np.float64))
        fam.append(int(clustered))
    return ms, ns, ks, sig, fam
