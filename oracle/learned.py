"""Learned l/r estimator in plain FP64 (oracle; test infrastructure only).

The paper assumes that the bounds alpha >= sigma_max and beta (here l) <=
sigma_min/sigma_max are known before the iteration starts (Algorithm 1 steps
1-2; Section 3.2, whose Table 3 reports what computing them costs).  The
library can replace the condition estimate for l by a small network that
reads cheap sketch features of X0 = A / alpha.  This module defines, in
FP64 and in the order written here, everything that network path computes:
the random sketch, the features, the training surrogate, the network, its
loss, gradient and optimiser step.  The GPU kernels are checked against it.

G1  Counter-based generator: SplitMix64 (Steele, Lea & Flood, "Fast
    splittable pseudorandom number generators", OOPSLA 2014).  Output k of
    stream `seed` is mix(seed + (k + 1) * 0x9E3779B97F4A7C15) with
    mix: z <- (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9,
         z <- (z ^ (z >> 27)) * 0x94D049BB133111EB,  z ^ (z >> 31)
    (all mod 2^64).  Uniform number k: ((x_k >> 11) + 0.5) * 2^-53 in (0, 1).
    Gaussian number k: sqrt(-2 ln u_{2k}) cos(2 pi u_{2k+1}) (Box-Muller,
    cosine branch).
G2  Sketch: Omega (n x 32) with Omega[i, j] = Gaussian number i + j n of the
    stream; Y = X0 Omega; s_1 >= ... >= s_32 are the square roots of the
    eigenvalues of the Gram matrix Y^T Y.  Through the Gram matrix an s_i
    carries an absolute error of about eps s_1^2 / s_i, so ratios below 1e-6
    are rounding noise in any implementation; G3 floors them there.
G3  Features (39), norms clamped below at 1e-20 before each logarithm:
      f0        log10 s_1
      f1..f31   max(log10(s_{i+1} / s_1), -6)
      f32, f33  mean and population std of log10 ||X0 e_j|| over the n columns
      f34, f35  the same over the m rows
      f36, f37  log10 n, log10(m / n)
      f38       log10(||X0||_F / sqrt(n))   (root-mean-square singular value)
G4  Surrogate features of a spectrum sigma (the training data).  For
    A = U diag(sigma) V^T with Haar V, V^T Omega is again Gaussian, so the
    sketch singular values of A have the law of those of diag(sigma) G with G
    (n x 32) Gaussian; a column of A has the norm of diag(sigma) v for v a
    row of V (uniform on the sphere, sampled as g / ||g||, g Gaussian of
    length n); a row of A has the norm of diag(sigma) u for u a row of the
    first n columns of a Haar m x m matrix (sampled as g[:n] / ||g||, g of
    length m).  Matrix b of a set draws from one stream with its Gaussian
    numbers offset by b * 2^32: G[i, j] is number i + j n, column sample t
    (t < 32) numbers 32 n + t n .. 32 n + (t + 1) n - 1, row sample t
    numbers 64 n + t m .. 64 n + (t + 1) m - 1.  The mean and std in f32..f35
    are then over the 32 samples; every other feature is exact.
G5  Network (3 layers, 64 hidden, tanh): x = (f - mu) / sd,
    h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = W3 h2 + b3.
    y0 estimates log10(sigma_min / sigma_max) of X0 and y1 the degree r.
G6  Loss: the batch mean of  w (t0 - y0)^2 + c_r (t1 - y1)^2  with
    w = 1 - q when y0 > t0 (l over-estimated) and w = q otherwise (an
    expectile loss).  The library's training uses q = 0.05, so an
    over-estimate costs nineteen times an under-estimate, y0 leans low and
    10^y0 tends to stay a lower bound; q is an argument here (default 0.05).
G7  Adam (Kingma & Ba, ICLR 2015): m <- b1 m + (1 - b1) g,
    v <- b2 v + (1 - b2) g^2, p <- p - lr (m / (1 - b1^t)) /
    (sqrt(v / (1 - b2^t)) + eps), for the trainable part (W, b) only.

Flat parameter layout (float32 on the GPU, the same order here):
mu[39], sd[39], W1[64][39], b1[64], W2[64][64], b2[64], W3[2][64], b3[2]
(W row-major: W1[o][i] multiplies input i into output o).
"""

import math

import numpy as np

from . import dense

NF = 39          # features
NH = 64          # hidden width
NO = 2           # outputs
NS = 32          # sketch columns
LOG_FLOOR = -6.0  # floor of the normalised log sketch singular values (G2)
N_PARAMS = 2 * NF + NH * NF + NH + NH * NH + NH + NO * NH + NO
N_STATS = 2 * NF  # mu and sd lead the layout and are not trained

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


# --- G1 -------------------------------------------------------------------
def splitmix64(seed, k):
    """Output(s) k (uint64 array or int) of the SplitMix64 stream `seed`."""
    with np.errstate(over="ignore"):
        k = np.asarray(k, dtype=np.uint64)
        z = np.uint64(seed) + (k + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform(seed, k):
    x = splitmix64(seed, k)
    return ((x >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53


def gaussian(seed, k):
    """Gaussian number(s) k of the stream (Box-Muller, cosine branch)."""
    k = np.asarray(k, dtype=np.uint64)
    u1 = uniform(seed, np.uint64(2) * k)
    u2 = uniform(seed, np.uint64(2) * k + np.uint64(1))
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


# --- G2, G3 ---------------------------------------------------------------
def sketch_matrix(n, seed):
    """Omega (n x 32): Omega[i, j] = Gaussian number i + j n."""
    k = np.arange(n * NS, dtype=np.uint64)
    return gaussian(seed, k).reshape(NS, n).T


def _log10c(x):
    return np.log10(np.maximum(x, 1e-20))


def features_from(svals, colnorms, rownorms, m, n, frob):
    """Assemble the 39 features (G3) from the sketch singular values (any
    order), column norms, row norms and ||X0||_F."""
    s = np.sort(np.maximum(np.asarray(svals, dtype=np.float64), 0.0))[::-1]
    f = np.empty(NF)
    f[0] = _log10c(s[0])
    f[1:NS] = np.maximum(_log10c(s[1:]) - _log10c(s[0]), LOG_FLOOR)
    lc, lr = _log10c(np.asarray(colnorms)), _log10c(np.asarray(rownorms))
    f[32], f[33] = lc.mean(), lc.std()
    f[34], f[35] = lr.mean(), lr.std()
    f[36], f[37] = math.log10(n), math.log10(m / n)
    f[38] = _log10c(frob / math.sqrt(n))
    return f


def features(X0, seed):
    """Features of X0 (m x n) with the sketch of stream `seed` (G2, G3).  The
    singular values of Y are the square roots of the eigenvalues of Y^T Y
    (the oracle's own Jacobi eigensolver)."""
    X0 = np.asarray(X0, dtype=np.float64)
    m, n = X0.shape
    Y = X0 @ sketch_matrix(n, seed)
    lam, _ = dense.jacobi_eigh(Y.T @ Y)
    s = np.sqrt(np.maximum(lam, 0.0))
    return features_from(s, np.linalg.norm(X0, axis=0), np.linalg.norm(X0, axis=1), m, n,
                         np.linalg.norm(X0))


def surrogate_features(sigma, m, seed, index):
    """Training features of matrix `index` with spectrum sigma (length n) and
    m rows, drawn from stream `seed` as G4 specifies."""
    sigma = np.asarray(sigma, dtype=np.float64)
    n = sigma.size
    base = np.uint64(index) << np.uint64(32)

    def gauss(first, count):
        return gaussian(seed, base + np.arange(first, first + count, dtype=np.uint64))

    G = gauss(0, n * NS).reshape(NS, n).T
    lam, _ = dense.jacobi_eigh((G * sigma[:, None] ** 2).T @ G)
    s = np.sqrt(np.maximum(lam, 0.0))
    cols = np.empty(NS)
    rows = np.empty(NS)
    for t in range(NS):
        g = gauss(NS * n + t * n, n)
        cols[t] = np.linalg.norm(sigma * g) / np.linalg.norm(g)
        g = gauss(2 * NS * n + t * m, m)
        rows[t] = np.linalg.norm(sigma * g[:n]) / np.linalg.norm(g)
    return features_from(s, cols, rows, m, n, np.linalg.norm(sigma))


# --- G5 -------------------------------------------------------------------
def unpack(p):
    """Flat parameter vector -> dict of arrays (views)."""
    p = np.asarray(p, dtype=np.float64)
    assert p.size == N_PARAMS
    o = 0
    out = {}
    for name, shape in (("mu", (NF,)), ("sd", (NF,)), ("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)),
                        ("b2", (NH,)), ("W3", (NO, NH)), ("b3", (NO,))):
        size = int(np.prod(shape))
        out[name] = p[o:o + size].reshape(shape)
        o += size
    return out


def init_params(seed, mu=None, sd=None):
    """Glorot-uniform weights, zero biases (NumPy generator, seeded)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(N_PARAMS)
    P = unpack(p)
    P["mu"][:] = 0.0 if mu is None else mu
    P["sd"][:] = 1.0 if sd is None else sd
    for W in (P["W1"], P["W2"], P["W3"]):
        lim = math.sqrt(6.0 / (W.shape[0] + W.shape[1]))
        W[:] = rng.uniform(-lim, lim, size=W.shape)
    return p


def standardize_stats(F):
    """mu, sd (population) of the features over the samples (rows of F);
    sd floored at 1e-6."""
    F = np.asarray(F, dtype=np.float64)
    return F.mean(axis=0), np.maximum(F.std(axis=0), 1e-6)


def forward(p, F):
    """F (batch x 39) -> outputs (batch x 2) and the cache for backward."""
    P = unpack(p)
    x = (np.asarray(F, dtype=np.float64) - P["mu"]) / P["sd"]
    h1 = np.tanh(x @ P["W1"].T + P["b1"])
    h2 = np.tanh(h1 @ P["W2"].T + P["b2"])
    y = h2 @ P["W3"].T + P["b3"]
    return y, {"x": x, "h1": h1, "h2": h2}


# --- G6 -------------------------------------------------------------------
def loss(y, T, q=0.05, c_r=0.1):
    """Batch loss and its gradient with respect to y (G6)."""
    y = np.asarray(y, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    B = y.shape[0]
    e0 = T[:, 0] - y[:, 0]
    w = np.where(y[:, 0] > T[:, 0], 1.0 - q, q)
    e1 = T[:, 1] - y[:, 1]
    L = float(np.sum(w * e0 * e0 + c_r * e1 * e1) / B)
    dy = np.stack([-2.0 * w * e0, -2.0 * c_r * e1], axis=1) / B
    return L, dy


def backward(p, cache, dy):
    """Gradient of a loss with dL/dy = dy with respect to the flat parameters
    (zeros for mu and sd)."""
    P = unpack(p)
    g = np.zeros(N_PARAMS)
    Gd = unpack(g)
    dy = np.asarray(dy, dtype=np.float64)
    h1, h2, x = cache["h1"], cache["h2"], cache["x"]
    Gd["W3"][:] = dy.T @ h2
    Gd["b3"][:] = dy.sum(axis=0)
    dz2 = (dy @ P["W3"]) * (1.0 - h2 * h2)
    Gd["W2"][:] = dz2.T @ h1
    Gd["b2"][:] = dz2.sum(axis=0)
    dz1 = (dz2 @ P["W2"]) * (1.0 - h1 * h1)
    Gd["W1"][:] = dz1.T @ x
    Gd["b1"][:] = dz1.sum(axis=0)
    return g


# --- G7 -------------------------------------------------------------------
def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1) on the trainable part of p; returns
    new (p, m, v)."""
    p, g, m, v = (np.array(a, dtype=np.float64) for a in (p, g, m, v))
    s = slice(N_STATS, N_PARAMS)
    m[s] = b1 * m[s] + (1.0 - b1) * g[s]
    v[s] = b2 * v[s] + (1.0 - b2) * g[s] * g[s]
    mh = m[s] / (1.0 - b1 ** t)
    vh = v[s] / (1.0 - b2 ** t)
    p[s] = p[s] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def predict(p, f):
    """(l, r) from the features of one matrix: l = 10^y0 clamped to
    [1e-20, 1], r = round(y1) clamped to [1, 8]."""
    y, _ = forward(p, np.asarray(f, dtype=np.float64)[None, :])
    l = min(1.0, max(1e-20, 10.0 ** float(y[0, 0])))
    r = int(min(8, max(1, round(float(y[0, 1])))))
    return l, r
