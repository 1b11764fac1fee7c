"""Training and evaluation of the learned l/r estimator (include/zolo_learn.h).

The paper takes the lower bound l on sigma_min(X0) and the degree r as given
(Algorithm 1 steps 2-3; Section 3.2).  The library can instead read them off
a 32-column sketch of X0 with a small network.  This module drives the
library to build a training set from generated spectra (the surrogate
features of definition G4, computed on the GPU), to train the network with
the library's forward, backward and Adam kernels, and to evaluate it.  It
only generates inputs (spectra, initial weights, minibatch orders) and
marshals arguments; every feature, activation and gradient is computed by
the library.
"""

import math

import numpy as np

from . import workloads as W
from . import zolo

NF, NPARAMS, NSTATS = zolo.NF, zolo.MLP_NPARAMS, zolo.MLP_NSTATS
NH, NO = 64, 2


def init_params(seed):
    """Glorot-uniform weights and zero biases (float32); mu = 0, sd = 1 until
    zolo_mlp_stats fills them from the training features."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAMS, dtype=np.float32)
    p[NF:2 * NF] = 1.0
    o = NSTATS
    for fan_out, fan_in in ((NH, NF), (NH, NH), (NO, NH)):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        p[o:o + fan_out * fan_in] = rng.uniform(-lim, lim, size=fan_out * fan_in)
        o += fan_out * fan_in + fan_out
    assert o == NPARAMS
    return p


def build_set(z, count, seed, feature_seed, nmin=128, nmax=2048, kmin=1.0, kmax=16.0, chunk=4096):
    """Surrogate features (count, 39) float64 and targets (count, 2) float32
    (t0 = log10(sigma_min / sigma_max), t1 = the policy degree) on the GPU,
    plus the generated specs (ms, ns, kappas, families)."""
    import torch
    ms, ns, ks, sig, fam = W.training_spectra(count, seed, nmin, nmax, kmin, kmax)
    feats = torch.empty((count, NF), dtype=torch.float64, device="cuda")
    for c0 in range(0, count, chunk):
        c1 = min(count, c0 + chunk)
        ld = max(ns[c0:c1])
        S = np.zeros((c1 - c0, ld))
        for b in range(c0, c1):
            S[b - c0, :ns[b]] = sig[b]
        feats[c0:c1] = z.surrogate_features(torch.from_numpy(S).to("cuda"), ms[c0:c1], ns[c0:c1], feature_seed,
                                            first_index=c0)
    t0 = np.array([math.log10(s[-1] / s[0]) for s in sig])
    t1 = np.array([zolo.choose_r(s[-1] / s[0]) for s in sig], dtype=np.float64)
    T = torch.from_numpy(np.stack([t0, t1], axis=1).astype(np.float32)).to("cuda")
    return feats, T, (ms, ns, ks, fam)


def train(z, feats, T, epochs=60, batch=512, lr=3e-3, seed=0, q=0.05, c_r=0.1, log=None):
    """Adam with a cosine learning-rate decay over `epochs` passes in shuffled
    minibatches.  Returns (params as a float32 device tensor, mean loss per
    epoch)."""
    import torch
    count = feats.shape[0]
    params = torch.from_numpy(init_params(seed)).to("cuda")
    z.mlp_stats(feats, params)
    m = torch.zeros(NPARAMS, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    work = z.mlp_work(batch)
    grad = torch.zeros_like(m)
    rng = np.random.default_rng(seed + 1)
    steps = max(1, count // batch)
    t = 1
    history = []
    for ep in range(epochs):
        order = rng.permutation(count)
        if steps * batch > count:
            order = np.concatenate([order, rng.integers(0, count, steps * batch - count)])
        idx = torch.from_numpy(order[:steps * batch].reshape(steps, batch).astype(np.int32)).to("cuda")
        lr_ep = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * ep / epochs)))
        losses = z.mlp_train(feats, T, idx, params, m, v, t, lr_ep, q, c_r, work, grad)
        t += steps
        history.append(float(np.mean(losses.cpu().numpy())))
        if log:
            log(f"epoch {ep}: lr {lr_ep:.2e} loss {history[-1]:.4f}")
    return params, history


def evaluate(z, params, feats, T, mask=None):
    """Prediction quality on a feature set (optionally the rows where mask
    is true): errors of log10 l, share of over-estimates (10^y0 above the
    true sigma_min / sigma_max), share with the right degree."""
    y, _ = z.mlp_forward(params, feats)
    y = y.cpu().numpy().astype(np.float64)
    t = T.cpu().numpy().astype(np.float64)
    if mask is not None:
        y, t = y[np.asarray(mask, dtype=bool)], t[np.asarray(mask, dtype=bool)]
    err = y[:, 0] - t[:, 0]
    r_pred = np.clip(np.rint(y[:, 1]), 1, 8)
    return {"count": int(t.shape[0]), "median_abs_log10_err": float(np.median(np.abs(err))),
            "p90_abs_log10_err": float(np.quantile(np.abs(err), 0.9)),
            "overestimate_share": float(np.mean(err > 0.0)),
            "overestimate_by_10x_share": float(np.mean(err > 1.0)),
            "r_exact_share": float(np.mean(r_pred == t[:, 1])),
            "r_within_1_share": float(np.mean(np.abs(r_pred - t[:, 1]) <= 1))}
