"""Pins of the learned-estimator oracle (oracle/learned.py) against facts
outside it: the SplitMix64 reference outputs, the normal law, NumPy's SVD,
closed forms for orthonormal and scaled inputs, the distribution of real
sketches of Haar matrices, central finite differences, and closed forms of
the loss and of Adam's first step."""

import math

import numpy as np
import pytest

from oracle import learned as L


def test_splitmix64_reference_outputs():
    # First outputs of SplitMix64 started from state 0, as printed by the
    # reference implementation (Steele, Lea & Flood 2014; Vigna's splitmix64.c).
    got = [int(x) for x in L.splitmix64(0, np.arange(3))]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_gaussian_numbers_are_standard_normal():
    from scipy import stats
    g = L.gaussian(12345, np.arange(200_000, dtype=np.uint64))
    assert abs(g.mean()) < 0.01 and abs(g.var() - 1.0) < 0.01
    assert stats.kstest(g, "norm").statistic < 0.005
    # Different streams and offsets give different numbers.
    assert not np.array_equal(L.gaussian(1, np.arange(8)), L.gaussian(2, np.arange(8)))


def test_features_match_numpy_svd_of_the_sketch():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((90, 70)) @ np.diag(np.logspace(0, -5, 70))
    f = L.features(X, 99)
    Y = X @ L.sketch_matrix(70, 99)
    s = np.linalg.svd(Y, compute_uv=False)
    ref = L.features_from(s, np.linalg.norm(X, axis=0), np.linalg.norm(X, axis=1), 90, 70, np.linalg.norm(X))
    assert np.abs(f - ref).max() <= 1e-10
    assert f[0] == pytest.approx(math.log10(s[0]), abs=1e-12)
    assert f[36] == pytest.approx(math.log10(70)) and f[37] == pytest.approx(math.log10(90 / 70))
    cn = np.log10(np.linalg.norm(X, axis=0))
    assert f[32] == pytest.approx(cn.mean(), abs=1e-12) and f[33] == pytest.approx(cn.std(), abs=1e-12)


def test_features_of_orthonormal_columns_and_scaling():
    rng = np.random.default_rng(1)
    Q = np.linalg.qr(rng.standard_normal((80, 40)))[0]
    f = L.features(Q, 5)
    assert abs(f[32]) < 1e-12 and abs(f[33]) < 1e-12          # unit columns
    assert abs(f[38]) < 1e-12                                   # ||Q||_F = sqrt(n)
    # A scale c shifts the absolute logs by log10 c and leaves the rest.
    g = L.features(1e-3 * Q, 5)
    shift = np.zeros(L.NF)
    shift[[0, 32, 34, 38]] = -3.0
    assert np.abs(g - (f + shift)).max() < 1e-9


def test_surrogate_has_the_law_of_real_sketches():
    # G4: for Haar U, V the sketch features of U diag(sigma) V^T and the
    # surrogate built from sigma alone have the same distribution.  Compare
    # the means of all features over independent draws (4 standard errors).
    from paper_1806_06204_amd import workloads as W
    m, n, N = 60, 40, 80
    sigma = np.logspace(0, -6, n)
    real = np.array([L.features(W.svd_matrix(m, n, 1.0, 50 + i, 500 + i, sigma=sigma)[0], 7000 + i)
                     for i in range(N)])
    sur = np.array([L.surrogate_features(sigma, m, 31, i) for i in range(N)])
    se = np.sqrt(real.var(axis=0) / N + sur.var(axis=0) / N) + 1e-12
    z = np.abs(real.mean(axis=0) - sur.mean(axis=0)) / se
    assert z.max() < 4.0, (np.argmax(z), z.max())


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    p = L.init_params(3, mu=rng.standard_normal(L.NF), sd=rng.uniform(0.5, 2.0, L.NF))
    F = rng.standard_normal((5, L.NF))
    T = np.stack([rng.uniform(-16, 0, 5), rng.integers(1, 9, 5)], axis=1).astype(float)

    def total(pp):
        y, _ = L.forward(pp, F)
        return L.loss(y, T)[0]

    y, cache = L.forward(p, F)
    _, dy = L.loss(y, T)
    g = L.backward(p, cache, dy)
    assert np.all(g[:L.N_STATS] == 0.0)
    h = 1e-6
    idx = np.arange(L.N_STATS, L.N_PARAMS)
    fd = np.empty(idx.size)
    for t, i in enumerate(idx):
        e = np.zeros(L.N_PARAMS)
        e[i] = h
        fd[t] = (total(p + e) - total(p - e)) / (2 * h)
    assert np.abs(g[idx] - fd).max() <= 1e-6 * max(1.0, np.abs(fd).max())


def test_loss_closed_forms():
    # One sample: over-estimate by 1 costs (1 - q), under-estimate by 1 costs q.
    L_over, d_over = L.loss(np.array([[1.0, 3.0]]), np.array([[0.0, 3.0]]), q=0.1)
    L_under, d_under = L.loss(np.array([[-1.0, 3.0]]), np.array([[0.0, 3.0]]), q=0.1)
    assert L_over == pytest.approx(0.9) and L_under == pytest.approx(0.1)
    assert d_over[0, 0] == pytest.approx(1.8) and d_under[0, 0] == pytest.approx(-0.2)
    L_r, d_r = L.loss(np.array([[0.0, 5.0]]), np.array([[0.0, 3.0]]), c_r=0.1)
    assert L_r == pytest.approx(0.4) and d_r[0, 1] == pytest.approx(0.4)


def test_adam_first_step_closed_form():
    # At t = 1 the bias corrections give m_hat = g and v_hat = g^2, so each
    # trainable parameter moves by -lr g / (|g| + eps).
    rng = np.random.default_rng(4)
    p = rng.standard_normal(L.N_PARAMS)
    g = rng.standard_normal(L.N_PARAMS)
    z = np.zeros(L.N_PARAMS)
    p1, m1, v1 = L.adam_step(p, g, z, z, 1, 1e-2)
    s = slice(L.N_STATS, None)
    assert np.allclose(p1[s], p[s] - 1e-2 * g[s] / (np.abs(g[s]) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.array_equal(p1[:L.N_STATS], p[:L.N_STATS])
    assert np.allclose(m1[s], 0.1 * g[s]) and np.allclose(v1[s], 0.001 * g[s] ** 2)


def test_predict_clamps_and_layout():
    assert L.N_PARAMS == 6928
    p = np.zeros(L.N_PARAMS)
    P = L.unpack(p)
    P["sd"][:] = 1.0
    P["b3"][:] = [5.0, 11.7]       # 10^5 > 1 and r > 8 clamp
    assert L.predict(p, np.zeros(L.NF)) == (1.0, 8)
    P["b3"][:] = [-40.0, 0.2]
    assert L.predict(p, np.zeros(L.NF)) == (1e-20, 1)
    P["b3"][:] = [-6.0, 4.4]
    l, r = L.predict(p, np.zeros(L.NF))
    assert l == pytest.approx(1e-6) and r == 4


def _random_params(seed):
    rng = np.random.default_rng(seed)
    p = L.init_params(seed + 1, mu=rng.standard_normal(L.NF), sd=rng.uniform(0.3, 3.0, L.NF))
    P = L.unpack(p)
    for b in ("b1", "b2", "b3"):
        P[b][:] = rng.uniform(-0.5, 0.5, P[b].shape)
    return p


def test_forward_matches_torch_modules_in_float64():
    # G5 against an independent implementation: torch.nn.Linear / tanh layers
    # in float64 holding the same weights (nn.Linear computes x W^T + b with W
    # of shape (out, in), the layout W1[o][i] of the flat vector).
    import torch
    p = _random_params(40)
    P = L.unpack(p)
    F = np.random.default_rng(41).standard_normal((7, L.NF)) * 3.0
    net = torch.nn.Sequential(torch.nn.Linear(L.NF, L.NH), torch.nn.Tanh(), torch.nn.Linear(L.NH, L.NH),
                              torch.nn.Tanh(), torch.nn.Linear(L.NH, L.NO)).double()
    with torch.no_grad():
        for lin, w, b in ((net[0], "W1", "b1"), (net[2], "W2", "b2"), (net[4], "W3", "b3")):
            lin.weight.copy_(torch.from_numpy(P[w].copy()))
            lin.bias.copy_(torch.from_numpy(P[b].copy()))
        x = (torch.from_numpy(F) - torch.from_numpy(P["mu"].copy())) / torch.from_numpy(P["sd"].copy())
        ref = net(x).numpy()
    y, cache = L.forward(p, F)
    assert np.abs(y - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())
    assert np.abs(cache["x"] - x.numpy()).max() == 0.0


def test_forward_hand_worked_example():
    # One path through the network, worked out by hand: x0 = (f0 - mu0)/sd0
    # = (1.5 - 0.5)/0.5 = 2; h1_0 = tanh(1 * 2 + 0.5); every other h1 is
    # tanh(0) = 0; h2_1 = tanh(2 h1_0 - 0.25), h2_0 = tanh(-0.25);
    # y0 = 3 h2_1 + 0.25, y1 = -h2_0 + 4.  Dividing by sd the other way,
    # dropping a bias or transposing W2 or W3 (off-diagonal entries) changes
    # the numbers.
    p = np.zeros(L.N_PARAMS)
    P = L.unpack(p)
    P["mu"][:] = 0.0
    P["sd"][:] = 1.0
    P["mu"][0], P["sd"][0] = 0.5, 0.5
    P["W1"][0, 0] = 1.0
    P["b1"][0] = 0.5
    P["W2"][1, 0] = 2.0
    P["b2"][:2] = -0.25
    P["W3"][0, 1] = 3.0
    P["W3"][1, 0] = -1.0
    P["b3"][:] = [0.25, 4.0]
    f = np.zeros(L.NF)
    f[0] = 1.5
    f[5] = 7.0            # W1[:, 5] = 0: no influence
    y, _ = L.forward(p, f[None, :])
    h1 = math.tanh(2.5)
    assert y[0, 0] == pytest.approx(3.0 * math.tanh(2.0 * h1 - 0.25) + 0.25, abs=1e-15)
    assert y[0, 1] == pytest.approx(-math.tanh(-0.25) + 4.0, abs=1e-15)


def test_standardize_stats_closed_forms():
    # Population statistics (divide by the number of samples, not one less)
    # with sd floored at 1e-6 for a constant feature.
    F = np.array([[0.0, 2.0, 5.0], [2.0, 2.0, 1.0], [4.0, 2.0, 3.0], [6.0, 2.0, 7.0]])
    mu, sd = L.standardize_stats(F)
    assert np.array_equal(mu, [3.0, 2.0, 4.0])
    assert sd[0] == pytest.approx(math.sqrt(5.0), abs=1e-15)    # (9+1+1+9)/4
    assert sd[1] == 1e-6
    assert sd[2] == pytest.approx(math.sqrt(5.0), abs=1e-15)    # (1+9+1+9)/4
    # Standardised features then have mean 0 and population variance 1.
    X = (F[:, [0, 2]] - mu[[0, 2]]) / sd[[0, 2]]
    assert np.abs(X.mean(axis=0)).max() == 0.0
    assert np.allclose((X * X).mean(axis=0), 1.0, rtol=1e-15)
