"""Pins for the oracle's Zolotarev coefficients (Section 2.2 of the paper).

Each test ties oracle.coeffs to something other than itself: the paper's
Table 1, 80-digit mpmath elliptic functions, the QDWH closed form for r = 1,
the l -> 1 limit, the partial-fraction identity of Theorem 2.1 and the
equioscillation property that defines the Zolotarev function (eqs. (5)-(6)).
"""

import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import coeffs as zc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_iterations.json")
LS = [1e-20, 1e-16, 1e-12, 1e-8, 1e-4, 1e-2, 0.1, 0.5, 0.7, 0.7072, 0.9, 0.99,
      1 - 1e-8, 1 - 1e-15]


def mp_coeffs(l, r, dps=80):
    """c_i of eq. (7) straight from mpmath's sn, cn and K at high precision."""
    with mp.workdps(dps):
        l = mp.mpf(l)
        m = 1 - l * l                      # parameter of modulus l'
        kp = mp.ellipk(m)                  # K' = K(l')
        out = []
        for i in range(1, 2 * r + 1):
            u = i * kp / (2 * r + 1)
            sn = mp.ellipfun("sn", u, m=m)
            cn = mp.ellipfun("cn", u, m=m)
            out.append(l * l * sn * sn / (cn * cn))
        return out


def mp_one_minus_zhat_l(l, r, dps=80):
    with mp.workdps(dps):
        c = mp_coeffs(l, r, dps)
        l = mp.mpf(l)
        mh = mp.mpf(1)
        z = l
        for j in range(r):
            mh *= (1 + c[2 * j]) / (1 + c[2 * j + 1])
            z *= (l * l + c[2 * j + 1]) / (l * l + c[2 * j])
        return 1 - mh * z


def test_table1_all_cells():
    g = json.load(open(GOLDEN))
    for rs, row in g["iterations"].items():
        got = [zc.iterations_to_converge(k, int(rs)) for k in g["kappa"]]
        assert got == row, (rs, got, row)


@pytest.mark.parametrize("r", [1, 2, 3, 5, 8])
def test_c_against_mpmath(r):
    worst = 0.0
    for l in LS:
        c = zc.zolo_c(l, r)
        ref = mp_coeffs(l, r)
        for i in range(2 * r):
            worst = max(worst, abs(c[i] - float(ref[i])) / float(ref[i]))
    assert worst <= 1e-14, worst


def test_reflection_identity_mpmath():
    # c_i c_{2r+1-i} = l^2 (sn(K'-u) = cd(u), cn(K'-u) = l sd(u) for modulus l').
    for l in [1e-10, 0.3, 0.9]:
        for r in [2, 4]:
            ref = mp_coeffs(l, r, 60)
            for i in range(r):
                with mp.workdps(60):
                    ratio = ref[i] * ref[2 * r - 1 - i] / (mp.mpf(l) ** 2)
                    assert abs(ratio - 1) < mp.mpf("1e-40")


def qdwh_abc(l):
    """Dynamically weighted Halley parameters (a, b, c) in closed form."""
    g = (4.0 * (1.0 - l * l) / l ** 4) ** (1.0 / 3.0)
    a = math.sqrt(1.0 + g) + 0.5 * math.sqrt(8.0 - 4.0 * g + 8.0 * (2.0 - l * l) / (l * l * math.sqrt(1.0 + g)))
    b = (a - 1.0) ** 2 / 4.0
    return a, b, a + b - 1.0


@pytest.mark.parametrize("l", [1e-6, 1e-3, 0.05, 0.3, 0.6, 0.9])
def test_r1_is_qdwh(l):
    # x(a + b x^2)/(1 + c x^2) = (b/c) x (x^2 + a/b)/(x^2 + 1/c)  (Section 2.2, eq. (5)).
    a, b, c = qdwh_abc(l)
    co = zc.coefficients(l, 1)
    assert co["c"][0] == pytest.approx(1.0 / c, rel=1e-10)
    assert co["c"][1] == pytest.approx(a / b, rel=1e-10)
    assert co["mhat"] == pytest.approx(b / c, rel=1e-10)


@pytest.mark.parametrize("r", [1, 3, 8])
def test_l_to_one_limit(r):
    t = [math.tan(i * math.pi / (2 * (2 * r + 1))) ** 2 for i in range(1, 2 * r + 1)]
    assert np.allclose(zc.zolo_c(1.0, r), t, rtol=1e-14, atol=0)
    assert np.allclose(zc.zolo_c(1 - 1e-13, r), t, rtol=1e-11, atol=0)


@pytest.mark.parametrize("r", [1, 2, 3, 4, 6, 8])
def test_partial_fractions_and_positivity(r):
    # Theorem 2.1: product form (8) equals partial fractions (9); a_j > 0.
    for l in [1e-16, 1e-8, 1e-3, 0.2, 0.8]:
        co = zc.coefficients(l, r)
        assert np.all(co["a"] > 0)
        assert np.all(np.diff(co["c"]) > 0)
        x = np.concatenate([np.geomspace(l, 1.0, 400), [1.3, 2.0]])
        p = zc.zhat(x, co["c"], co["mhat"])
        s = zc.zhat_partial_fractions(x, co["c"], co["a"], co["mhat"])
        assert np.max(np.abs(p - s) / np.abs(p)) < 1e-12
        assert zc.zhat(1.0, co["c"], co["mhat"]) == pytest.approx(1.0, abs=4e-16)


def test_product_of_printed_aj_fails_identity():
    # The product printed in eq. (10) does not satisfy eq. (9): documents the reading.
    co = zc.coefficients(1e-4, 3)
    c = co["c"]
    r = 3
    bad = []
    for j in range(1, r + 1):
        p1 = np.prod([c[2 * j - 2] - c[2 * k - 1] for k in range(1, r + 1)])
        p2 = np.prod([c[2 * j - 2] - c[2 * k - 2] for k in range(1, r + 1) if k != j])
        bad.append(-p1 * p2)
    x = np.geomspace(1e-4, 1, 50)
    p = zc.zhat(x, c, co["mhat"])
    s = zc.zhat_partial_fractions(x, c, np.array(bad), co["mhat"])
    assert np.max(np.abs(p - s) / p) > 1e-3


def extrema(f, lo, hi, npts=200001):
    x = np.geomspace(lo, hi, npts)
    y = f(x)
    idx = [0]
    for k in range(1, npts - 1):
        if (y[k] - y[k - 1]) * (y[k + 1] - y[k]) < 0:
            idx.append(k)
    idx.append(npts - 1)
    return x[idx], y[idx]


@pytest.mark.parametrize("l,r", [(1e-8, 3), (1e-2, 2), (0.5, 1), (1e-4, 4)])
def test_equioscillation(l, r):
    # eqs. (5)-(6): on [l, 1] the best approximation alternates 2r+2 times
    # between Zhat(l) (minima) and 1 (maxima).
    co = zc.coefficients(l, r)
    zl = float(zc.zhat(l, co["c"], co["mhat"]))
    assert 1.0 - zl > 1e-6
    xs, ys = extrema(lambda x: zc.zhat(x, co["c"], co["mhat"]), l, 1.0)
    assert len(xs) == 2 * r + 2
    mins = ys[0::2]
    maxs = ys[1::2]
    dev = 1.0 - zl
    assert np.all(np.abs(mins - zl) < 1e-6 * dev + 1e-12)
    assert np.all(np.abs(maxs - 1.0) < 1e-6 * dev + 1e-12)


@pytest.mark.parametrize("r", [1, 2, 4, 7, 8])
def test_l_next_against_mpmath(r):
    for l in [1e-16, 1e-8, 1e-3, 0.1, 0.5, 0.9]:
        ref = float(mp_one_minus_zhat_l(l, r))
        got = 1.0 - zc.coefficients(l, r)["l_next"]
        if ref < 1e-3:
            got = zc.one_minus_l_next(l, r)
            assert abs(got - ref) <= 1e-12 * ref + 1e-300, (l, r, got, ref)
        else:
            assert abs(got - ref) <= 1e-13, (l, r, got, ref)


def test_choose_r_policy_matches_table1():
    # The smallest r with at most two iterations, read off Table 1 columns.
    assert zc.choose_r(1 / 10) == 3
    assert zc.choose_r(1 / 1e3) == 4
    assert zc.choose_r(1 / 1e5) == 5
    assert zc.choose_r(1 / 1e7) == 6
    assert zc.choose_r(1e-16) == 8
    assert zc.choose_r(1 / 1.001) == 1


def test_domain_errors():
    with pytest.raises(ValueError):
        zc.zolo_c(0.0, 3)
    with pytest.raises(ValueError):
        zc.zolo_c(0.5, 0)
    with pytest.raises(ValueError):
        zc.zolo_c(1.5, 2)
