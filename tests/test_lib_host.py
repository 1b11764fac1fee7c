"""CPU-side checks of the native library: it loads, exports every symbol the
headers declare, and its host-only coefficient routine (zolo_coeffs) agrees
with the oracle.  No GPU work is launched here."""

import os
import re

import numpy as np
import pytest

from oracle import coeffs as oc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in ("zolo.h", "zolo_blocks.h", "zolo_stats.h", "zolo_learn.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        names += re.findall(r"^\s*(?:int|void|long long)\s+(zolo_\w+)\s*\(", txt, flags=re.M)
    return names


@pytest.fixture(scope="module")
def lib():
    from paper_1806_06204_amd import zolo
    if not os.path.exists(zolo.LIB_PATH):
        pytest.skip("libzolo.so not built")
    return zolo.load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def test_binding_lists_all_declared(lib):
    from paper_1806_06204_amd import zolo
    assert sorted(declared_functions()) == sorted(zolo.EXPORTS)


@pytest.mark.parametrize("r", [1, 2, 3, 5, 8])
def test_coeffs_match_oracle(lib, r):
    from paper_1806_06204_amd import zolo
    for l in [1e-20, 1e-16, 1e-8, 1e-3, 0.2, 0.7, 0.71, 0.95, 1 - 1e-12, 1.0]:
        got = zolo.coeffs(l, r)
        ref = oc.coefficients(l, r)
        assert np.allclose(got["c"], ref["c"], rtol=2e-14, atol=0), (l, r)
        assert np.allclose(got["a"], ref["a"], rtol=1e-12, atol=0), (l, r)
        assert got["mhat"] == pytest.approx(ref["mhat"], rel=1e-13)
        assert abs((1 - got["l_next"]) - (1 - ref["l_next"])) <= 1e-13 * max(1e-300, 1 - ref["l_next"]) + 4e-16


def test_coeffs_rejects_bad_arguments(lib):
    from paper_1806_06204_amd import zolo
    with pytest.raises(ValueError):
        zolo.coeffs(0.0, 3)
    with pytest.raises(ValueError):
        zolo.coeffs(0.5, 9)
    with pytest.raises(ValueError):
        zolo.coeffs(1.5, 2)


def test_table1_through_library(lib):
    # The library's l-update reproduces the paper's Table 1 as well.
    import json
    from paper_1806_06204_amd import zolo
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "table1_iterations.json")))
    for rs, row in g["iterations"].items():
        got = []
        for kap in g["kappa"]:
            l, k = 1.0 / kap, 0
            while l < 1 - 1e-15 and k < 20:
                l = zolo.coeffs(l, int(rs))["l_next"]
                k += 1
            got.append(k)
        assert got == row, rs


def test_choose_r_matches_oracle_policy(lib):
    from paper_1806_06204_amd import zolo
    for l in [1e-20, 1e-16, 1e-12, 1e-8, 1e-4, 0.01, 0.3, 0.9, 1.0]:
        assert zolo.choose_r(l) == oc.choose_r(l), l


def test_learned_layout_constants(lib):
    from oracle import learned as OL
    from paper_1806_06204_amd import zolo
    assert (zolo.NF, zolo.MLP_NPARAMS, zolo.MLP_NSTATS) == (OL.NF, OL.N_PARAMS, OL.N_STATS)
    assert lib.zolo_mlp_work_elems(100) >= (OL.NF + 4 * OL.NH) * 100


def test_autotune_switch_is_host_only(lib):
    # Turning the GEMM tile autotuner on and off and forgetting its choices
    # touch only host state (no device is needed); both calls return 0.
    assert lib.zolo_autotune_enable(1) == 0
    assert lib.zolo_autotune_reset() == 0
    assert lib.zolo_autotune_enable(0) == 0
    assert lib.zolo_autotune_reset() == 0


def _oracle_kinds(l, r, chol_switch=100.0):
    from oracle import zolo as oz
    kinds = []
    while len(kinds) < 16:
        co = oc.coefficients(l, r)
        kinds.append(oz.step_kind(l, co["c"], chol_switch))
        l = co["l_next"]
        if l >= oc.CONVERGED:
            break
    return "".join(kinds)


def test_predicted_schedule_matches_oracle_rules(lib):
    # zolo_predict follows the solve's own step rules (R6 step kind, the
    # l-update of eqs. (7)-(10)); the schedules equal the oracle's scalar
    # recursion (no verified re-estimate happens when l is exact).
    from paper_1806_06204_amd import zolo
    for l in [1e-16, 1e-12, 1e-8, 1e-4, 0.1, 0.9]:
        for r in range(1, 9):
            kinds, ms = zolo.predict(l, r, 8192, 8192)
            assert kinds == _oracle_kinds(l, r), (l, r)
            assert ms > 0.0
    # QDWH (r = 1) at kappa = 1e16 takes two QR-type and four Cholesky-type steps.
    assert zolo.predict(1e-16, 1, 8192, 8192)[0] == "QQCCCC"
    with pytest.raises(ValueError):
        zolo.predict(0.0, 3, 10, 10)
    with pytest.raises(ValueError):
        zolo.predict(0.5, 9, 10, 10)
    with pytest.raises(ValueError):
        zolo.predict(0.5, 3, 5, 10)


def test_predicted_time_grows_with_work(lib):
    # The cost model prices flops: more columns, more rows or another step
    # never make a solve cheaper.
    from paper_1806_06204_amd import zolo
    for r in (1, 3, 8):
        t1 = zolo.predict(1e-8, r, 2048, 1024)[1]
        t2 = zolo.predict(1e-8, r, 4096, 1024)[1]
        t3 = zolo.predict(1e-8, r, 4096, 2048)[1]
        assert t1 < t2 < t3
    assert zolo.predict(1e-16, 3, 4096, 4096)[1] >= zolo.predict(1e-4, 3, 4096, 4096)[1]


def test_release_events_is_host_only(lib):
    # With no statistics or autotuner events alive, releasing them touches
    # no device; recording can start again afterwards.
    assert lib.zolo_release_events() == 0
    assert lib.zolo_release_events() == 0
