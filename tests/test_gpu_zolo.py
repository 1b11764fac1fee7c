"""End-to-end GPU parity of Zolo-PD / Zolo-SVD (C ABI) against the CPU oracle.

Bar (FP64): backward error ||A - Qp H||_F / ||A||_F <= 1e-13 and
||Qp^T Qp - I||_F / sqrt(n) <= 1e-13, the same step kinds as the oracle, and
||H - H_oracle||_F / ||H_oracle||_F <= 1e-12 (H is well conditioned: a
perturbation of A moves H by at most sqrt(2) times as much).  Qp itself is
compared only where the polar factor is well posed (kappa <= 1e8), with a
tolerance of kappa * 1e-15 per sqrt(n).
"""

import math

import numpy as np
import pytest

from oracle import zolo as oz
from paper_1806_06204_amd import workloads as W

pytestmark = pytest.mark.gpu
BAR = 1e-13


@pytest.fixture(scope="module")
def z():
    import torch
    from paper_1806_06204_amd import zolo
    assert torch.cuda.is_available()
    h = zolo.Zolo()
    yield h
    h.close()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def same_schedule(info, io, tau=5e-14):
    """Step kinds follow from identical host scalars and must agree.  The only
    rounding-dependent decision is the verified stop ||X^T X - I||_F/sqrt(n) <= tau:
    when one side needs one more step, the oracle's check taken after the
    last common step (the one where the two diverge) must have been within a
    factor 10 of tau."""
    g, o = info["kinds"], io["kinds"]
    k = min(len(g), len(o))
    assert g[:k] == o[:k]
    if len(g) != len(o):
        assert abs(len(g) - len(o)) == 1, (g, o)
        at = [d for d, i in zip(io["orth_checks"], io["check_iters"]) if i == k - 1]
        assert at and 0.1 * tau <= at[0] <= 10 * tau, (io["orth_checks"], io["check_iters"], k)


def run_and_compare(z, A, alpha, l, r, kappa=None, h_tol=1e-12, **opts):
    Qp, H, info = z.pd(dev(A), alpha=alpha, l=l, r=r, compute_errors=1, **opts)
    Qp, H = Qp.cpu().numpy(), H.cpu().numpy()
    oopts = {}
    if opts.get("stop_rule") in (1, "paper"):
        oopts["stop"] = "paper"
    if "chol_switch" in opts:
        oopts["chol_switch"] = opts["chol_switch"]
    Qo, Ho, io = oz.zolo_pd(A, alpha, l, r, **oopts)
    bwd = oz.backward_error(A, Qp, H)
    orth = oz.orthogonality(Qp)
    dh = np.linalg.norm(H - Ho) / np.linalg.norm(Ho)
    print(f"  gpu kinds={''.join(info['kinds'])} oracle={''.join(io['kinds'])} bwd={bwd:.2e} orth={orth:.2e} "
          f"dH={dh:.2e} lib bwd={info['bwd_err']:.2e} orth={info['orth_err']:.2e}", flush=True)
    assert info["status"] == 0
    same_schedule(info, io)
    assert bwd <= BAR and orth <= BAR
    assert abs(info["bwd_err"] - bwd) <= 1e-15 + 0.1 * bwd
    assert dh <= h_tol
    if kappa is not None and kappa <= 1e8:
        dq = np.linalg.norm(Qp - Qo) / math.sqrt(A.shape[1])
        assert dq <= max(1e-13, kappa * 1e-15), dq
    return info, io


def test_small_config(z):
    cfg = W.config_small()
    info, io = run_and_compare(z, cfg["A"], cfg["alpha"], cfg["l"], cfg["r"], kappa=1e8)
    assert info["kinds"] == ["Q", "C", "C"]
    assert np.allclose(info["ls"], io["ls"], rtol=1e-12)


def test_cholesky_only_schedule(z):
    A = W.svd_matrix(256, 128, 10.0, 1100, 2100)[0]
    info, _ = run_and_compare(z, A, 1.0, 0.1, 3, kappa=10.0)
    assert set(info["kinds"]) == {"C"}


def test_paper_stop_rule(z):
    cfg = W.config_small()
    run_and_compare(z, cfg["A"], 1.0, cfg["l"], 3, kappa=1e8, stop_rule=1)


@pytest.mark.parametrize("m,n,kappa,r", [(200, 77, 1e4, 2), (65, 65, 1e6, 4), (130, 1, 1.0, 1),
                                         (300, 150, 1e12, 5), (96, 96, 1e16, 8)])
def test_ragged_shapes(z, m, n, kappa, r):
    A = W.svd_matrix(m, n, kappa, 1200 + m, 2200 + n)[0]
    run_and_compare(z, A, 1.0, 1.0 / kappa, r, kappa=kappa)


def test_kappa_1e16_n512(z):
    A = W.svd_matrix(512, 512, 1e16, 1300, 2300)[0]
    info, io = run_and_compare(z, A, 1.0, 1e-16, 8)
    assert info["kinds"][:2] == ["Q", "C"]


def host_errors(A, Qp, H):
    """Backward error and orthogonality recomputed on the host in FP64 (torch
    CPU products, independent of the library's GEMM)."""
    import torch
    At, Qt, Ht = (torch.from_numpy(np.ascontiguousarray(x)) for x in (A, Qp, H))
    bwd = float(torch.linalg.norm(At - Qt @ Ht) / torch.linalg.norm(At))
    n = Qt.shape[1]
    orth = float(torch.linalg.norm(Qt.T @ Qt - torch.eye(n, dtype=torch.float64)) / math.sqrt(n))
    return bwd, orth


def exact_h_error(H, sigma, V):
    """||H - V diag(sigma) V^T||_F / ||V diag(sigma) V^T||_F on the host (the
    polar factor H of A = U diag(sigma) V^T is known exactly)."""
    import torch
    Vt = torch.from_numpy(np.ascontiguousarray(V))
    Hx = (Vt * torch.from_numpy(sigma)) @ Vt.T
    return float(torch.linalg.norm(torch.from_numpy(np.ascontiguousarray(H)) - Hx) / torch.linalg.norm(Hx))


def test_many_panel_workgroups(z):
    # n = 4096, r = 4: the QR step's panels (4160 live rows) run 29 LDS-slab
    # workgroups per matrix (the per-matrix cap), 116 in all, with every
    # column's exchange across them.  H is compared with the exact
    # V diag(sigma) V^T and the errors are recomputed on the host.
    A, U, sig, V = W.svd_matrix(4096, 4096, 1e12, 1400, 2400)
    Qp, H, info = z.pd(dev(A), alpha=1.0, l=1e-12, r=4, compute_errors=1)
    Qp, H = Qp.cpu().numpy(), H.cpu().numpy()
    bwd, orth = host_errors(A, Qp, H)
    dh = exact_h_error(H, sig, V)
    print(f"  kinds={''.join(info['kinds'])} bwd={bwd:.2e} orth={orth:.2e} dH_exact={dh:.2e}", flush=True)
    assert info["status"] == 0 and info["kinds"][0] == "Q"
    assert bwd <= BAR and orth <= BAR and dh <= 1e-12
    assert abs(info["bwd_err"] - bwd) <= 1e-15 + 0.1 * bwd


def test_headline_config_full_h(z):
    # The benchmarked solve: 8192 x 8192, kappa = 1e16, r = 8, alpha = 1,
    # l = 1e-16, FP64.  The whole H against V diag(sigma) V^T (H is
    # well conditioned: its error is at most sqrt(2) times the backward
    # error), and the backward error and orthogonality of Qp recomputed on
    # the host in FP64.
    cfg = W.config_large()
    A = cfg["A"]
    print("  8192^2 kappa=1e16 r=8: solving", flush=True)
    Qp, H, info = z.pd(dev(A), alpha=1.0, l=cfg["l"], r=cfg["r"], compute_errors=1)
    Qp, H = Qp.cpu().numpy(), H.cpu().numpy()
    bwd, orth = host_errors(A, Qp, H)
    dh = exact_h_error(H, cfg["sigma"], cfg["V"])
    print(f"  kinds={''.join(info['kinds'])} checks={info['checks']} bwd={bwd:.2e} orth={orth:.2e} "
          f"dH_exact={dh:.2e} (library bwd={info['bwd_err']:.2e} orth={info['orth_err']:.2e})", flush=True)
    assert info["status"] == 0 and info["kinds"][:2] == ["Q", "C"]
    assert bwd <= BAR and orth <= BAR
    assert dh <= 1e-12
    assert abs(info["bwd_err"] - bwd) <= 1e-15 + 0.1 * bwd


def test_estimated_alpha_and_l(z):
    A = W.sparse_pattern(256, bandwidth=16, p=0.01, seed=3001)
    Qp, H, info = z.pd(dev(A), compute_errors=1)
    Qo, Ho, io = oz.zolo_pd(A)
    assert info["status"] == 0
    assert info["alpha"] == pytest.approx(io["alpha"], rel=1e-8)
    assert info["l0"] == pytest.approx(io["l0"], rel=1e-6)
    assert info["r"] == io["r"]
    Qp, H = Qp.cpu().numpy(), H.cpu().numpy()
    assert oz.backward_error(A, Qp, H) <= BAR and oz.orthogonality(Qp) <= BAR
    assert np.linalg.norm(H - Ho) / np.linalg.norm(Ho) <= 1e-12


def test_failure_modes(z):
    cfg = W.config_small()
    Qp, H, info = z.pd(dev(cfg["A"]), alpha=1.0, l=cfg["l"], r=3, max_iter=1, check=False)
    assert info["status"] == 1 and info["iters"] == 1
    bad = cfg["A"].copy()
    bad[3, 4] = np.inf
    _, _, info = z.pd(dev(bad), alpha=1.0, l=1e-8, r=3, check=False)
    assert info["status"] == 2
    with pytest.raises(ValueError):
        z.pd(dev(cfg["A"].T), alpha=1.0, l=1e-8, r=3)
    with pytest.raises(ValueError):
        z.pd(dev(cfg["A"]), alpha=1.0, l=1e-8, r=9)
    # Exactly rank deficient: the polar factor is not unique.  In exact
    # arithmetic the zero column stays zero and the orthogonality check never
    # passes (status 1, as the oracle reports); rounding in the null direction,
    # amplified once l is re-estimated at 1e-20, may instead fill it with a
    # unit vector orthogonal to range(A), which is a valid polar factor.
    A = W.svd_matrix(40, 20, 10.0, 71, 72)[0]
    A[:, 7] = 0.0
    Qp, H, info = z.pd(dev(A), alpha=1.0, l=1e-3, r=3, check=False, compute_errors=1)
    assert info["status"] in (0, 1)
    if info["status"] == 0:
        assert info["bwd_err"] <= BAR and info["orth_err"] <= BAR
    else:
        assert info["orth_check"] > 0.1


def test_forced_cholesky_breakdown_falls_back(z):
    A = W.svd_matrix(100, 100, 1e16, 1400, 2400)[0]
    Qp, H, info = z.pd(dev(A), alpha=1.0, l=1e-16, r=8, chol_switch=1e300, compute_errors=1)
    assert info["chol_fallbacks"] >= 1 and info["kinds"][0] == "Q"
    assert info["status"] == 0 and info["bwd_err"] <= BAR and info["orth_err"] <= BAR


def test_svd(z):
    A, U, s, V = W.svd_matrix(90, 60, 1e6, 1500, 2500)
    Uc, S, Vc, info = z.svd(dev(A), alpha=1.0, l=1e-6, r=4)
    Uc, Vc = Uc.cpu().numpy(), Vc.cpu().numpy()
    assert info["status"] == 0
    assert np.allclose(S, s, rtol=1e-10, atol=1e-14)   # eigenvalues: absolute error ~ eps ||H||
    res, ol, orr = oz.svd_residual_paper(A, Uc, S, Vc), oz.orth_paper(Uc), oz.orth_paper(Vc)
    print(f"  svd res={res:.2e} OrthL={ol:.2e} OrthR={orr:.2e}", flush=True)
    assert res <= 1e-13
    # OrthL / OrthR below 1.0e-15, the bound the paper reports (Section 4.1).
    assert ol <= 1e-15 and orr <= 1e-15


def test_batched_uneven(z):
    # Many matrices of different shapes, kappa and degree in one call.
    specs = W.batch_specs(count=12, seed=4100, nmin=20, nmax=140, kmin=2.0, kmax=12.0)
    mats = [W.svd_matrix(sp["m"], sp["n"], sp["kappa"], sp["seed_u"], sp["seed_v"])[0] for sp in specs]
    ls = [1.0 / sp["kappa"] for sp in specs]
    rs = [None] * len(specs)
    from oracle import coeffs as oc
    rs = [oc.choose_r(l) for l in ls]
    Qs, Hs, infos = z.pd_batched([dev(A) for A in mats], alphas=[1.0] * len(mats), ls=ls, rs=rs)
    for A, Q, H, inf, l, r in zip(mats, Qs, Hs, infos, ls, rs):
        Q, H = Q.cpu().numpy(), H.cpu().numpy()
        Qo, Ho, io = oz.zolo_pd(A, 1.0, l, r)
        assert inf["status"] == 0
        same_schedule(inf, io)
        assert oz.backward_error(A, Q, H) <= BAR and oz.orthogonality(Q) <= BAR
        assert np.linalg.norm(H - Ho) / np.linalg.norm(Ho) <= 1e-12


def test_batched_mid_sizes(z):
    # Matrices of the 512-matrix uneven workload with n = 600..1000 (one
    # workgroup per panel, the leaf held in registers and LDS), solved in one
    # batched call.  Exact H = V diag(sigma) V^T is known from the
    # construction.
    specs = W.batch_specs(count=512, seed=4000)
    pick = [specs[i] for i in (127, 143, 195, 268)]
    built = [W.svd_matrix(sp["m"], sp["n"], sp["kappa"], sp["seed_u"], sp["seed_v"]) for sp in pick]
    ls = [1.0 / sp["kappa"] for sp in pick]
    Qs, Hs, infos = z.pd_batched([dev(b[0]) for b in built], alphas=[1.0] * len(pick), ls=ls)
    for (A, U, sig, V), Q, H, inf in zip(built, Qs, Hs, infos):
        Q, H = Q.cpu().numpy(), H.cpu().numpy()
        assert inf["status"] == 0, inf
        assert oz.backward_error(A, Q, H) <= BAR and oz.orthogonality(Q) <= BAR
        Hx = (V * sig) @ V.T
        assert np.linalg.norm(H - Hx) / np.linalg.norm(Hx) <= 1e-12


def test_batched_resident_leaf_boundaries(z):
    # Single-workgroup panels of the many-matrix call keep a thread's first
    # 3 rows (1536 rows in all) of each 16-column leaf in registers and the
    # rest in LDS.  Live rows m + 64 just below, at and above that boundary,
    # at the 2304-row limit of single-workgroup panels, with a ragged last
    # leaf (n = 40) and a ragged second panel (n = 70), against the oracle.
    cases = [(1471, 40, 1e6), (1472, 70, 1e9), (1473, 40, 1e4), (2240, 70, 1e6)]
    from oracle import coeffs as oc
    mats = [W.svd_matrix(m, n, kappa, 50 + m, 60 + n)[0] for m, n, kappa in cases]
    ls = [1.0 / kappa for _, _, kappa in cases]
    rs = [oc.choose_r(l) for l in ls]
    Qs, Hs, infos = z.pd_batched([dev(A) for A in mats], alphas=[1.0] * len(mats), ls=ls, rs=rs)
    for A, Q, H, inf, l, r in zip(mats, Qs, Hs, infos, ls, rs):
        Q, H = Q.cpu().numpy(), H.cpu().numpy()
        Qo, Ho, io = oz.zolo_pd(A, 1.0, l, r)
        assert inf["status"] == 0, inf
        same_schedule(inf, io)
        assert oz.backward_error(A, Q, H) <= BAR and oz.orthogonality(Q) <= BAR
        assert np.linalg.norm(H - Ho) / np.linalg.norm(Ho) <= 1e-12


def test_lookahead_same_bits(z):
    # One-matrix QR-type steps (r = 1, QDWH-PD) split each trailing update
    # into the next superblock's columns and the far columns; the far part
    # runs on a second stream once zolo_pd has created it.  A fresh handle
    # whose first call is the allocation-free entry point has no second
    # stream: both give the same bits, and H matches the exact
    # V diag(sigma) V^T.  n = 700 has three superblocks, so far parts exist.
    # The second case leaves r to the least-predicted-time policy (one
    # matrix per factorisation only if the policy picks r = 1).
    from paper_1806_06204_amd import zolo
    m, n, kappa = 1100, 700, 1e12
    A, U, sig, V = W.svd_matrix(m, n, kappa, 81, 82)
    Ad = zolo.to_device(A)
    Hx = (V * sig) @ V.T
    for kw in ({"r": 1}, {"r": None, "r_policy": 1}):
        fresh = zolo.Zolo()
        try:
            Qa, Ha, ia = fresh.pd(Ad, alpha=1.0, l=1.0 / kappa, noalloc=True, **kw)
            Qa, Ha = Qa.cpu().numpy(), Ha.cpu().numpy()
        finally:
            fresh.close()
        Qb, Hb, ib = z.pd(Ad, alpha=1.0, l=1.0 / kappa, **kw)
        Qb, Hb = Qb.cpu().numpy(), Hb.cpu().numpy()
        assert ia["status"] == 0 and ib["status"] == 0 and ia["kinds"] == ib["kinds"], kw
        assert ia["r"] == ib["r"] and ia["kinds"][0] == "Q", (kw, ia["r"], ia["kinds"])
        assert np.array_equal(Qa, Qb) and np.array_equal(Ha, Hb), kw
        assert oz.backward_error(A, Qb, Hb) <= BAR and oz.orthogonality(Qb) <= BAR
        assert np.linalg.norm(Hb - Hx) / np.linalg.norm(Hx) <= 1e-12


def test_mixed_schedule_fp32_middle_step(z):
    # 256 x 128, kappa = 1e8, r = 3: schedule Q, C, C; the middle Cholesky-type
    # step is the only one the mixed schedule runs in FP32.  Orthogonality is
    # restored by the final FP64 step, but the backward error stays at the
    # size of the FP32 perturbation (the polar factor of the perturbed iterate
    # is what the remaining steps converge to).
    cfg = W.config_small()
    A = cfg["A"]
    Ad = dev(A)
    Q64, H64, i64 = z.pd(Ad, alpha=1.0, l=cfg["l"], r=3)
    Qm, Hm, im = z.pd(Ad, alpha=1.0, l=cfg["l"], r=3, precision=1)
    assert "".join(i64["kinds"]) == "QCC" and i64["prec"] == "ddd"
    assert "".join(im["kinds"]) == "QCC" and im["prec"] == "dsd"
    assert im["status"] == 0
    Qm, Hm = Qm.cpu().numpy(), Hm.cpu().numpy()
    assert oz.orthogonality(Qm) <= BAR
    bwd = oz.backward_error(A, Qm, Hm)
    assert 1e-11 < bwd <= 1e-5
    Ho = oz.zolo_pd(A, 1.0, cfg["l"], 3)[1]
    assert np.linalg.norm(Hm - Ho) / np.linalg.norm(Ho) <= 1e-5


def test_mixed_schedule_without_middle_step_is_fp64(z):
    # kappa = 1e8 with the policy degree (schedule Q, C): no step is predicted
    # to be followed by another Cholesky step, so mixed equals FP64 exactly.
    cfg = W.config_small()
    Ad = dev(cfg["A"])
    Q64, H64, i64 = z.pd(Ad, alpha=1.0, l=cfg["l"], r=6)
    Qm, Hm, im = z.pd(Ad, alpha=1.0, l=cfg["l"], r=6, precision=1)
    assert "".join(im["kinds"]) == "".join(i64["kinds"]) and set(im["prec"]) == {"d"}
    assert np.array_equal(Q64.cpu().numpy(), Qm.cpu().numpy())
    assert np.array_equal(H64.cpu().numpy(), Hm.cpu().numpy())


@pytest.mark.parametrize("m,n,kappa,l_given,r", [(120, 80, 1e12, 1e-4, 4), (90, 90, 1e14, 1e-2, 3),
                                                  (150, 100, 1e8, 0.5, 2)])
def test_overestimated_l_is_reestimated(z, m, n, kappa, l_given, r):
    # The verified stop finds sqrt(n) d >= 1 after the predicted last step and
    # restarts from the condition estimate of the current X, as the oracle does.
    A, U, s, V = W.svd_matrix(m, n, kappa, 5, 6)
    Q, H, info = z.pd(dev(A), alpha=1.0, l=l_given, r=r, compute_errors=1)
    _, Ho, io = oz.zolo_pd(A, 1.0, l_given, r)
    assert info["status"] == 0 and info["l_reestimates"] == io["l_reestimates"] >= 1
    assert "".join(info["kinds"]) == "".join(io["kinds"])
    assert info["bwd_err"] <= BAR and info["orth_err"] <= BAR
    assert np.linalg.norm(H.cpu().numpy() - Ho) <= 1e-12 * np.linalg.norm(Ho)


def test_batched_streams_match_sequential(z):
    # Concurrent solves (several streams; single-workgroup panels on each
    # solve's stream, cooperative ones on one shared panel stream) give the
    # same bits as one solve after another: every kernel is deterministic and
    # the panel geometry does not depend on the number of streams.  One
    # matrix has more live rows than single-workgroup panels take.
    specs = W.batch_specs(count=10, seed=4200, nmin=40, nmax=700)
    mats = [W.svd_matrix(sp["m"], sp["n"], sp["kappa"], sp["seed_u"], sp["seed_v"])[0] for sp in specs]
    ls = [1.0 / sp["kappa"] for sp in specs]
    for m, n, kappa in ((2048, 1024, 1e6), (2400, 200, 1e3)):
        mats.append(W.svd_matrix(m, n, kappa, 31 + n, 32 + n)[0])
        ls.append(1.0 / kappa)
    dmats = [dev(A) for A in mats]
    Qs1, Hs1, i1 = z.pd_batched(dmats, alphas=[1.0] * len(mats), ls=ls, batch_streams=1)
    for streams in (4, 0):
        Qs, Hs, inf = z.pd_batched(dmats, alphas=[1.0] * len(mats), ls=ls, batch_streams=streams)
        for a, b, c, d, x, y in zip(Qs1, Qs, Hs1, Hs, i1, inf):
            assert x["status"] == 0 and y["status"] == 0 and x["kinds"] == y["kinds"]
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
            assert np.array_equal(c.cpu().numpy(), d.cpu().numpy())
    for A, Q, H in zip(mats, Qs1, Hs1):
        Q, H = Q.cpu().numpy(), H.cpu().numpy()
        assert np.linalg.norm(A - Q @ H) <= BAR * np.linalg.norm(A)
        assert np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1])) <= BAR * math.sqrt(Q.shape[1])


@pytest.mark.parametrize("r", [1, 2])
def test_small_degrees_qdwh(z, r):
    # r = 1 is QDWH-PD (Section 2.1, eqs. (2)-(4)): the Zolotarev function of
    # degree 1 is the dynamically weighted Halley map, here with the same QR
    # to Cholesky switch.  kappa = 1e12 gives several QR-type steps.
    A = W.svd_matrix(300, 200, 1e12, 1600 + r, 2600 + r)[0]
    info, io = run_and_compare(z, A, 1.0, 1e-12, r)
    assert info["kinds"][:2] == ["Q", "Q"] and info["r"] == r


def test_dense_qr_variant_matches_oracle(z):
    # qr_variant = 1 factors [X; sqrt(c) I] as a dense (m + n) x n matrix (the
    # comparison of Section 3.1 / Table 2).  It is still Algorithm 1 with the
    # same step kinds; H agrees with the oracle and with the structured form.
    A = W.svd_matrix(260, 140, 1e10, 1700, 2700)[0]
    info, io = run_and_compare(z, A, 1.0, 1e-10, 4, qr_variant=1)
    assert info["kinds"][0] == "Q"
    Ad = dev(A)
    _, Hs, _ = z.pd(Ad, alpha=1.0, l=1e-10, r=4)
    _, Hd, _ = z.pd(Ad, alpha=1.0, l=1e-10, r=4, qr_variant=1)
    Hs, Hd = Hs.cpu().numpy(), Hd.cpu().numpy()
    assert np.linalg.norm(Hs - Hd) <= 1e-12 * np.linalg.norm(Hs)
    # The dense form executes more flops for the same step.
    _, _, i0 = z.pd(Ad, alpha=1.0, l=1e-10, r=4)
    _, _, i1 = z.pd(Ad, alpha=1.0, l=1e-10, r=4, qr_variant=1)
    assert i1["flops_exec"] > i0["flops_exec"]


def test_time_policy_picks_least_predicted(z):
    # r_policy = 1: the degree with the least predicted time from the
    # library's own cost model; the solve then meets the FP64 bar.
    from paper_1806_06204_amd import zolo
    A = W.svd_matrix(384, 256, 1e14, 1800, 2800)[0]
    _, H, info = z.pd(dev(A), alpha=1.0, l=1e-14, r_policy=1, compute_errors=1)
    pred = {r: zolo.predict(1e-14, r, 384, 256)[1] for r in range(1, 9)}
    best = min(pred, key=lambda r: (pred[r], r))
    assert info["r"] == best
    assert info["status"] == 0 and info["bwd_err"] <= BAR and info["orth_err"] <= BAR
    Ho = oz.zolo_pd(A, 1.0, 1e-14, best)[1]
    assert np.linalg.norm(H.cpu().numpy() - Ho) <= 1e-12 * np.linalg.norm(Ho)


def test_batched_512_uneven_all_exact(z):
    # The 512-matrix uneven workload (n ~ U{64..1024}, m ~ U{n..2n}, log10
    # kappa ~ U[2, 12], r by the two-iteration rule) in one zolo_pd_batched
    # call on 16 worker streams: every matrix converged, backward error and
    # orthogonality <= 1e-13 recomputed on the host, and H against the exact
    # V diag(sigma) V^T (<= 1e-12).
    import torch
    from paper_1806_06204_amd import zolo
    specs = W.batch_specs(count=512, seed=4000)
    built = [W.svd_matrix(sp["m"], sp["n"], sp["kappa"], sp["seed_u"], sp["seed_v"]) for sp in specs]
    print("  512 matrices generated", flush=True)
    As = [zolo.to_device(b[0]) for b in built]
    Qs, Hs, infos = z.pd_batched(As, alphas=[1.0] * len(As), ls=[1.0 / sp["kappa"] for sp in specs])
    worst = [0.0, 0.0, 0.0]
    for (A, U, sig, V), Q, H, inf in zip(built, Qs, Hs, infos):
        assert inf["status"] == 0, inf
        Qn, Hn = Q.cpu().numpy(), H.cpu().numpy()
        bwd, orth = host_errors(A, Qn, Hn)
        Vt = torch.from_numpy(V)
        Hx = ((Vt * torch.from_numpy(sig)) @ Vt.T).numpy()
        dh = np.linalg.norm(Hn - Hx) / np.linalg.norm(Hx)
        worst = [max(worst[0], bwd), max(worst[1], orth), max(worst[2], dh)]
    print(f"  worst over 512: bwd={worst[0]:.2e} orth={worst[1]:.2e} dH_exact={worst[2]:.2e}", flush=True)
    assert worst[0] <= BAR and worst[1] <= BAR and worst[2] <= 1e-12
