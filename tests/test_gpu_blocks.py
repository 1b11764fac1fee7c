"""GPU parity of the library's building blocks (through the C ABI) against
NumPy FP64 references and the oracle's own factorisations.  Shapes span
several tiles and ragged tails (64-row MFMA tiles, 64-column panels)."""

import numpy as np
import pytest

from oracle import dense

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("m,n,k", [(16, 16, 4), (1, 1, 1), (37, 53, 29), (130, 70, 200), (257, 129, 65)])
def test_gemm(z, ta, tb, m, n, k):
    rng = np.random.default_rng(m * 7 + n * 3 + k + 11 * ta + 5 * tb)
    batch = 2
    A = rng.standard_normal((batch, k, m) if ta else (batch, m, k))
    B = rng.standard_normal((batch, n, k) if tb else (batch, k, n))
    C = rng.standard_normal((batch, m, n))
    out = z.gemm(dev(A), dev(B), dev(C), transa=ta, transb=tb, alpha=0.7, beta=-1.3).cpu().numpy()
    opA = np.swapaxes(A, 1, 2) if ta else A
    opB = np.swapaxes(B, 1, 2) if tb else B
    ref = 0.7 * opA @ opB - 1.3 * C
    assert np.abs(out - ref).max() <= 1e-13 * (k + 1) * 4


def test_gemm_mfma_layout_identity(z):
    # Each output element must land in its own (row, column): product with a
    # permutation-like operand exposes any lane-layout mix-up.
    rng = np.random.default_rng(1)
    A = rng.standard_normal((1, 128, 128))
    P = np.eye(128)[rng.permutation(128)][None]
    out = z.gemm(dev(A), dev(P)).cpu().numpy()
    assert np.array_equal(out, A @ P)


def test_gemm_large(z):
    rng = np.random.default_rng(2)
    A = rng.standard_normal((1, 1000, 777))
    B = rng.standard_normal((1, 777, 1031))
    out = z.gemm(dev(A), dev(B)).cpu().numpy()
    assert np.abs(out - A @ B).max() <= 1e-12 * 777


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_gemm_vector_kernel_shapes(z, ta, tb):
    # Large enough for the vector-FMA kernel (128 x 128 tiles) where its
    # rule takes it: ragged in m, n and k, batch 8, alpha and beta.
    rng = np.random.default_rng(40 + 2 * ta + tb)
    m, n, k, batch = 1000, 1100, 120 if ta else 300, 8
    A = rng.standard_normal((batch, k, m) if ta else (batch, m, k))
    B = rng.standard_normal((batch, n, k) if tb else (batch, k, n))
    C = rng.standard_normal((batch, m, n))
    out = z.gemm(dev(A), dev(B), dev(C), transa=ta, transb=tb, alpha=-0.6, beta=1.7).cpu().numpy()
    opA = np.swapaxes(A, 1, 2) if ta else A
    opB = np.swapaxes(B, 1, 2) if tb else B
    ref = -0.6 * opA @ opB + 1.7 * C
    assert np.abs(out - ref).max() <= 1e-13 * (k + 1) * 4


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("m,n,k", [(130, 258, 300), (131, 257, 517), (256, 384, 1000), (64, 64, 129)])
def test_gemm_pipe_kernel_shapes(z, ta, tb, m, n, k):
    # Long-k products (the pipelined kernel where its rule takes them): even
    # and odd edges (clamped rows), k not a multiple of the 16-deep slice
    # (even: the last slice shifted back and its overlap zeroed; odd with an
    # operand contiguous along k: the last slice taken apart with
    # element-wise loads), batch 3, alpha and beta.
    rng = np.random.default_rng(m + 3 * n + 7 * k + 2 * ta + tb)
    batch = 3
    A = rng.standard_normal((batch, k, m) if ta else (batch, m, k))
    B = rng.standard_normal((batch, n, k) if tb else (batch, k, n))
    C = rng.standard_normal((batch, m, n))
    out = z.gemm(dev(A), dev(B), dev(C), transa=ta, transb=tb, alpha=1.3, beta=-0.4).cpu().numpy()
    opA = np.swapaxes(A, 1, 2) if ta else A
    opB = np.swapaxes(B, 1, 2) if tb else B
    ref = 1.3 * opA @ opB - 0.4 * C
    assert np.abs(out - ref).max() <= 1e-13 * (k + 1) * 4


@pytest.mark.parametrize("ta,tb,m,n,k", [(0, 0, 130, 258, 300), (1, 0, 131, 257, 518), (0, 1, 256, 384, 1000),
                                          (1, 1, 192, 320, 160)])
def test_gemm_autotune_bitwise(z, ta, tb, m, n, k):
    # The autotuner runs every candidate tile shape of the pipelined kernel on
    # the first calls of a shape class, then the fastest: every call must
    # give the same bits, and all three shapes must have run.
    from paper_1806_06204_amd import zolo
    rng = np.random.default_rng(11 * m + n + k + 2 * ta + tb)
    A = rng.standard_normal((2, k, m) if ta else (2, m, k))
    B = rng.standard_normal((2, n, k) if tb else (2, k, n))
    C = rng.standard_normal((2, m, n))
    dA, dB, dC = dev(A), dev(B), dev(C)
    zolo.autotune_enable(True)
    zolo.autotune_reset()
    zolo.stats_enable(True)
    zolo.stats_reset()
    try:
        outs = [z.gemm(dA, dB, dC, transa=ta, transb=tb, alpha=0.7, beta=1.5).cpu().numpy() for _ in range(8)]
        names = {nm for nm in zolo.stats() if nm.startswith("dgemm_pipe<")}
    finally:
        zolo.stats_enable(False)
        zolo.autotune_enable(False)
    tag = ",%s,%s>" % ("T" if ta else "N", "T" if tb else "N")
    assert names == {"dgemm_pipe<%d,%d%s" % (bm, bn, tag) for bm, bn in ((64, 128), (64, 64), (128, 64))}
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    opA = np.swapaxes(A, 1, 2) if ta else A
    opB = np.swapaxes(B, 1, 2) if tb else B
    ref = 0.7 * opA @ opB + 1.5 * C
    assert np.abs(outs[0] - ref).max() <= 1e-13 * (k + 1) * 4


def test_gemm_vector_kernel_layout_identity(z):
    # Exact permutation products pin the 8 x 8 per-thread output layout.
    rng = np.random.default_rng(3)
    A = rng.standard_normal((8, 1030, 1024))
    P = np.stack([np.eye(1024)[rng.permutation(1024)] for _ in range(8)])
    out = z.gemm(dev(A), dev(P)).cpu().numpy()
    assert np.array_equal(out, A @ P)


# --- FP32 building blocks (the FP32 steps of the mixed schedule) ----------
# References are FP64 products of the same FP32 inputs; the bound is the
# usual k u |A||B| with u = 2^-24, taken elementwise.
U32 = 2.0 ** -24


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("m,n,k", [(16, 16, 4), (37, 53, 29), (257, 129, 65), (300, 260, 400)])
def test_sgemm(z, ta, tb, m, n, k):
    import torch
    rng = np.random.default_rng(m * 5 + n + k + 3 * ta + 7 * tb)
    A = rng.standard_normal((2, k, m) if ta else (2, m, k)).astype(np.float32)
    B = rng.standard_normal((2, n, k) if tb else (2, k, n)).astype(np.float32)
    C = rng.standard_normal((2, m, n)).astype(np.float32)
    out = z.gemm(dev(A), dev(B), dev(C), transa=ta, transb=tb, alpha=0.5, beta=2.0)
    assert out.dtype == torch.float32
    out = out.cpu().numpy().astype(np.float64)
    opA = np.swapaxes(A, 1, 2).astype(np.float64) if ta else A.astype(np.float64)
    opB = np.swapaxes(B, 1, 2).astype(np.float64) if tb else B.astype(np.float64)
    ref = 0.5 * opA @ opB + 2.0 * C
    bound = (k + 2) * U32 * (0.5 * np.abs(opA) @ np.abs(opB) + 2.0 * np.abs(C)) + 1e-30
    assert np.all(np.abs(out - ref) <= bound)


def test_sgemm_mfma_layout_identity(z):
    # Exact in FP32: a product with a permutation matrix moves every entry to
    # its own (row, column), so any mix-up of the FP32 accumulator rows shows.
    rng = np.random.default_rng(3)
    A = rng.standard_normal((1, 256, 128)).astype(np.float32)
    P = np.eye(128, dtype=np.float32)[rng.permutation(128)][None]
    out = z.gemm(dev(A), dev(P)).cpu().numpy()
    assert np.array_equal(out, A @ P)
    out_t = z.gemm(dev(P), dev(np.swapaxes(A, 1, 2).copy()), transa=True).cpu().numpy()
    assert np.array_equal(out_t, np.swapaxes(P, 1, 2) @ np.swapaxes(A, 1, 2))


@pytest.mark.parametrize("n", [1, 64, 200])
def test_spotrf_strtri(z, n):
    # Well conditioned (kappa <= 100, the Cholesky-step regime) FP32 Z_j.
    rng = np.random.default_rng(n + 7)
    Zs = []
    for b in range(3):
        Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
        Zs.append((Q * np.linspace(1.0, 100.0, n)) @ Q.T)
    Zs = np.stack(Zs).astype(np.float32)
    R, info = z.potrf(dev(Zs))
    assert info == [0, 0, 0]
    Ri = z.trtri(R).cpu().numpy().astype(np.float64)
    R = R.cpu().numpy().astype(np.float64)
    for b in range(3):
        Z64 = Zs[b].astype(np.float64)
        assert np.allclose(np.tril(R[b], -1), 0.0) and np.allclose(np.tril(Ri[b], -1), 0.0)
        # backward error of the factor and residual of the inverse, FP32 sized
        assert np.linalg.norm(R[b].T @ R[b] - Z64) <= 8 * n * U32 * np.linalg.norm(Z64)
        assert np.abs(Ri[b] @ R[b] - np.eye(n)).max() <= 8 * n * U32 * 10.0


@pytest.mark.parametrize("n", [1, 64, 200])
def test_potrf(z, n):
    rng = np.random.default_rng(n)
    Zs = []
    for b in range(3):
        M = rng.standard_normal((n + 10, n))
        Zs.append(M.T @ M + 0.5 * np.eye(n))
    Zs = np.stack(Zs)
    R, info = z.potrf(dev(Zs))
    R = R.cpu().numpy()
    assert info == [0, 0, 0]
    for b in range(3):
        ref = dense.cholesky_upper(Zs[b])
        assert np.allclose(np.tril(R[b], -1), 0.0)
        assert np.abs(R[b] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_potrf_breakdown_reported(z):
    n = 150
    rng = np.random.default_rng(9)
    M = rng.standard_normal((n, n))
    good = M.T @ M + np.eye(n)
    bad = good.copy()
    bad[100, 100] = -5.0
    _, info = z.potrf(dev(np.stack([good, bad])))
    assert info[0] == 0 and info[1] > 0


@pytest.mark.parametrize("n", [1, 63, 64, 65, 300])
def test_trtri(z, n):
    rng = np.random.default_rng(n + 100)
    R = np.stack([np.triu(rng.standard_normal((n, n))) + (n ** 0.5) * np.eye(n) for _ in range(2)])
    Ri = z.trtri(dev(R)).cpu().numpy()
    for b in range(2):
        ref = dense.invert_upper(R[b])
        assert np.allclose(np.tril(Ri[b], -1), 0.0)
        assert np.abs(Ri[b] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("m,n", [(40, 7), (300, 150), (129, 129), (200, 65)])
def test_structured_qr(z, m, n):
    # eq. (12) / Section 3.1: QR of the stacked [Y; p I] with m + 64 live rows per panel.
    rng = np.random.default_rng(m + n)
    pivots = [0.3, 1.0, 1e-3]
    Y = rng.standard_normal((len(pivots), m, n))
    V, Rg = z.structured_qr(dev(Y), pivots, form_q=False)
    Q, Rq = z.structured_qr(dev(Y), pivots, form_q=True)
    Rg, Q, Rq = Rg.cpu().numpy(), Q.cpu().numpy(), Rq.cpu().numpy()
    assert np.array_equal(Rg, Rq)
    for b, p in enumerate(pivots):
        S = np.vstack([Y[b], p * np.eye(n)])
        assert np.linalg.norm(Q[b].T @ Q[b] - np.eye(n)) <= 1e-13 * n
        assert np.linalg.norm(Q[b] @ Rg[b] - S) <= 1e-13 * n * np.linalg.norm(S)
        assert np.allclose(np.tril(Rg[b], -1), 0.0)
        assert np.allclose(np.tril(Q[b][m:], -1), 0.0, atol=1e-14)   # Q_2 upper triangular
        # R agrees with the oracle's Householder QR up to row signs, and the
        # eq. (12) product Q_1 Q_2^T is sign independent.
        Qo, Ro = dense.householder_qr(S)
        s = np.sign(np.diag(Rg[b])) * np.sign(np.diag(Ro))
        assert np.abs(Rg[b] * s[:, None] - Ro).max() <= 1e-12 * np.abs(Ro).max()
        assert np.abs(Q[b][:m] @ Q[b][m:].T - Qo[:m] @ Qo[m:].T).max() <= 1e-11


@pytest.mark.parametrize("m,n,batch", [(1025, 881, 5), (700, 600, 16)])
def test_structured_qr_many_slabs(z, m, n, batch):
    # Mid-size panels split over 11-18 workgroups per matrix and up to 16
    # matrices per launch, so the cross-workgroup reduction of every column
    # runs with many slabs at once.  Pivots are the sqrt(c_{2j-1}) of a
    # degree-5 Zolotarev step at l = 1/9e4 (large and small shifts together).
    from oracle import coeffs as oc
    co = oc.coefficients(1.0 / 9e4, 5)
    base = [float(np.sqrt(co["c"][2 * j])) for j in range(5)]
    pivots = [base[b % 5] * (1.0 + 0.1 * (b // 5)) for b in range(batch)]
    rng = np.random.default_rng(m * n + batch)
    Y = rng.standard_normal((batch, m, n)) / np.sqrt(m)
    for rep in range(2):
        Q, R = z.structured_qr(dev(Y), pivots, form_q=True)
        Q, R = Q.cpu().numpy(), R.cpu().numpy()
        for b, p in enumerate(pivots):
            S = np.vstack([Y[b], p * np.eye(n)])
            assert np.linalg.norm(Q[b].T @ Q[b] - np.eye(n)) <= 1e-14 * n, (rep, b)
            assert np.linalg.norm(Q[b] @ R[b] - S) <= 1e-14 * n * np.linalg.norm(S), (rep, b)
            Rl = np.linalg.qr(S, mode="r")
            s = np.sign(np.diag(R[b])) * np.sign(np.diag(Rl))
            assert np.abs(R[b] * s[:, None] - Rl).max() <= 1e-12 * np.abs(Rl).max(), (rep, b)


def test_structured_qr_global_slabs(z):
    # 12064 live rows per panel and 8 matrices: the slabs do not fit in LDS
    # with every workgroup resident, so the panels run the global-memory
    # variant (32 workgroups per matrix, 377 rows each) with the cooperative
    # exchange.
    rng = np.random.default_rng(12000)
    m, n, batch = 12000, 128, 8
    pivots = [0.5 ** b for b in range(batch)]
    Y = rng.standard_normal((batch, m, n)) / np.sqrt(m)
    Q, R = z.structured_qr(dev(Y), pivots, form_q=True)
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    for b, p in enumerate(pivots):
        S = np.vstack([Y[b], p * np.eye(n)])
        assert np.linalg.norm(Q[b].T @ Q[b] - np.eye(n)) <= 1e-14 * n, b
        assert np.linalg.norm(Q[b] @ R[b] - S) <= 1e-14 * n * np.linalg.norm(S), b
        Rl = np.linalg.qr(S, mode="r")
        s = np.sign(np.diag(R[b])) * np.sign(np.diag(Rl))
        assert np.abs(R[b] * s[:, None] - Rl).max() <= 1e-12 * np.abs(Rl).max(), b


@pytest.mark.parametrize("m,n", [(100, 100), (333, 129), (64, 1)])
def test_plain_qr(z, m, n):
    rng = np.random.default_rng(3 * m + n)
    Y = rng.standard_normal((2, m, n))
    Q, R = z.structured_qr(dev(Y), None, form_q=True)
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    for b in range(2):
        assert np.linalg.norm(Q[b].T @ Q[b] - np.eye(n)) <= 1e-13 * n
        assert np.linalg.norm(Q[b] @ R[b] - Y[b]) <= 1e-13 * n * np.linalg.norm(Y[b])
        _, Ro = dense.householder_qr(Y[b])
        s = np.sign(np.diag(R[b])) * np.sign(np.diag(Ro))
        assert np.abs(R[b] * s[:, None] - Ro).max() <= 1e-12 * np.abs(Ro).max()
