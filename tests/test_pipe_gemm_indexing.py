"""Indexing invariants of the pipelined FP64 GEMM (dgemm_pipe_kernel in
csrc/gemm.hip), checked on the CPU by replaying the kernel's address and mask
arithmetic for every tile, slice and chunk of small launches.

For every launch the dispatcher accepts (16-byte pairs aligned and never
straddling an edge of op(A) or op(B); odd k with an operand contiguous along
k only without a sum over the batch) the replay checks that

* every 16-byte load of the pipelined loop (the shifted ragged slice and the
  clamped edge rows included) and every element load of a peeled slice lies
  inside the operand's storage, and pairs start at even element offsets;
* every element op(A)[i][k] (op(B)[k][j]) of a tile's k-range that lies
  inside the triangle of a triangular operand is stored unmasked exactly
  once over the slices of its batch (split-K pieces together), and every
  element outside the triangle is never stored unmasked.

A mistake in the shift of the ragged slice, the peel condition, the zeroing
bounds or the row clamp fails one of these on the shapes below.
"""

import itertools

import numpy as np
import pytest

BK = 16
A_UPPER, A_LOWER, B_UPPER, B_LOWER = 1, 2, 4, 8


def coords(R, kc, slot):
    """(r, kk) of each 16-byte chunk slot of an R x 16 slice (Lay<R, KC>)."""
    if not kc:
        kk = slot // (R // 2)
        r = 2 * ((slot % (R // 2)) ^ ((kk & 1) * 8))
    else:
        r = slot // (BK // 2)
        kk = 2 * ((slot % (BK // 2)) ^ (r & 7))
    return r, kk


def eligible(ta, tb, m, n, k, lda, ldb, reduce_batch):
    """The dispatcher's conditions for this kernel (alignment of the base
    pointers and even strides assumed)."""
    even_edges = (ta or m % 2 == 0) and ((not tb) or n % 2 == 0)
    kc_any = ta or not tb
    odd_k_ok = (not kc_any) or k % 2 == 0 or not reduce_batch
    return even_edges and odd_k_ok and lda % 2 == 0 and ldb % 2 == 0 and k > 128


def replay_operand(R, kc, ext, ld, k, lo0, kb, ke, tri, kfull, t_begin, t_main, t_end, nk, peel, count, store):
    """Replay one operand of one tile over slices [t_begin, t_end).

    kc: memory contiguous along k (pairs along k); ext: m (or n); lo0: row0
    (or col0); tri(i, gk) -> inside the triangle; kfull: (lo, hi) bounds of
    the slices that need no zeroing.  count[b][i - lo0, gk] accumulates the
    unmasked stores."""
    slots = np.arange(R * BK // 2)
    r, kk = coords(R, kc, slots)
    last = ext - 1 if kc else ext - 2
    g = np.clip(lo0 + r, 0, last)
    for t in range(t_begin, t_end):
        b, s = divmod(t, nk)
        kq = kb + s * BK
        for h in (0, 1):
            i_log = lo0 + r + (0 if kc else h)     # logical row (column) of the element
            if t < t_main:
                k0 = min(kq, ke - BK)
                gk = k0 + kk + (h if kc else 0)
                gi = g + (0 if kc else h)
                off = gk + gi * ld if kc else gi + gk * ld
                assert off.min() >= 0 and off.max() < store, (t, h)
                if h == 0:
                    assert np.all(off % 2 == 0)
                full = kq >= kfull[0] and kq + BK <= kfull[1]
                ok = np.ones_like(gk, bool) if full else (gk >= kq) & (gk < ke) & tri(i_log, gk)
            else:
                assert peel and t == t_main
                gk = kq + kk + (h if kc else 0)
                ok = (i_log < ext) & (gk < ke) & tri(i_log, gk)
                off = gk + i_log * ld if kc else i_log + gk * ld
                assert off[ok].min(initial=0) >= 0 and off[ok].max(initial=0) < store
            sel = ok & (i_log < ext)
            np.add.at(count[b], (i_log[sel] - lo0, gk[sel]), 1)


def replay(BM, BN, ta, tb, m, n, k, lda, ldb, flags, nbatch, splitk):
    tiles_m, tiles_n = -(-m // BM), -(-n // BN)
    store_a = (m - 1) * lda + k if ta else (k - 1) * lda + m
    store_b = (k - 1) * ldb + n if tb else (n - 1) * ldb + k
    for tm, tn in itertools.product(range(tiles_m), range(tiles_n)):
        row0, col0 = tm * BM, tn * BN
        kb, ke = 0, k
        if flags & A_UPPER:
            kb = max(kb, row0)
        if flags & B_LOWER:
            kb = max(kb, col0)
        if flags & A_LOWER:
            ke = min(ke, row0 + BM)
        if flags & B_UPPER:
            ke = min(ke, col0 + BN)
        nk = -(-(ke - kb) // BK) if ke > kb else 0
        ntiles = nk * nbatch
        kfull = [kb, ke]
        if flags & A_UPPER:
            kfull[0] = max(kfull[0], row0 + BM - 1)
        if flags & B_LOWER:
            kfull[0] = max(kfull[0], col0 + BN - 1)
        if flags & A_LOWER:
            kfull[1] = min(kfull[1], row0 + 1)
        if flags & B_UPPER:
            kfull[1] = min(kfull[1], col0 + 1)

        def tri_a(i, gk):
            ok = np.ones_like(gk, bool)
            if flags & A_UPPER:
                ok &= gk >= i
            if flags & A_LOWER:
                ok &= gk <= i
            return ok

        def tri_b(j, gk):
            ok = np.ones_like(gk, bool)
            if flags & B_UPPER:
                ok &= gk <= j
            if flags & B_LOWER:
                ok &= gk >= j
            return ok

        cnt_a = [np.zeros((BM, k + BK), int) for _ in range(nbatch)]
        cnt_b = [np.zeros((BN, k + BK), int) for _ in range(nbatch)]
        for z in range(splitk):
            t_begin = z * ntiles // splitk
            t_end = (z + 1) * ntiles // splitk
            if t_end <= t_begin:
                continue
            peel = (ta or not tb) and (ke % 2 == 1) and t_end == ntiles
            t_main = t_end - 1 if peel else t_end
            replay_operand(BM, ta, m, lda, k, row0, kb, ke, tri_a, kfull, t_begin, t_main, t_end, nk, peel, cnt_a,
                           store_a)
            replay_operand(BN, not tb, n, ldb, k, col0, kb, ke, tri_b, kfull, t_begin, t_main, t_end, nk, peel,
                           cnt_b, store_b)
        # Exactly once inside the triangle, never outside, over [kb, ke).
        for cnt, lo0, ext, R, tri in ((cnt_a, row0, m, BM, tri_a), (cnt_b, col0, n, BN, tri_b)):
            rows = np.arange(lo0, min(lo0 + R, ext))
            ks = np.arange(kb, ke)
            ii, kk = np.meshgrid(rows, ks, indexing="ij")
            want = tri(ii, kk).astype(int)
            for b in range(nbatch):
                got = cnt[b][rows - lo0][:, kb:ke]
                assert np.array_equal(got, want), (tm, tn, b)
                assert cnt[b][:, :kb].sum() == 0 and cnt[b][:, ke:].sum() == 0


CASES = [
    # (BM, BN, ta, tb, m, n, k, flags, nbatch, splitk); nbatch > 1: a sum over
    # the batch (one sequence of (batch, k) slices); independent matrices of
    # a batch each replay as nbatch = 1.
    (64, 128, 0, 0, 130, 258, 300, 0, 1, 1),       # even ragged k: shifted last slice
    (64, 128, 1, 0, 131, 258, 517, 0, 1, 1),       # odd k, both operands along k: peeled slice
    (64, 64, 0, 0, 64, 64, 129, 0, 1, 1),          # odd k, B along k: peeled (each matrix of a batch alike)
    (64, 64, 0, 1, 256, 384, 1000, 0, 1, 1),       # neither along k
    (128, 64, 1, 1, 192, 320, 161, 0, 1, 1),       # A along k, odd k
    (64, 128, 1, 0, 256, 130, 1030, 0, 1, 4),      # split-K pieces, ragged last piece
    (64, 128, 1, 0, 256, 130, 1031, 0, 1, 4),      # split-K, odd k: peel in the last piece only
    (64, 64, 0, 1, 130, 130, 300, 0, 3, 1),        # sum over the batch, R-layout both, ragged k
    (64, 64, 1, 0, 130, 130, 302, 0, 3, 1),        # sum over the batch, even ragged k along k
    (64, 128, 0, 0, 256, 256, 256, A_UPPER, 1, 1),  # triangular A (upper)
    (64, 128, 0, 0, 256, 256, 256, A_LOWER, 1, 1),  # triangular A (lower)
    (64, 64, 1, 0, 192, 192, 192, B_UPPER, 1, 1),   # triangular B (upper)
    (64, 64, 0, 1, 192, 200, 200, B_LOWER, 2, 1),   # triangular B (lower), batch 2
    (64, 64, 1, 0, 260, 130, 262, A_UPPER, 1, 1),   # triangular A with a ragged k-range
]


@pytest.mark.parametrize("BM,BN,ta,tb,m,n,k,flags,nbatch,splitk", CASES)
def test_pipe_gemm_indexing(BM, BN, ta, tb, m, n, k, flags, nbatch, splitk):
    lda = (k if ta else m) + (k if ta else m) % 2 + 2
    ldb = (n if tb else k) + (n if tb else k) % 2 + 2
    if not eligible(ta, tb, m, n, k, lda, ldb, nbatch > 1):
        pytest.skip("the dispatcher sends this shape to another kernel")
    replay(BM, BN, ta, tb, m, n, k, lda, ldb, flags, nbatch, splitk)


def test_pipe_gemm_indexing_tight_leading_dimension():
    # Leading dimension equal to the extent along memory (no padding): the
    # shifted ragged slice and the peeled slice must stay inside the last
    # column of the operand.
    replay(64, 128, 1, 0, 256, 130, 302, 302, 302, 0, 1, 1)
    replay(64, 64, 1, 0, 130, 64, 301, 302, 302, 0, 1, 1)


def test_pipe_gemm_dispatch_rules():
    # Shapes the pairs cannot serve go elsewhere.
    assert not eligible(0, 0, 131, 128, 300, 132, 300, False)      # odd m along pairs of A
    assert not eligible(0, 1, 128, 131, 300, 128, 132, False)      # odd n along pairs of B
    assert not eligible(1, 0, 128, 128, 301, 302, 302, True)       # odd k along k, summed over the batch
    assert eligible(1, 0, 128, 128, 301, 302, 302, False)          # the same without the sum: peeled
    assert eligible(0, 1, 128, 128, 301, 128, 128, True)           # odd k, neither along k
