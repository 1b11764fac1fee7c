"""zolo_pd_noalloc (the allocation-free Zolo-PD entry point, workspace in the
library's fixed device scratch) against zolo_pd on the same inputs: the same
kernels on the same workspace layout give the same bits.  Two calls in a
row, the second smaller (the scratch keeps the first call's contents), then
a problem too large for the scratch is rejected before any work."""

import numpy as np
import pytest

from oracle import zolo as oz
from paper_1806_06204_amd import workloads as W

pytestmark = pytest.mark.gpu
BAR = 1e-13


def test_noalloc_matches_zolo_pd():
    import torch
    from paper_1806_06204_amd import zolo
    assert torch.cuda.is_available()
    z = zolo.Zolo()
    try:
        cases = [(700, 512, 1e12, 8, 1.0, 1e-12), (200, 77, 1e4, None, None, None)]
        for m, n, kappa, r, alpha, l in cases:
            print(f"  noalloc m={m} n={n} kappa={kappa:g} r={r}", flush=True)
            A, U, sig, V = W.svd_matrix(m, n, kappa, 60 + m, 70 + n)
            Ad = zolo.to_device(A)
            Qa, Ha, ia = z.pd(Ad, alpha=alpha, l=l, r=r, compute_errors=1, noalloc=True)
            Qb, Hb, ib = z.pd(Ad, alpha=alpha, l=l, r=r, compute_errors=1)
            Qa, Ha, Qb, Hb = (t.cpu().numpy() for t in (Qa, Ha, Qb, Hb))
            print(f"  kinds={''.join(ia['kinds'])} bwd={ia['bwd_err']:.2e} orth={ia['orth_err']:.2e}", flush=True)
            assert ia["status"] == 0 and ib["status"] == 0
            assert ia["kinds"] == ib["kinds"] and ia["r"] == ib["r"] and ia["l0"] == ib["l0"]
            assert np.array_equal(Qa, Qb) and np.array_equal(Ha, Hb)
            assert oz.backward_error(A, Qa, Ha) <= BAR and oz.orthogonality(Qa) <= BAR
            Hx = (V * sig) @ V.T
            assert np.linalg.norm(Ha - Hx) <= 1e-12 * np.linalg.norm(Hx)
        # Larger than the fixed scratch (256 MiB): rejected with ZOLO_SCRATCH.
        big = torch.zeros((2048, 1024), dtype=torch.float64, device="cuda")
        _, _, info = z.pd(big, alpha=1.0, l=1e-3, r=8, check=False, noalloc=True)
        assert info["status"] == 7
        with pytest.raises(zolo.ZoloError):
            z.pd(big, alpha=1.0, l=1e-3, r=8, noalloc=True)
    finally:
        z.close()
