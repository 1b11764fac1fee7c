"""CPU FP64 oracle for Zolo-PD (test infrastructure only).

This package is a slow, plain, obviously-correct reference implementation of
the polar decomposition by composed Zolotarev functions (Zolo-PD, Algorithm 1
of Li, Liu & Du, "A New High Performance and Scalable SVD algorithm on
Distributed Memory Systems", arXiv 1806.06204).  It exists to check the HIP
library against the paper.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path never does.

It shares no code with the HIP library: its own Zolotarev coefficients
(theta-series evaluation of eq. (7)), its own unblocked Householder QR,
Cholesky and triangular solves, and its own Jacobi eigensolver.  NumPy is used
for array storage and the ``@`` product only.

Modules
-------
coeffs   Zolotarev coefficients c_i, a_j, M-hat, the l-update and r policy
         (Section 2.2, eqs. (6)-(10), Table 1).
dense    Householder QR, Cholesky, triangular solves, Jacobi eigensolver.
zolo     Zolo-PD (Algorithm 1 / Algorithm 3 steps 1-4) and Zolo-SVD
         (Algorithm 2), plus the accuracy metrics of Section 4.1.

Parity pins: every function here is pinned by tests marked "not gpu" against
the paper's Table 1, closed forms, mpmath, invariants and brute force; none is
"parity unpinned".
"""
