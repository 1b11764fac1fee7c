"""Zolo-PD on MI355X: a HIP library for the polar decomposition by composed
Zolotarev functions (Li, Liu & Du, arXiv 1806.06204).

The native library (``csrc/``, built into ``libzolo.so``) does every step of
the iteration on the GPU; ``paper_1806_06204_amd.zolo`` is a thin ctypes
binding over its C ABI (``include/zolo.h``).  Import it explicitly:

    from paper_1806_06204_amd import zolo

``workloads`` builds seeded synthetic inputs.
"""
