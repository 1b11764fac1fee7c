"""ctypes binding of libzolo.so (include/zolo.h, include/zolo_blocks.h).

Argument marshalling only: every matrix operation runs in the library's HIP
kernels.  PyTorch supplies device memory and the current HIP stream.

Matrices cross the boundary in column-major order.  A tensor ``A`` of shape
(m, n) is passed as-is when it is already column-major (``A.stride() ==
(1, ld)``), otherwise as ``A.t().contiguous()``.  Results come back as
column-major views (``buf.t()``), which behave like ordinary (m, n) tensors.
Stacks of matrices for the batched building blocks are tensors of shape
(batch, m, n) and are handled the same way per matrix.
"""

import atexit
import ctypes
import os
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzolo.so")

c_int, c_double, c_void_p, c_longlong = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_longlong
MAX_ITER = 16
STATUS = {0: "ok", 1: "not converged", 2: "non-finite input", 3: "allocation failed", 4: "HIP error",
          5: "kernel barrier failure", 6: "factorisation breakdown", 7: "workspace exceeds the fixed scratch"}


class ZoloOpts(ctypes.Structure):
    _fields_ = [("max_iter", c_int), ("stop_rule", c_int), ("tau", c_double), ("chol_switch", c_double),
                ("qr_variant", c_int), ("precision", c_int), ("compute_errors", c_int), ("l_source", c_int),
                ("batch_streams", c_int), ("r_policy", c_int), ("reserved", c_int * 6)]


class ZoloInfo(ctypes.Structure):
    _fields_ = [("status", c_int), ("iters", c_int), ("r_used", c_int), ("chol_fallbacks", c_int), ("l_from", c_int),
                ("l_reestimates", c_int), ("checks", c_int),
                ("kind", ctypes.c_char * (MAX_ITER + 1)), ("prec", ctypes.c_char * (MAX_ITER + 1)),
                ("alpha", c_double), ("l0", c_double),
                ("l_seq", c_double * MAX_ITER), ("orth_check", c_double), ("t_stage", c_double * 8),
                ("flops_exec", c_double), ("flops_paper", c_double), ("bwd_err", c_double),
                ("orth_err", c_double)]

    def as_dict(self):
        it = self.iters
        return {"status": self.status, "iters": it, "r": self.r_used, "chol_fallbacks": self.chol_fallbacks,
                "l_from": ("given", "condition estimate", "learned")[self.l_from],
                "l_reestimates": self.l_reestimates, "checks": self.checks,
                "kinds": list(self.kind.decode()), "prec": self.prec.decode(), "alpha": self.alpha,
                "l0": self.l0,
                "ls": list(self.l_seq[:it]), "orth_check": self.orth_check,
                "t_stage_ms": list(self.t_stage), "flops_exec": self.flops_exec,
                "flops_paper": self.flops_paper, "bwd_err": self.bwd_err, "orth_err": self.orth_err}


_lib = None

EXPORTS = ["zolo_default_opts", "zolo_create", "zolo_set_stream", "zolo_destroy", "zolo_coeffs", "zolo_pd",
           "zolo_pd_batched", "zolo_svd", "zolo_dgemm", "zolo_dpotrf_batched", "zolo_dtrtri_batched",
           "zolo_sgemm", "zolo_spotrf_batched", "zolo_strtri_batched", "zolo_structured_qr_batched",
           "zolo_stats_enable", "zolo_stats_reset", "zolo_stats_get", "zolo_stats_count",
           "zolo_autotune_enable", "zolo_autotune_reset",
           "zolo_sketch_features", "zolo_surrogate_features", "zolo_mlp_stats", "zolo_mlp_work_elems",
           "zolo_mlp_forward", "zolo_mlp_loss", "zolo_mlp_backward", "zolo_mlp_adam", "zolo_mlp_train",
           "zolo_set_estimator", "zolo_choose_r", "zolo_predict", "zolo_release_events", "zolo_pd_noalloc", "zolo_dsyevd"]
NF, MLP_NPARAMS, MLP_NSTATS = 39, 6928, 78


def load():
    """Load libzolo.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python -m paper_1806_06204_amd.build_lib)")
    lib = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    D = ctypes.POINTER(c_double)
    lib.zolo_default_opts.argtypes = [ctypes.POINTER(ZoloOpts)]
    lib.zolo_default_opts.restype = None
    lib.zolo_create.argtypes = [ctypes.POINTER(P), P]
    lib.zolo_set_stream.argtypes = [P, P]
    lib.zolo_destroy.argtypes = [P]
    lib.zolo_coeffs.argtypes = [c_double, c_int, D, D, D, D]
    lib.zolo_pd.argtypes = [P, c_int, c_int, P, c_int, c_double, c_double, c_int, P, c_int, P, c_int,
                            ctypes.POINTER(ZoloOpts), ctypes.POINTER(ZoloInfo)]
    lib.zolo_pd_noalloc.argtypes = lib.zolo_pd.argtypes
    lib.zolo_dsyevd.argtypes = [P, c_int, P, c_int, D, P, c_int]
    PP = ctypes.POINTER(c_void_p)
    IP = ctypes.POINTER(c_int)
    lib.zolo_pd_batched.argtypes = [P, c_int, IP, IP, PP, IP, D, D, IP, PP, IP, PP, IP,
                                    ctypes.POINTER(ZoloOpts), ctypes.POINTER(ZoloInfo)]
    lib.zolo_svd.argtypes = [P, c_int, c_int, P, c_int, c_double, c_double, c_int, P, c_int, D, P, c_int,
                             ctypes.POINTER(ZoloOpts), ctypes.POINTER(ZoloInfo)]
    lib.zolo_dgemm.argtypes = [P, c_int, c_int, c_int, c_int, c_int, c_double, P, c_int, c_longlong, P, c_int,
                               c_longlong, c_double, P, c_int, c_longlong, c_int]
    lib.zolo_sgemm.argtypes = [P, c_int, c_int, c_int, c_int, c_int, ctypes.c_float, P, c_int, c_longlong, P,
                               c_int, c_longlong, ctypes.c_float, P, c_int, c_longlong, c_int]
    lib.zolo_dpotrf_batched.argtypes = [P, c_int, P, c_int, c_longlong, c_int, ctypes.POINTER(c_int)]
    lib.zolo_spotrf_batched.argtypes = [P, c_int, P, c_int, c_longlong, c_int, ctypes.POINTER(c_int)]
    lib.zolo_dtrtri_batched.argtypes = [P, c_int, P, c_int, c_longlong, P, c_int, c_longlong, c_int]
    lib.zolo_strtri_batched.argtypes = [P, c_int, P, c_int, c_longlong, P, c_int, c_longlong, c_int]
    lib.zolo_structured_qr_batched.argtypes = [P, c_int, c_int, D, P, c_int, c_longlong, P, c_int, c_longlong,
                                               c_int, c_int]  # M, ldm, strideM, R, ldr, strideR, batch, form_q
    lib.zolo_stats_enable.argtypes = [c_int]
    lib.zolo_stats_reset.argtypes = []
    lib.zolo_autotune_enable.argtypes = [c_int]
    lib.zolo_autotune_reset.argtypes = []
    lib.zolo_stats_count.argtypes = []
    lib.zolo_stats_get.argtypes = [c_int, ctypes.c_char_p, c_int, ctypes.POINTER(c_longlong), D, D, D]
    F = ctypes.c_float
    U64 = ctypes.c_ulonglong
    lib.zolo_sketch_features.argtypes = [P, c_int, c_int, P, c_int, U64, D]
    lib.zolo_surrogate_features.argtypes = [P, c_int, IP, IP, P, c_int, U64, U64, P]
    lib.zolo_mlp_stats.argtypes = [P, c_int, P, P]
    lib.zolo_mlp_work_elems.argtypes = [c_int]
    lib.zolo_mlp_forward.argtypes = [P, c_int, P, P, P, P]
    lib.zolo_mlp_loss.argtypes = [P, c_int, P, P, F, F, P, ctypes.POINTER(F)]
    lib.zolo_mlp_backward.argtypes = [P, c_int, P, P, P, P]
    lib.zolo_mlp_adam.argtypes = [P, P, P, P, P, c_int, F, F, F, F]
    lib.zolo_mlp_train.argtypes = [P, c_int, c_int, c_int, P, P, P, P, P, P, c_int, F, F, F, P, P, P]
    lib.zolo_set_estimator.argtypes = [P, P, c_int]
    lib.zolo_choose_r.argtypes = [c_double]
    lib.zolo_predict.argtypes = [c_double, c_int, c_int, c_int, c_double, ctypes.c_char_p, D]
    lib.zolo_release_events.argtypes = []
    for name in EXPORTS:
        if name not in ("zolo_default_opts",):
            getattr(lib, name).restype = c_int
    lib.zolo_mlp_work_elems.restype = c_longlong
    _lib = lib
    return lib


def coeffs(l, r):
    """Host-only Zolotarev coefficients: dict(c, a, mhat, l_next)."""
    lib = load()
    c = (c_double * (2 * r))()
    a = (c_double * r)()
    mh = c_double()
    ln = c_double()
    rc = lib.zolo_coeffs(float(l), int(r), c, a, ctypes.byref(mh), ctypes.byref(ln))
    if rc != 0:
        raise ValueError(f"zolo_coeffs rejected l={l}, r={r} (code {rc})")
    return {"c": list(c), "a": list(a), "mhat": mh.value, "l_next": ln.value}


def predict(l, r, m, n, chol_switch=100.0):
    """The library's predicted schedule and milliseconds of a solve (host
    only): (kinds string, ms)."""
    kinds = ctypes.create_string_buffer(MAX_ITER + 1)
    ms = c_double()
    rc = load().zolo_predict(float(l), int(r), int(m), int(n), float(chol_switch), kinds, ctypes.byref(ms))
    if rc != 0:
        raise ValueError(f"zolo_predict rejected l={l}, r={r}, m={m}, n={n} (code {rc})")
    return kinds.value.decode(), ms.value


_live = []


def shutdown():
    """Close every open handle and release the library's HIP events.  Runs
    at interpreter exit (atexit), before the HIP runtime's own teardown."""
    for ref in list(_live):
        z = ref()
        if z is not None:
            z.close()
    _live.clear()
    if _lib is not None:
        _lib.zolo_release_events()


def stats_enable(on=True):
    load().zolo_stats_enable(int(on))


def stats_reset():
    load().zolo_stats_reset()


def autotune_enable(on=True):
    """Turn the GEMM tile autotuner on or off (results do not change)."""
    load().zolo_autotune_enable(int(on))


def autotune_reset():
    """Forget the autotuner's tile choices."""
    load().zolo_autotune_reset()


def stats():
    """Per-kernel launch statistics: {name: (launches, ms, flops, bytes)}."""
    lib = load()
    out = {}
    for i in range(lib.zolo_stats_count()):
        name = ctypes.create_string_buffer(128)
        n = c_longlong()
        ms = c_double()
        fl = c_double()
        by = c_double()
        if lib.zolo_stats_get(i, name, 128, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl),
                              ctypes.byref(by)) == 0:
            out[name.value.decode()] = (n.value, ms.value, fl.value, by.value)
    return out


def _torch():
    import torch
    return torch


def to_device(A, device="cuda:0"):
    """A host (m, n) float64 array -> a device tensor of shape (m, n) whose
    memory is column-major (leading dimension m), copied into one device
    buffer that the returned view keeps alive."""
    torch = _torch()
    import numpy as np
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    buf = torch.empty(m * n, dtype=torch.float64, device=device)
    buf.copy_(torch.from_numpy(np.asfortranarray(A).reshape(-1, order="F")))
    return buf.as_strided((m, n), (1, m))


def _colmajor(A):
    """(tensor whose memory is A column-major, leading dimension)."""
    if A.dim() == 2 and A.stride(0) == 1 and A.stride(1) >= max(1, A.shape[0]):
        return A, A.stride(1)
    return A.t().contiguous().t(), A.shape[0]


def _check_tensor(A, name):
    torch = _torch()
    if not isinstance(A, torch.Tensor) or A.device.type != "cuda" or A.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA/HIP tensor")


class ZoloError(RuntimeError):
    pass


def _raise(rc, what):
    if rc < 0:
        raise ValueError(f"{what}: argument {-rc} is invalid")
    raise ZoloError(f"{what}: {STATUS.get(rc, rc)} (code {rc})")


class Zolo:
    """A library handle bound to the current device and a HIP stream."""

    def __init__(self, stream=None):
        torch = _torch()
        self.lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the Zolo-PD library runs on HIP devices only")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = c_void_p()
        rc = self.lib.zolo_create(ctypes.byref(h), c_void_p(self.stream.cuda_stream))
        if rc != 0:
            _raise(rc, "zolo_create")
        self.h = h
        _live.append(weakref.ref(self))

    def close(self):
        """Wait for the handle's stream, then release the handle and its
        workspace (deterministic; also called by shutdown() at exit)."""
        if getattr(self, "h", None):
            self.stream.synchronize()
            self.lib.zolo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def options(**kw):
        o = ZoloOpts()
        load().zolo_default_opts(ctypes.byref(o))
        names = {"max_iter", "stop_rule", "tau", "chol_switch", "qr_variant", "precision", "compute_errors",
                 "l_source", "batch_streams", "r_policy"}
        for k, v in kw.items():
            if k not in names:
                raise TypeError(f"unknown option {k}")
            if k == "stop_rule" and isinstance(v, str):
                v = {"verified": 0, "paper": 1}[v]
            if k == "l_source" and isinstance(v, str):
                v = {"condest": 0, "learned": 1}[v]
            if k == "precision" and isinstance(v, str):
                v = {"fp64": 0, "mixed": 1}[v]
            if k == "r_policy" and isinstance(v, str):
                v = {"two-step": 0, "time": 1}[v]
            if k == "qr_variant" and isinstance(v, str):
                v = {"structured": 0, "dense": 1}[v]
            setattr(o, k, v)
        return o

    def pd(self, A, alpha=None, l=None, r=None, check=True, noalloc=False, **opts):
        """Polar decomposition A = Qp H.  Returns (Qp, H, info).  noalloc:
        through zolo_pd_noalloc (the library's fixed device scratch)."""
        torch = _torch()
        _check_tensor(A, "A")
        m, n = A.shape
        Ac, lda = _colmajor(A)
        Qbuf = torch.empty((n, m), dtype=torch.float64, device=A.device)
        Hbuf = torch.empty((n, n), dtype=torch.float64, device=A.device)
        o = self.options(**opts)
        info = ZoloInfo()
        fn = self.lib.zolo_pd_noalloc if noalloc else self.lib.zolo_pd
        rc = fn(self.h, m, n, c_void_p(Ac.data_ptr()), lda,
                float(alpha) if alpha is not None else 0.0,
                float(l) if l is not None else 0.0, int(r) if r is not None else 0,
                c_void_p(Qbuf.data_ptr()), m, c_void_p(Hbuf.data_ptr()), n,
                ctypes.byref(o), ctypes.byref(info))
        if check and rc not in (0, 1):
            _raise(rc, "zolo_pd_noalloc" if noalloc else "zolo_pd")
        return Qbuf.t(), Hbuf.t(), info.as_dict()

    def pd_batched(self, As, alphas=None, ls=None, rs=None, check=True, **opts):
        """Zolo-PD of a list of matrices of any shapes.  Returns (Qps, Hs, infos)."""
        torch = _torch()
        count = len(As)
        cols = [_colmajor(A) for A in As]
        for A in As:
            _check_tensor(A, "A")
        ms = (c_int * count)(*[A.shape[0] for A in As])
        ns = (c_int * count)(*[A.shape[1] for A in As])
        ldas = (c_int * count)(*[ld for _, ld in cols])
        Qb = [torch.empty((A.shape[1], A.shape[0]), dtype=torch.float64, device=A.device) for A in As]
        Hb = [torch.empty((A.shape[1], A.shape[1]), dtype=torch.float64, device=A.device) for A in As]
        Ap = (c_void_p * count)(*[c.data_ptr() for c, _ in cols])
        Qpp = (c_void_p * count)(*[q.data_ptr() for q in Qb])
        Hpp = (c_void_p * count)(*[x.data_ptr() for x in Hb])
        ldqs = (c_int * count)(*[A.shape[0] for A in As])
        ldhs = (c_int * count)(*[A.shape[1] for A in As])
        al = (c_double * count)(*alphas) if alphas is not None else None
        lv = (c_double * count)(*ls) if ls is not None else None
        rv = (c_int * count)(*rs) if rs is not None else None
        infos = (ZoloInfo * count)()
        o = self.options(**opts)
        rc = self.lib.zolo_pd_batched(self.h, count, ms, ns, Ap, ldas, al, lv, rv, Qpp, ldqs, Hpp, ldhs,
                                      ctypes.byref(o), infos)
        if check and rc not in (0, 1):
            _raise(rc, "zolo_pd_batched")
        return [q.t() for q in Qb], [x.t() for x in Hb], [i.as_dict() for i in infos]

    def svd(self, A, alpha=None, l=None, r=None, check=True, **opts):
        """Zolo-SVD A = U diag(S) V^T.  Returns (U, S (numpy), V, info)."""
        torch = _torch()
        import numpy as np
        _check_tensor(A, "A")
        m, n = A.shape
        Ac, lda = _colmajor(A)
        Ubuf = torch.empty((n, m), dtype=torch.float64, device=A.device)
        Vbuf = torch.empty((n, n), dtype=torch.float64, device=A.device)
        S = np.zeros(n)
        o = self.options(**opts)
        info = ZoloInfo()
        rc = self.lib.zolo_svd(self.h, m, n, c_void_p(Ac.data_ptr()), lda,
                               float(alpha) if alpha is not None else 0.0,
                               float(l) if l is not None else 0.0, int(r) if r is not None else 0,
                               c_void_p(Ubuf.data_ptr()), m, S.ctypes.data_as(ctypes.POINTER(c_double)),
                               c_void_p(Vbuf.data_ptr()), n, ctypes.byref(o), ctypes.byref(info))
        if check and rc not in (0, 1):
            _raise(rc, "zolo_svd")
        return Ubuf.t(), S, Vbuf.t(), info.as_dict()

    # -- building blocks ----------------------------------------------------
    @staticmethod
    def _stack_cm(X):
        """(batch, rows, cols) tensor -> contiguous buffer (batch, cols, rows)."""
        return X.transpose(-1, -2).contiguous()

    def _prefix(self, X):
        torch = _torch()
        if X.dtype == torch.float64:
            return "d"
        if X.dtype == torch.float32:
            return "s"
        raise TypeError("building blocks take float64 (FP64) or float32 (FP32) stacks")

    def gemm(self, A, B, C=None, transa=False, transb=False, alpha=1.0, beta=0.0):
        """Batched C = alpha op(A) op(B) + beta C on (batch, rows, cols) stacks
        (float64 -> zolo_dgemm, float32 -> zolo_sgemm)."""
        torch = _torch()
        p = self._prefix(A)
        Ab, Bb = self._stack_cm(A), self._stack_cm(B.to(A.dtype))
        batch = A.shape[0]
        m = A.shape[2] if transa else A.shape[1]
        k = A.shape[1] if transa else A.shape[2]
        n = B.shape[1] if transb else B.shape[2]
        if C is None:
            Cb = torch.zeros((batch, n, m), dtype=A.dtype, device=A.device)
        else:
            Cb = self._stack_cm(C.to(A.dtype))
        rc = getattr(self.lib, f"zolo_{p}gemm")(self.h, int(transa), int(transb), m, n, k, float(alpha),
                                                c_void_p(Ab.data_ptr()), A.shape[1], A.shape[1] * A.shape[2],
                                                c_void_p(Bb.data_ptr()), B.shape[1], B.shape[1] * B.shape[2],
                                                float(beta), c_void_p(Cb.data_ptr()), m, m * n, batch)
        if rc:
            _raise(rc, f"zolo_{p}gemm")
        return Cb.transpose(-1, -2)

    def potrf(self, Z):
        """Batched upper Cholesky of a (batch, n, n) stack: returns (R, info list)."""
        p = self._prefix(Z)
        Zb = self._stack_cm(Z)
        batch, n = Z.shape[0], Z.shape[1]
        info = (c_int * batch)()
        rc = getattr(self.lib, f"zolo_{p}potrf_batched")(self.h, n, c_void_p(Zb.data_ptr()), n, n * n, batch, info)
        if rc not in (0, 6):
            _raise(rc, f"zolo_{p}potrf_batched")
        return Zb.transpose(-1, -2), list(info)

    def trtri(self, R):
        torch = _torch()
        p = self._prefix(R)
        Rb = self._stack_cm(R)
        batch, n = R.shape[0], R.shape[1]
        Ib = torch.empty_like(Rb)
        rc = getattr(self.lib, f"zolo_{p}trtri_batched")(self.h, n, c_void_p(Rb.data_ptr()), n, n * n,
                                                         c_void_p(Ib.data_ptr()), n, n * n, batch)
        if rc:
            _raise(rc, f"zolo_{p}trtri_batched")
        return Ib.transpose(-1, -2)

    def syevd(self, A):
        """Symmetric eigen-decomposition of an (n, n) float64 device tensor
        (lower triangle read): (w numpy descending, Z device (n, n))."""
        torch = _torch()
        import numpy as np
        _check_tensor(A, "A")
        n = A.shape[0]
        Ac, lda = _colmajor(A)
        Zbuf = torch.empty((n, n), dtype=torch.float64, device=A.device)
        w = np.zeros(n)
        rc = self.lib.zolo_dsyevd(self.h, n, c_void_p(Ac.data_ptr()), lda, w.ctypes.data_as(ctypes.POINTER(c_double)),
                                  c_void_p(Zbuf.data_ptr()), n)
        if rc:
            _raise(rc, "zolo_dsyevd")
        return w, Zbuf.t()

    # -- learned l/r estimator (zolo_learn.h) -------------------------------
    def sketch_features(self, X0, seed):
        """Features (numpy, 39) of X0 (float64 device tensor, m x n)."""
        import numpy as np
        _check_tensor(X0, "X0")
        Xc, ld = _colmajor(X0)
        m, n = X0.shape
        out = np.zeros(NF)
        rc = self.lib.zolo_sketch_features(self.h, m, n, c_void_p(Xc.data_ptr()), ld, int(seed),
                                           out.ctypes.data_as(ctypes.POINTER(c_double)))
        if rc:
            _raise(rc, "zolo_sketch_features")
        return out

    def surrogate_features(self, sigma, ms, ns, seed, first_index=0):
        """Surrogate features (G4) of `count` spectra.  sigma: contiguous
        float64 device tensor (count, ldsigma), row b holding the ns[b] values
        of spectrum b; ms: row counts.  Returns a (count, 39) float64 device
        tensor (each feature vector contiguous)."""
        torch = _torch()
        count, ldsig = sigma.shape
        if not sigma.is_contiguous() or sigma.dtype != torch.float64:
            raise TypeError("sigma must be a contiguous float64 device tensor (count, ldsigma)")
        feat = torch.empty((count, NF), dtype=torch.float64, device=sigma.device)
        mv = (c_int * count)(*[int(x) for x in ms])
        nv = (c_int * count)(*[int(x) for x in ns])
        rc = self.lib.zolo_surrogate_features(self.h, count, mv, nv, c_void_p(sigma.data_ptr()), ldsig, int(seed),
                                              int(first_index), c_void_p(feat.data_ptr()))
        if rc:
            _raise(rc, "zolo_surrogate_features")
        return feat

    def mlp_stats(self, feat, params):
        rc = self.lib.zolo_mlp_stats(self.h, feat.shape[0], c_void_p(feat.data_ptr()), c_void_p(params.data_ptr()))
        if rc:
            _raise(rc, "zolo_mlp_stats")

    def mlp_work(self, batch):
        torch = _torch()
        return torch.zeros(int(self.lib.zolo_mlp_work_elems(batch)) + 4 * batch, dtype=torch.float32,
                           device="cuda")

    def mlp_forward(self, params, feat, work=None):
        """y (batch, 2) float32 for feature rows feat (batch, 39) float64."""
        torch = _torch()
        batch = feat.shape[0]
        work = self.mlp_work(batch) if work is None else work
        y = torch.empty((batch, 2), dtype=torch.float32, device=feat.device)
        rc = self.lib.zolo_mlp_forward(self.h, batch, c_void_p(params.data_ptr()), c_void_p(feat.data_ptr()),
                                       c_void_p(y.data_ptr()), c_void_p(work.data_ptr()))
        if rc:
            _raise(rc, "zolo_mlp_forward")
        return y, work

    def mlp_loss(self, y, t, q=0.1, c_r=0.1):
        torch = _torch()
        dy = torch.empty_like(y)
        loss = ctypes.c_float()
        rc = self.lib.zolo_mlp_loss(self.h, y.shape[0], c_void_p(y.data_ptr()), c_void_p(t.data_ptr()),
                                    float(q), float(c_r), c_void_p(dy.data_ptr()), ctypes.byref(loss))
        if rc:
            _raise(rc, "zolo_mlp_loss")
        return loss.value, dy

    def mlp_backward(self, params, work, dy):
        torch = _torch()
        grad = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=dy.device)
        rc = self.lib.zolo_mlp_backward(self.h, dy.shape[0], c_void_p(params.data_ptr()), c_void_p(work.data_ptr()),
                                        c_void_p(dy.data_ptr()), c_void_p(grad.data_ptr()))
        if rc:
            _raise(rc, "zolo_mlp_backward")
        return grad

    def mlp_adam(self, params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
        rc = self.lib.zolo_mlp_adam(self.h, c_void_p(params.data_ptr()), c_void_p(grad.data_ptr()),
                                    c_void_p(m.data_ptr()), c_void_p(v.data_ptr()), int(t), float(lr), float(b1),
                                    float(b2), float(eps))
        if rc:
            _raise(rc, "zolo_mlp_adam")

    def mlp_train(self, feat, t, idx, params, m, v, t0, lr, q=0.1, c_r=0.1, work=None, grad=None):
        """len(idx) // batch steps; idx is an int32 device tensor (steps, batch).
        Returns the per-step losses (float32 device tensor)."""
        torch = _torch()
        steps, batch = idx.shape
        work = self.mlp_work(batch) if work is None else work
        grad = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=feat.device) if grad is None else grad
        losses = torch.empty(steps, dtype=torch.float32, device=feat.device)
        rc = self.lib.zolo_mlp_train(self.h, steps, batch, feat.shape[0], c_void_p(feat.data_ptr()),
                                     c_void_p(t.data_ptr()), c_void_p(idx.data_ptr()), c_void_p(params.data_ptr()),
                                     c_void_p(m.data_ptr()), c_void_p(v.data_ptr()), int(t0), float(lr), float(q),
                                     float(c_r), c_void_p(work.data_ptr()), c_void_p(grad.data_ptr()),
                                     c_void_p(losses.data_ptr()))
        if rc:
            _raise(rc, "zolo_mlp_train")
        return losses

    def set_estimator(self, params):
        """Install trained parameters (numpy float32, 6928) or remove (None)."""
        import numpy as np
        if params is None:
            rc = self.lib.zolo_set_estimator(self.h, None, 0)
        else:
            p = np.ascontiguousarray(params, dtype=np.float32)
            rc = self.lib.zolo_set_estimator(self.h, c_void_p(p.ctypes.data), p.size)
        if rc:
            _raise(rc, "zolo_set_estimator")

    def structured_qr(self, Y, pivots=None, form_q=True):
        """QR of [Y_b; p_b I] (pivots given) or of Y_b (pivots None) for a
        (batch, m, n) stack.  Returns (Q or Householder vectors, R): Q is
        (batch, m + n, n) ((batch, m, n) without pivots)."""
        torch = _torch()
        batch, m, n = Y.shape
        e = n if pivots is not None else 0
        Mb = torch.zeros((batch, n, m + e), dtype=torch.float64, device=Y.device)
        Mb[:, :, :m] = Y.transpose(-1, -2)
        Rb = torch.empty((batch, n, n), dtype=torch.float64, device=Y.device)
        piv = (c_double * batch)(*[float(p) for p in pivots]) if pivots is not None else None
        rc = self.lib.zolo_structured_qr_batched(self.h, m, n, piv, c_void_p(Mb.data_ptr()), m + e, (m + e) * n,
                                                 c_void_p(Rb.data_ptr()), n, n * n, batch, int(form_q))
        if rc:
            _raise(rc, "zolo_structured_qr_batched")
        return Mb.transpose(-1, -2), Rb.transpose(-1, -2)


def choose_r(l):
    """The library's degree policy (host only)."""
    return int(load().zolo_choose_r(float(l)))


atexit.register(shutdown)
