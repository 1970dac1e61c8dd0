"""ctypes binding of libiht.so (the C ABI in include/iht.h).

Argument marshalling only: every step of the IHT path runs in the library's HIP kernels. torch
supplies device memory and the current stream. There is no CPU fallback: if the library is not
built, or no HIP device is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libiht.so")

OK, NOT_CONVERGED, STALLED = 0, 1, 2
EINVAL, ENOMEM, EDEVICE, ENONFINITE, EUNSUPPORTED = -1, -2, -3, -4, -5
FP64, FP32, MIXED_I8 = 0, 1, 2
GAUSSIAN, LOGISTIC = 0, 1
HOST_PTR, DEVICE_PTR = 0, 1
MAX_K = 4096

EXPORTS = ("iht_opts_default", "iht_geno_create", "iht_geno_destroy", "iht_geno_shape", "iht_stats_create",
           "iht_stats_destroy", "iht_stats_read", "iht_gradient", "iht_gradient_batch", "iht_project",
           "iht_project_hint", "iht_fit", "iht_fit_batch", "iht_cv", "iht_predict", "iht_server_create", "iht_server_submit", "iht_server_step",
           "iht_server_poll", "iht_server_info", "iht_server_destroy", "iht_batch_tuning", "iht_status_str",
           "iht_last_error", "iht_workspace_bytes", "iht_workspace_bytes_batch",
           "iht_gradient_noalloc", "iht_gradient_noalloc_max_bytes", "iht_geno_bytes", "iht_geno_create_in",
           "iht_stats_bytes", "iht_stats_create_in")


class IHTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("max_backtrack", ctypes.c_int32),
                ("c", ctypes.c_double), ("shrink", ctypes.c_double), ("precision", ctypes.c_int32),
                ("mixed_tol", ctypes.c_double), ("polish_iter", ctypes.c_int32), ("family", ctypes.c_int32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_uint64)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("slots_busy", ctypes.c_int32), ("stats_blocks", ctypes.c_int32),
                ("queued", ctypes.c_int64), ("running", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("turns", ctypes.c_int64), ("device_bytes", ctypes.c_int64)]


_lib = None


def load():
    """Load libiht.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1608_01398_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    PP = ctypes.POINTER(ctypes.c_void_p)
    L.iht_opts_default.argtypes = [ctypes.POINTER(Opts)]
    L.iht_opts_default.restype = None
    L.iht_geno_create.argtypes = [P, I64, I64, I64, I32, P, PP]
    L.iht_geno_bytes.argtypes = [I64, I64]
    L.iht_geno_bytes.restype = ctypes.c_uint64
    L.iht_geno_create_in.argtypes = [P, I64, I64, I64, P, ctypes.c_uint64, P, PP]
    L.iht_geno_create_in.restype = ctypes.c_int
    L.iht_stats_bytes.argtypes = [P]
    L.iht_stats_bytes.restype = ctypes.c_uint64
    L.iht_stats_create_in.argtypes = [P, P, P, ctypes.c_uint64, P, PP]
    L.iht_stats_create_in.restype = ctypes.c_int
    L.iht_geno_destroy.argtypes = [P]
    L.iht_geno_shape.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]
    L.iht_stats_create.argtypes = [P, P, P, PP]
    L.iht_stats_destroy.argtypes = [P]
    L.iht_stats_read.argtypes = [P, P, P, P]
    L.iht_gradient.argtypes = [P, P, P, P, I32, P]
    L.iht_gradient_batch.argtypes = [P, ctypes.POINTER(ctypes.c_void_p), I32, P, P, P]
    L.iht_gradient_noalloc.argtypes = [P, P, P, P, I32, P]
    L.iht_gradient_noalloc.restype = ctypes.c_int
    L.iht_gradient_noalloc_max_bytes.argtypes = []
    L.iht_gradient_noalloc_max_bytes.restype = ctypes.c_size_t
    L.iht_project.argtypes = [P, I64, I32, P, P, P]
    L.iht_project_hint.argtypes = [P, I64, I32, P, P, P, P]
    L.iht_fit.argtypes = [P, P, P, P, I32, I32, I32, ctypes.POINTER(Opts), P, P, P, P, ctypes.POINTER(I32), P]
    L.iht_fit_batch.argtypes = [P, ctypes.POINTER(ctypes.c_void_p), I32, P, I64, P, I32, I32, P, ctypes.POINTER(Opts),
                                P, P, P, P, P, P, P]
    L.iht_cv.argtypes = [P, P, P, I32, I32, P, I32, P, I32, ctypes.POINTER(Opts), P, ctypes.POINTER(I32), P, P, P, P,
                         ctypes.POINTER(I32), P]
    L.iht_predict.argtypes = [P, P, P, P, I32, P, I32, I32, P, P, P]
    L.iht_server_create.argtypes = [P, I32, I32, I64, P, I32, I32, ctypes.POINTER(Opts), P, PP]
    L.iht_server_submit.argtypes = [P, P, P, I64, I32, P, P, P, P, P, P, P, ctypes.POINTER(I64)]
    L.iht_server_step.argtypes = [P, ctypes.POINTER(I32)]
    L.iht_server_poll.argtypes = [P, I64, ctypes.POINTER(I32)]
    L.iht_server_info.argtypes = [P, ctypes.POINTER(ServerInfo)]
    L.iht_server_destroy.argtypes = [P]
    L.iht_batch_tuning.argtypes = [P, I32, ctypes.POINTER(I32)]
    for f in ("iht_geno_create", "iht_geno_destroy", "iht_geno_shape", "iht_stats_create", "iht_stats_destroy",
              "iht_stats_read", "iht_gradient", "iht_gradient_batch", "iht_project", "iht_project_hint", "iht_fit",
              "iht_fit_batch", "iht_cv", "iht_predict", "iht_server_create", "iht_server_submit", "iht_server_step",
              "iht_server_poll", "iht_server_info", "iht_server_destroy", "iht_batch_tuning"):
        getattr(L, f).restype = ctypes.c_int
    L.iht_workspace_bytes.argtypes = [I64, I64, I32, I32, I32]
    L.iht_workspace_bytes.restype = ctypes.c_size_t
    L.iht_workspace_bytes_batch.argtypes = [I64, I64, I32, I32, I32, I32]
    L.iht_workspace_bytes_batch.restype = ctypes.c_size_t
    L.iht_status_str.argtypes = [ctypes.c_int]
    L.iht_status_str.restype = ctypes.c_char_p
    L.iht_last_error.argtypes = []
    L.iht_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc, allow_warnings=False):
    if rc < 0 or (rc > 0 and not allow_warnings):
        L = load()
        raise IHTError(rc, L.iht_last_error().decode() or L.iht_status_str(rc).decode())
    return rc


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device: the IHT library runs only on the GPU")
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, shape=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def default_opts(**kw):
    """iht_opts with the library defaults and the given fields; `workspace` may be a CUDA tensor (its
    bytes become the workspace; the caller keeps it alive for the call)."""
    o = Opts()
    load().iht_opts_default(ctypes.byref(o))
    ws = kw.pop("workspace", None)
    for k, v in kw.items():
        if not hasattr(o, k) or k == "workspace_bytes":
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    if ws is not None:
        torch = _torch()
        if not isinstance(ws, torch.Tensor) or not ws.is_cuda or not ws.is_contiguous():
            raise TypeError("workspace must be a contiguous CUDA tensor")
        o.workspace = ws.data_ptr()
        o.workspace_bytes = ws.numel() * ws.element_size()
    return o


def workspace_bytes(n: int, p: int, k: int, c: int, precision: int = 0, T: int | None = None) -> int:
    """Device bytes of the workspace of one fit (iht_workspace_bytes) or of T solves with model sizes up
    to k (iht_workspace_bytes_batch); c = unpenalised columns (covariates + intercept)."""
    L = load()
    if T is None:
        return int(L.iht_workspace_bytes(n, p, k, c, precision))
    return int(L.iht_workspace_bytes_batch(n, p, T, k, c, precision))


class Geno:
    """Resident, re-tiled PLINK genotype matrix (iht_geno_create). With borrow=True the re-tiled
    matrix lives in a torch tensor (`self.storage`) that the handle borrows (iht_geno_create_in: the
    library allocates no device memory for it); `bed` is then uploaded to the device first."""

    def __init__(self, bed, n: int, borrow: bool = False):
        torch = _torch()
        L = load()
        self._h = ctypes.c_void_p()
        self.storage = None
        if borrow:
            src = bed if isinstance(bed, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(bed, dtype=np.uint8))
            if src.dtype != torch.uint8 or src.dim() != 2:
                raise TypeError("bed must be a 2-D uint8 array [p, row_bytes]")
            src = src.to("cuda").contiguous()
            p, rb = src.shape
            nbytes = int(L.iht_geno_bytes(n, p))
            if nbytes == 0:
                raise ValueError("n or p out of range")
            self.storage = torch.empty(nbytes, dtype=torch.uint8, device="cuda")  # 256-byte aligned by torch
            _check(L.iht_geno_create_in(ctypes.c_void_p(src.data_ptr()), n, p, rb, ctypes.c_void_p(self.storage.data_ptr()),
                                        nbytes, _stream(), ctypes.byref(self._h)))
            self._pid = os.getpid()
            self.n, self.p = int(n), int(p)
            return
        if isinstance(bed, torch.Tensor):
            if bed.dtype != torch.uint8 or bed.dim() != 2:
                raise TypeError("bed must be a 2-D uint8 tensor [p, row_bytes]")
            bed = bed.contiguous()
            flags = DEVICE_PTR if bed.is_cuda else HOST_PTR
            ptr = ctypes.c_void_p(bed.data_ptr())
            p, rb = bed.shape
            keep = bed
        else:
            keep = np.ascontiguousarray(bed, dtype=np.uint8)
            p, rb = keep.shape
            flags = HOST_PTR
            ptr = keep.ctypes.data_as(ctypes.c_void_p)
        _check(L.iht_geno_create(ptr, n, p, rb, flags, _stream(), ctypes.byref(self._h)))
        self._pid = os.getpid()
        del keep
        self.n, self.p = int(n), int(p)

    def close(self):
        # only the creating process may free the device memory: a forked child (a worker pool
        # started after the handle existed) holds a copy of the object but no usable device state
        if getattr(self, "_h", None) and self._h.value and getattr(self, "_pid", None) == os.getpid():
            load().iht_geno_destroy(self._h)
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stats:
    """u, v over a subject subset (iht_stats_create). With borrow=True they live in a torch tensor
    (`self.storage`) that the handle borrows (iht_stats_create_in)."""

    def __init__(self, geno: Geno, subset=None, borrow: bool = False):
        L = load()
        self.geno = geno
        self._h = ctypes.c_void_p()
        self.storage = None
        m = None
        if subset is not None:
            m = np.ascontiguousarray(subset, dtype=np.uint8)
            if m.shape != (geno.n,):
                raise ValueError("subset must have n entries")
        mp = None if m is None else m.ctypes.data_as(ctypes.c_void_p)
        if borrow:
            torch = _torch()
            nbytes = int(L.iht_stats_bytes(geno._h))
            self.storage = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            _check(L.iht_stats_create_in(geno._h, mp, ctypes.c_void_p(self.storage.data_ptr()), nbytes, _stream(),
                                         ctypes.byref(self._h)))
        else:
            _check(L.iht_stats_create(geno._h, mp, _stream(), ctypes.byref(self._h)))
        self._pid = os.getpid()

    def read(self):
        torch = _torch()
        u = torch.empty(self.geno.p, dtype=torch.float64, device="cuda")
        v = torch.empty(self.geno.p, dtype=torch.float64, device="cuda")
        _check(load().iht_stats_read(self._h, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(v.data_ptr()), _stream()))
        return u, v

    def close(self):
        if getattr(self, "_h", None) and self._h.value and getattr(self, "_pid", None) == os.getpid():
            load().iht_stats_destroy(self._h)
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gradient(geno: Geno, stats: Stats, r, precision: int = FP64, out=None):
    """g = X_st^T r (iht_gradient). r: float64 CUDA tensor [n]."""
    torch = _torch()
    rp = _dev(r, torch.float64, (geno.n,), "r")
    if out is None:
        out = torch.empty(geno.p, dtype=torch.float64, device=r.device)
    gp = _dev(out, torch.float64, (geno.p,), "out")
    _check(load().iht_gradient(geno._h, stats._h, rp, gp, precision, _stream()))
    return out


def gradient_noalloc(geno: Geno, stats: Stats, r, out, precision: int = FP64):
    """g = X_st^T r into the preallocated `out` (iht_gradient_noalloc: the library allocates nothing)."""
    torch = _torch()
    rp = _dev(r, torch.float64, (geno.n,), "r")
    gp = _dev(out, torch.float64, (geno.p,), "out")
    _check(load().iht_gradient_noalloc(geno._h, stats._h, rp, gp, precision, _stream()))
    return out


def gradient_batch(geno: Geno, stats, R, out=None):
    """G[t] = X_st^T R[t] for T solves (iht_gradient_batch). stats: one Stats per solve; R: float64 CUDA [T, n]."""
    torch = _torch()
    T = len(stats)
    rp = _dev(R, torch.float64, (T, geno.n), "R")
    if out is None:
        out = torch.empty((T, geno.p), dtype=torch.float64, device=R.device)
    gp = _dev(out, torch.float64, (T, geno.p), "out")
    arr = (ctypes.c_void_p * T)(*[s._h.value for s in stats])
    _check(load().iht_gradient_batch(geno._h, arr, T, rp, gp, _stream()))
    return out


def project(w, k: int, hint=None):
    """(support int64 [k] ascending, w_out [p]) of the k largest |w| (iht_project; with `hint`, k
    distinct indices such as the previous support, iht_project_hint)."""
    torch = _torch()
    wp = _dev(w, torch.float64, None, "w")
    p = w.shape[0]
    sup = torch.empty(k, dtype=torch.int64, device=w.device)
    out = torch.empty(p, dtype=torch.float64, device=w.device)
    if hint is None:
        _check(load().iht_project(wp, p, k, ctypes.c_void_p(sup.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  _stream()))
    else:
        hp = _dev(hint, torch.int64, (k,), "hint")
        _check(load().iht_project_hint(wp, p, k, hp, ctypes.c_void_p(sup.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), _stream()))
    return sup, out


def fit(geno: Geno, stats: Stats, y, k: int, Z=None, intercept: bool = True, **opts):
    """Full IHT solve (iht_fit). y: float64 CUDA [n]; Z: float32 CUDA [c, n] (column-major [n x c]) or None.

    Returns dict(status, support, beta_S, beta_cov, loss_trace, n_iter) with device tensors.
    """
    torch = _torch()
    o = default_opts(**opts)
    yp = _dev(y, torch.float64, (geno.n,), "y")
    cz = 0
    zp = None
    if Z is not None:
        cz = Z.shape[0]
        zp = _dev(Z, torch.float32, (cz, geno.n), "Z")
    nc = cz + (1 if intercept else 0)
    dev = y.device
    sup = torch.empty(k, dtype=torch.int64, device=dev)
    bS = torch.empty(k, dtype=torch.float64, device=dev)
    bc = torch.empty(max(nc, 1), dtype=torch.float64, device=dev)
    trace = torch.full((o.max_iter + 1,), float("nan"), dtype=torch.float64, device=dev)
    nit = ctypes.c_int32(0)
    rc = load().iht_fit(geno._h, stats._h, yp, zp, cz, 1 if intercept else 0, k, ctypes.byref(o),
                        ctypes.c_void_p(sup.data_ptr()), ctypes.c_void_p(bS.data_ptr()),
                        ctypes.c_void_p(bc.data_ptr()) if nc else None, ctypes.c_void_p(trace.data_ptr()),
                        ctypes.byref(nit), _stream())
    _check(rc, allow_warnings=True)
    it = nit.value
    return dict(status=rc, support=sup, beta_S=bS, beta_cov=bc[:nc], loss_trace=trace[:it + 1], n_iter=it)


def fit_batch(geno: Geno, stats, Y, ks, Z=None, intercept: bool = True, **opts):
    """T lock-step IHT solves sharing the genotypes (iht_fit_batch).

    stats: T Stats handles; Y: float64 CUDA [T, n] (row t = trait of solve t); ks: T model sizes;
    Z: float32 CUDA [c, n] shared covariates or None. Returns dict(status (call), statuses [T], support
    [T, kmax] (-1 past k_t), beta_S [T, kmax], beta_cov [T, nc], loss_trace [T, max_iter+1], n_iter [T]).
    """
    torch = _torch()
    o = default_opts(**opts)
    T = len(stats)
    if len(ks) != T:
        raise ValueError("ks must have one entry per solve")
    yp = _dev(Y, torch.float64, (T, geno.n), "Y")
    cz = 0
    zp = None
    if Z is not None:
        cz = Z.shape[0]
        zp = _dev(Z, torch.float32, (cz, geno.n), "Z")
    nc = cz + (1 if intercept else 0)
    kmax = int(max(ks))
    dev = Y.device
    sup = torch.empty((T, kmax), dtype=torch.int64, device=dev)
    bS = torch.empty((T, kmax), dtype=torch.float64, device=dev)
    bc = torch.empty((T, max(nc, 1)), dtype=torch.float64, device=dev)
    trace = torch.full((T, o.max_iter + 1), float("nan"), dtype=torch.float64, device=dev)
    ks_arr = np.ascontiguousarray(ks, dtype=np.int32)
    nit = np.zeros(T, dtype=np.int32)
    st = np.zeros(T, dtype=np.int32)
    arr = (ctypes.c_void_p * T)(*[s._h.value for s in stats])
    rc = load().iht_fit_batch(geno._h, arr, T, yp, geno.n, zp, cz, 1 if intercept else 0,
                              ks_arr.ctypes.data_as(ctypes.c_void_p), ctypes.byref(o),
                              ctypes.c_void_p(sup.data_ptr()), ctypes.c_void_p(bS.data_ptr()),
                              ctypes.c_void_p(bc.data_ptr()) if nc else None, ctypes.c_void_p(trace.data_ptr()),
                              nit.ctypes.data_as(ctypes.c_void_p), st.ctypes.data_as(ctypes.c_void_p), _stream())
    if rc < 0 and rc != ENONFINITE:
        _check(rc)
    return dict(status=rc, statuses=st, support=sup, beta_S=bS, beta_cov=bc[:, :nc], loss_trace=trace, n_iter=nit)


def cv(geno: Geno, y, ks, folds, q: int, Z=None, intercept: bool = True, **opts):
    """q-fold cross-validation over the model sizes ks, then the refit at the chosen size (iht_cv).

    y: float64 CUDA [n]; folds: host uint8 [n] (fold of each subject, < q); Z as in fit. Returns
    dict(mse (numpy [len(ks), q]), k_best, refit=dict as returned by fit).
    """
    torch = _torch()
    o = default_opts(**opts)
    yp = _dev(y, torch.float64, (geno.n,), "y")
    cz = 0
    zp = None
    if Z is not None:
        cz = Z.shape[0]
        zp = _dev(Z, torch.float32, (cz, geno.n), "Z")
    nc = cz + (1 if intercept else 0)
    folds = np.ascontiguousarray(folds, dtype=np.uint8)
    if folds.shape != (geno.n,):
        raise ValueError(f"folds must have shape ({geno.n},)")
    ks_arr = np.ascontiguousarray(ks, dtype=np.int32)
    r = ks_arr.size
    kmax = int(ks_arr.max()) if r else 1
    dev = y.device
    mse = np.zeros((r, q), dtype=np.float64)
    kb = ctypes.c_int32(0)
    sup = torch.empty(kmax, dtype=torch.int64, device=dev)
    bS = torch.empty(kmax, dtype=torch.float64, device=dev)
    bc = torch.empty(max(nc, 1), dtype=torch.float64, device=dev)
    trace = torch.full((o.max_iter + 1,), float("nan"), dtype=torch.float64, device=dev)
    nit = ctypes.c_int32(0)
    rc = load().iht_cv(geno._h, yp, zp, cz, 1 if intercept else 0, folds.ctypes.data_as(ctypes.c_void_p), q,
                       ks_arr.ctypes.data_as(ctypes.c_void_p), r, ctypes.byref(o),
                       mse.ctypes.data_as(ctypes.c_void_p), ctypes.byref(kb), ctypes.c_void_p(sup.data_ptr()),
                       ctypes.c_void_p(bS.data_ptr()), ctypes.c_void_p(bc.data_ptr()) if nc else None,
                       ctypes.c_void_p(trace.data_ptr()), ctypes.byref(nit), _stream())
    _check(rc, allow_warnings=True)
    k = kb.value
    it = nit.value
    refit = dict(status=rc, support=sup[:k], beta_S=bS[:k], beta_cov=bc[:nc], loss_trace=trace[:it + 1], n_iter=it)
    return dict(mse=mse, k_best=k, refit=refit)


def predict(geno: Geno, stats: Stats, support, beta_S, Z=None, intercept: bool = False, beta_cov=None):
    """Prediction of every subject, X_st[:, support] beta_S (+ covariates), standardised with stats (iht_predict).

    support: int64 CUDA [k]; beta_S: float64 CUDA [k]; Z: float32 CUDA [c, n] or None; beta_cov: float64
    CUDA [c + intercept] when covariates or the intercept are used. Returns float64 CUDA [n].
    """
    torch = _torch()
    k = int(support.numel())
    sp = _dev(support, torch.int64, (k,), "support") if k else None
    bp = _dev(beta_S, torch.float64, (k,), "beta_S") if k else None
    cz = 0
    zp = None
    if Z is not None:
        cz = Z.shape[0]
        zp = _dev(Z, torch.float32, (cz, geno.n), "Z")
    nc = cz + (1 if intercept else 0)
    cp = _dev(beta_cov, torch.float64, (nc,), "beta_cov") if nc else None
    out = torch.empty(geno.n, dtype=torch.float64, device=support.device)
    _check(load().iht_predict(geno._h, stats._h, sp, bp, k, zp, cz, 1 if intercept else 0, cp,
                              ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


def batch_tuning(geno: Geno, T: int) -> int:
    """SNPs per workgroup the autotuner chose for the matrix-core pass over T solves (0: not tuned yet)."""
    v = ctypes.c_int32(0)
    _check(load().iht_batch_tuning(geno._h, T, ctypes.byref(v)))
    return v.value


class Server:
    """Solve server with continuous batching over one resident matrix (iht_server_*).

    Requests (a subject subset, T traits, a model size per trait) are admitted between turns as slots
    and statistics blocks free up; step() advances every admitted solve by one turn and writes out
    the finished ones. Every result is the same alone and in any mix.
    """

    def __init__(self, geno: Geno, slots: int, kmax: int, hbm_budget: int, Z=None, intercept: bool = True,
                 **opts):
        torch = _torch()
        self.geno = geno
        self.o = default_opts(**opts)
        self.kmax = int(kmax)
        cz = 0
        zp = None
        self._Z = Z
        if Z is not None:
            cz = Z.shape[0]
            zp = _dev(Z, torch.float32, (cz, geno.n), "Z")
        self.nc = cz + (1 if intercept else 0)
        self._h = ctypes.c_void_p()
        _check(load().iht_server_create(geno._h, slots, kmax, int(hbm_budget), zp, cz, 1 if intercept else 0,
                                        ctypes.byref(self.o), _stream(), ctypes.byref(self._h)))
        self._pid = os.getpid()
        self._req = {}

    def submit(self, Y, ks, subset=None) -> int:
        """Queue a request: Y float64 CUDA [T, n] (kept alive until done), ks [T], subset host 0/1 [n] or None."""
        torch = _torch()
        ks_arr = np.ascontiguousarray(ks, dtype=np.int32)
        T = int(ks_arr.size)
        yp = _dev(Y, torch.float64, (T, self.geno.n), "Y")
        m = None
        if subset is not None:
            m = np.ascontiguousarray(subset, dtype=np.uint8)
            if m.shape != (self.geno.n,):
                raise ValueError("subset must have n entries")
        kr = int(ks_arr.max())
        dev = Y.device
        out = dict(support=torch.empty((T, kr), dtype=torch.int64, device=dev),
                   beta_S=torch.empty((T, kr), dtype=torch.float64, device=dev),
                   beta_cov=torch.empty((T, max(self.nc, 1)), dtype=torch.float64, device=dev),
                   loss_trace=torch.full((T, self.o.max_iter + 1), float("nan"), dtype=torch.float64, device=dev),
                   n_iter=np.zeros(T, dtype=np.int32), statuses=np.zeros(T, dtype=np.int32))
        rid = ctypes.c_int64(0)
        _check(load().iht_server_submit(
            self._h, None if m is None else m.ctypes.data_as(ctypes.c_void_p), yp, self.geno.n, T,
            ks_arr.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(out["support"].data_ptr()),
            ctypes.c_void_p(out["beta_S"].data_ptr()),
            ctypes.c_void_p(out["beta_cov"].data_ptr()) if self.nc else None,
            ctypes.c_void_p(out["loss_trace"].data_ptr()), out["n_iter"].ctypes.data_as(ctypes.c_void_p),
            out["statuses"].ctypes.data_as(ctypes.c_void_p), ctypes.byref(rid)))
        self._req[rid.value] = (out, Y, ks_arr, m)  # keep inputs and outputs alive
        return rid.value

    def step(self) -> int:
        """Admit what fits, run one turn, write out what finished. Returns the requests completed."""
        c = ctypes.c_int32(0)
        _check(load().iht_server_step(self._h, ctypes.byref(c)))
        return c.value

    def done(self, rid: int) -> bool:
        d = ctypes.c_int32(0)
        _check(load().iht_server_poll(self._h, rid, ctypes.byref(d)))
        return bool(d.value)

    def result(self, rid: int):
        """The finished request's outputs (dict as fit_batch: support [T, kr], beta_S, beta_cov [T, nc],
        loss_trace [T, max_iter+1], n_iter [T], statuses [T]); releases the server's reference."""
        if not self.done(rid):
            raise RuntimeError(f"request {rid} has not finished")
        out, _, ks, _ = self._req.pop(rid)
        res = dict(out)
        res["beta_cov"] = out["beta_cov"][:, :self.nc]
        res["ks"] = ks
        return res

    def info(self) -> dict:
        i = ServerInfo()
        _check(load().iht_server_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in ServerInfo._fields_}

    def run_until_idle(self, max_steps: int = 100000):
        """Step until nothing is queued or running."""
        for _ in range(max_steps):
            inf = self.info()
            if inf["queued"] == 0 and inf["running"] == 0:
                return
            self.step()
        raise RuntimeError("server did not drain")

    def close(self):
        if getattr(self, "_h", None) and self._h.value and getattr(self, "_pid", None) == os.getpid():
            load().iht_server_destroy(self._h)
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
