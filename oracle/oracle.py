"""NumPy front end of the FP64 CPU oracle (``iht_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the benchmark's
CPU-baseline leg, never by the device library or its binding. It shares no code with the device
path; the only thing both sides consume is the seeded input generator.

Every function here is a thin ctypes call; the arithmetic lives in ``iht_oracle.c``, which cites
the paper's equations and sections for each step.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "iht_oracle.c")
_LIB = os.path.join(_HERE, "libiht_oracle.so")

OK, NOT_CONVERGED, STALLED = 0, 1, 2
EINVAL, ENOMEM, ENONFINITE = -1, -2, -4

# Defaults of the readings the paper leaves open (c, shrink, backtracking budget, stopping rule).
DEFAULTS = dict(tol=1e-10, max_iter=200, max_backtrack=50, c=0.01, shrink=0.5)


def build(force: bool = True) -> str:
    """Compile the oracle with plain gcc: -O2, no FP contraction, OpenMP over SNPs."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.iht_ref_decode.argtypes = [P, I64, I64, I64, P]
        L.iht_ref_stats.argtypes = [P, I64, I64, I64, P, P, P]
        L.iht_ref_standardize.argtypes = [P, I64, I64, I64, P, P, P]
        L.iht_ref_gradient.argtypes = [P, I64, I64, I64, P, P, P, P, P]
        L.iht_ref_project.argtypes = [P, I64, I32, P, P]
        L.iht_ref_fit.argtypes = [P, I64, I64, I64, P, P, P, I32, I32, I32, D, I32, I32, D, D, P, P, P, P, P, P]
        L.iht_ref_fit_family.argtypes = [P, I64, I64, I64, P, P, P, I32, I32, I32, D, I32, I32, D, D, I32, P, P, P, P, P,
                                         P]
        L.iht_ref_cv.argtypes = [P, I64, I64, I64, P, I32, P, P, I32, I32, P, I32, D, I32, I32, D, D, P, P]
        L.iht_ref_predict.argtypes = [P, I64, I64, I64, P, P, P, P, I32, P, I32, I32, P, P]
        for f in (L.iht_ref_decode, L.iht_ref_stats, L.iht_ref_standardize, L.iht_ref_gradient, L.iht_ref_project,
                  L.iht_ref_fit, L.iht_ref_cv, L.iht_ref_predict, L.iht_ref_fit_family):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _bed(bed):
    bed = np.ascontiguousarray(bed, dtype=np.uint8)
    return bed, bed.shape[0], bed.shape[1]


def _mask(subset, n):
    if subset is None:
        return None
    m = np.ascontiguousarray(subset, dtype=np.uint8)
    assert m.shape == (n,)
    return m


def decode(bed, n):
    """Dosage matrix [p, n] int8 (0/1/2, -1 = missing)."""
    bed, p, rb = _bed(bed)
    out = np.empty((p, n), dtype=np.int8)
    rc = lib().iht_ref_decode(_p(bed), n, p, rb, _p(out))
    if rc:
        raise ValueError(f"iht_ref_decode: {rc}")
    return out


def stats(bed, n, subset=None):
    bed, p, rb = _bed(bed)
    u = np.empty(p)
    v = np.empty(p)
    m = _mask(subset, n)
    rc = lib().iht_ref_stats(_p(bed), n, p, rb, _p(m), _p(u), _p(v))
    if rc:
        raise ValueError(f"iht_ref_stats: {rc}")
    return u, v


def standardize(bed, n, u, v):
    bed, p, rb = _bed(bed)
    out = np.empty((p, n))
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    rc = lib().iht_ref_standardize(_p(bed), n, p, rb, _p(u), _p(v), _p(out))
    if rc:
        raise ValueError(f"iht_ref_standardize: {rc}")
    return out


def gradient(bed, n, u, v, r, subset=None):
    bed, p, rb = _bed(bed)
    g = np.empty(p)
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    assert r.shape == (n,)
    m = _mask(subset, n)
    rc = lib().iht_ref_gradient(_p(bed), n, p, rb, _p(u), _p(v), _p(m), _p(r), _p(g))
    if rc:
        raise ValueError(f"iht_ref_gradient: {rc}")
    return g


def project(w, k):
    """(support ascending [k] int64, w_out [p]) for the k largest |w|, ties to the lower index."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    p = w.shape[0]
    sup = np.empty(k, dtype=np.int64)
    out = np.empty(p)
    rc = lib().iht_ref_project(_p(w), p, k, _p(sup), _p(out))
    if rc:
        raise ValueError(f"iht_ref_project: {rc}")
    return sup, out


def fit(bed, n, y, k, Z=None, intercept=True, subset=None, family=0, **opts):
    """Plain FP64 IHT. Z: float32 covariates as a [c, n] array (column-major [n x c]); family 0: least
    squares, 1: logistic (y in [0, 1]).

    Returns a dict with status, support, beta_S, beta_cov, loss_trace[:n_iter+1], n_iter, mu_trace.
    """
    o = dict(DEFAULTS)
    o.update(opts)
    bed, p, rb = _bed(bed)
    y = np.ascontiguousarray(y, dtype=np.float64)
    assert y.shape == (n,)
    cz = 0
    if Z is not None:
        Z = np.ascontiguousarray(Z, dtype=np.float32)
        cz = Z.shape[0]
        assert Z.shape == (cz, n)
    nc = cz + (1 if intercept else 0)
    m = _mask(subset, n)
    sup = np.empty(k, dtype=np.int64)
    bS = np.empty(k)
    bc = np.empty(max(nc, 1))
    trace = np.full(o["max_iter"] + 1, np.nan)
    mu = np.full(max(o["max_iter"], 1), np.nan)
    nit = ctypes.c_int32(0)
    rc = lib().iht_ref_fit_family(_p(bed), n, p, rb, _p(m), _p(y), _p(Z), cz, 1 if intercept else 0, k, o["tol"],
                                  o["max_iter"], o["max_backtrack"], o["c"], o["shrink"], family, _p(sup), _p(bS), _p(bc),
                                  _p(trace), ctypes.byref(nit), _p(mu))
    if rc < 0:
        raise ValueError(f"iht_ref_fit: {rc}")
    it = nit.value
    return dict(status=rc, support=sup, beta_S=bS, beta_cov=bc[:nc], loss_trace=trace[:it + 1], n_iter=it,
                mu_trace=mu[:it])


def cv(bed, n, y, ks, folds, q, Z=None, intercept=True, **opts):
    """q-fold cross-validation over the model sizes ks (Methods, "Model selection"), then the refit
    on every subject with the chosen k. folds: [n] fold index of each subject (0..q-1).

    Returns dict(mse [len(ks), q] held-out mean squared errors, k_best, refit = fit(...)).
    """
    o = dict(DEFAULTS)
    o.update(opts)
    bed_c, p, rb = _bed(bed)
    y = np.ascontiguousarray(y, dtype=np.float64)
    folds = np.ascontiguousarray(folds, dtype=np.uint8)
    assert y.shape == (n,) and folds.shape == (n,)
    ks = np.ascontiguousarray(ks, dtype=np.int32)
    cz = 0
    if Z is not None:
        Z = np.ascontiguousarray(Z, dtype=np.float32)
        cz = Z.shape[0]
    mse = np.empty((len(ks), q))
    kb = ctypes.c_int32(0)
    rc = lib().iht_ref_cv(_p(bed_c), n, p, rb, _p(folds), q, _p(y), _p(Z), cz, 1 if intercept else 0, _p(ks), len(ks),
                          o["tol"], o["max_iter"], o["max_backtrack"], o["c"], o["shrink"], _p(mse), ctypes.byref(kb))
    if rc < 0:
        raise ValueError(f"iht_ref_cv: {rc}")
    refit = fit(bed, n, y, kb.value, Z=Z, intercept=intercept, **opts)
    return dict(mse=mse, k_best=kb.value, refit=refit)


def predict(bed, n, u, v, support, beta_S, Z=None, intercept=False, beta_cov=None):
    """Prediction of every subject by a fitted model (the X_st beta product of Methods, "Bandwidth
    optimization of IHT"), standardised with u, v; plus covariates and intercept if given."""
    bed_c, p, rb = _bed(bed)
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    sup = np.ascontiguousarray(support, dtype=np.int64)
    b = np.ascontiguousarray(beta_S, dtype=np.float64)
    cz = 0
    if Z is not None:
        Z = np.ascontiguousarray(Z, dtype=np.float32)
        cz = Z.shape[0]
    bc = None if beta_cov is None else np.ascontiguousarray(beta_cov, dtype=np.float64)
    out = np.empty(n)
    rc = lib().iht_ref_predict(_p(bed_c), n, p, rb, _p(u), _p(v), _p(sup), _p(b), sup.size, _p(Z), cz,
                               1 if intercept else 0, _p(bc), _p(out))
    if rc < 0:
        raise ValueError(f"iht_ref_predict: {rc}")
    return out
