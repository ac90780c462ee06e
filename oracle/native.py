"""ctypes front end of the C oracle ``c/oracle.c`` (test infrastructure only).

The shared object is built by ``build()`` (plain gcc -O2, no fast-math) next to
its source; ``load()`` builds it on first use when it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "c", "oracle.c")
_LIB = os.path.join(_HERE, "c", "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build() -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    i64 = ctypes.c_int64
    lib.spo_state_dim.argtypes = [ctypes.c_int, _ip, _ip, _dp]
    lib.spo_edges.argtypes = [ctypes.c_int, _ip, _ip, _dp, i64, _dp, _dp, _dp, _dp, _dp]
    lib.spo_btd_factored.argtypes = [ctypes.c_int, _ip, _ip, _dp, i64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.spo_tangent_grad.argtypes = [ctypes.c_int, _ip, _ip, _dp, i64, _dp, _dp, _dp, _dp]
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _terms(terms):
    kinds = np.ascontiguousarray([k for k, _ in terms], dtype=np.int32)
    harm = np.ascontiguousarray([h for _, h in terms], dtype=np.int32)
    return kinds, harm


def state_dim(terms, hyper_row) -> int:
    kinds, harm = _terms(terms)
    hyper_row = np.ascontiguousarray(hyper_row, dtype=np.float64)
    return load().spo_state_dim(len(terms), kinds.ctypes.data_as(_ip), harm.ctypes.data_as(_ip), _ptr(hyper_row))


def edges(terms, hyper_row, t):
    """Closed-form (A_n, Q_n) for every edge, plus (P0, h)."""
    lib = load()
    kinds, harm = _terms(terms)
    hyper_row = np.ascontiguousarray(hyper_row, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    b = state_dim(terms, hyper_row)
    n = t.shape[0]
    A = np.zeros((max(n - 1, 0), b, b))
    Q = np.zeros((max(n - 1, 0), b, b))
    P = np.zeros((b, b))
    h = np.zeros(b)
    rc = lib.spo_edges(len(terms), kinds.ctypes.data_as(_ip), harm.ctypes.data_as(_ip), _ptr(hyper_row),
                       n, _ptr(t), _ptr(A), _ptr(Q), _ptr(P), _ptr(h))
    if rc:
        raise RuntimeError(f"spo_edges failed ({rc})")
    return A, Q, P, h


def btd_factored(terms, hyper_row, t, y, want_blocks: bool = True) -> dict:
    """Sequential BTD elimination of one series: logML, mean, variance, selected inverse."""
    lib = load()
    kinds, harm = _terms(terms)
    hyper_row = np.ascontiguousarray(hyper_row, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    b = state_dim(terms, hyper_row)
    n = t.shape[0]
    sc = np.zeros(3)
    fm = np.zeros(n)
    fv = np.zeros(n)
    zm = np.zeros((n, b)) if want_blocks else None
    Sd = np.zeros((n, b, b)) if want_blocks else None
    Ss = np.zeros((max(n - 1, 0), b, b)) if want_blocks else None
    rc = lib.spo_btd_factored(len(terms), kinds.ctypes.data_as(_ip), harm.ctypes.data_as(_ip), _ptr(hyper_row),
                              n, _ptr(t), _ptr(y), _ptr(sc), _ptr(fm), _ptr(fv), _ptr(zm), _ptr(Sd),
                              _ptr(Ss) if (Ss is not None and Ss.size) else None)
    if rc:
        raise RuntimeError(f"spo_btd_factored failed ({rc})")
    out = {"logml": sc[0], "datafit": sc[1], "logdet": sc[2], "f_mean": fm, "f_var": fv}
    if want_blocks:
        out.update(z_mean=zm, S_diag=Sd, S_sub=Ss)
    return out


def tangent_grad(terms, hyper_row, t, y) -> dict:
    lib = load()
    kinds, harm = _terms(terms)
    hyper_row = np.ascontiguousarray(hyper_row, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    ll = np.zeros(1)
    g = np.zeros(hyper_row.shape[0])
    rc = lib.spo_tangent_grad(len(terms), kinds.ctypes.data_as(_ip), harm.ctypes.data_as(_ip), _ptr(hyper_row),
                              t.shape[0], _ptr(t), _ptr(y), _ptr(ll), _ptr(g))
    if rc:
        raise RuntimeError(f"spo_tangent_grad failed ({rc})")
    return {"logml": float(ll[0]), "grad": g}


def workload_reference(w, series=None, want_grad=True, want_blocks=False) -> list:
    """Oracle results for each series of a workload (or the listed series)."""
    idx = range(w.n_series) if series is None else series
    out = []
    for i in idx:
        t, y, hyp = w.series(i)
        r = btd_factored(w.terms, hyp, t, y, want_blocks=want_blocks)
        if want_grad:
            g = tangent_grad(w.terms, hyp, t, y)
            r["grad"] = g["grad"]
            r["logml_tangent"] = g["logml"]
        out.append(r)
    return out
