"""CPU oracle for the inclusion-based CCD root finder (test infrastructure).

This package is the plain, slow, single-threaded reference implementation of
Algorithm 2 of Wang et al. 2021 (with the minimum-separation variant of its
Sec. 6) that the GPU library is checked against, plus an exact-rational checker
(`oracle.exact`).  Only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark may import it; the product library never does.  It shares no
source with the HIP library.

`build()` compiles ``ccd_oracle.cpp`` into ``liboracle.so`` with
``-ffp-contract=off`` so that every floating-point operation is a single
correctly rounded binary64 operation in the written order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ccd_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

VF, EE = 0, 1
ST_CAP, ST_CARRY, ST_DEPTH = 1, 2, 4


def build(force: bool = True) -> str:
    """Compile the oracle shared library in place; returns its path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class OracleResult(ctypes.Structure):
    _fields_ = [
        ("toi", ctypes.c_double),
        ("t_width", ctypes.c_double),
        ("n_checks", ctypes.c_uint64),
        ("n_raw", ctypes.c_uint64),
        ("hit", ctypes.c_uint8),
        ("status", ctypes.c_uint8),
        ("pad", ctypes.c_uint8 * 6),
        ("box", ctypes.c_double * 6),
        ("level", ctypes.c_int32),
        ("depth", ctypes.c_int32 * 3),
    ]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.oracle_F.argtypes = [ctypes.c_int, _D, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, _D]
        L.oracle_F.restype = ctypes.c_int
        L.oracle_filter.argtypes = [ctypes.c_int, _D, ctypes.c_double, _D]
        L.oracle_filter.restype = None
        L.oracle_kappa.argtypes = [ctypes.c_int, _D, _D]
        L.oracle_kappa.restype = None
        L.oracle_split_axis.argtypes = [_D, _D]
        L.oracle_split_axis.restype = ctypes.c_int
        L.oracle_box_check.argtypes = [ctypes.c_int, _D, _D, _D, ctypes.c_double,
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                       _D, _D, _D]
        L.oracle_box_check.restype = None
        L.oracle_validate.argtypes = [_D, ctypes.c_double, ctypes.c_int64, ctypes.c_double]
        L.oracle_validate.restype = ctypes.c_int
        L.oracle_solve.argtypes = [ctypes.c_int, _D, ctypes.c_double, ctypes.c_int64,
                                   ctypes.c_double, ctypes.c_int, ctypes.POINTER(OracleResult)]
        L.oracle_solve.restype = ctypes.c_int
        L.oracle_solve_tmax.argtypes = [ctypes.c_int, _D, ctypes.c_double, ctypes.c_int64,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                        ctypes.POINTER(OracleResult)]
        L.oracle_solve_tmax.restype = ctypes.c_int
        L.oracle_solve_full.argtypes = [ctypes.c_int, _D, ctypes.c_double, ctypes.c_int64,
                                        ctypes.c_double, ctypes.c_double, _D, ctypes.c_int,
                                        ctypes.POINTER(OracleResult)]
        L.oracle_solve_full.restype = ctypes.c_int
        L.oracle_filter_gamma.argtypes = [ctypes.c_int, _D, ctypes.c_double, _D]
        L.oracle_filter_gamma.restype = None
        L.oracle_solve_batch.argtypes = [
            ctypes.c_int64, _D, ctypes.POINTER(ctypes.c_uint8), ctypes.c_int,
            _D, ctypes.c_double, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
            _D, ctypes.c_double, ctypes.c_double, _D, ctypes.c_int,
            _D, _D, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_uint64),
            ctypes.POINTER(ctypes.c_uint8)]
        L.oracle_solve_batch.restype = ctypes.c_int64
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _as_x(X) -> np.ndarray:
    """Query as 24 doubles: X[3k+c], points 0..3 at t0 then the same 4 at t1."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64).reshape(24))
    return X


def F(kind: int, X, t: float, u: float, v: float) -> np.ndarray:
    X = _as_x(X)
    out = np.zeros(3)
    lib().oracle_F(kind, _dptr(X), t, u, v, _dptr(out))
    return out


def filter_eps_gamma(kind: int, gamma, min_sep: float = 0.0) -> np.ndarray:
    """eq. ccd-error / msccd-error for a given gamma per axis."""
    g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64))
    eps = np.empty(3)
    lib().oracle_filter_gamma(kind, _dptr(g), float(min_sep), _dptr(eps))
    return eps


def filter_eps(kind: int, X, min_sep: float = 0.0) -> np.ndarray:
    X = _as_x(X)
    out = np.zeros(3)
    lib().oracle_filter(kind, _dptr(X), min_sep, _dptr(out))
    return out


def kappa(kind: int, X) -> np.ndarray:
    X = _as_x(X)
    out = np.zeros(3)
    lib().oracle_kappa(kind, _dptr(X), _dptr(out))
    return out


def split_axis(kap, widths) -> int:
    k = np.ascontiguousarray(np.asarray(kap, dtype=np.float64))
    w = np.ascontiguousarray(np.asarray(widths, dtype=np.float64))
    return lib().oracle_split_axis(_dptr(k), _dptr(w))


def box_check(kind: int, X, box, eps, min_sep: float = 0.0):
    """Returns (collide, inside, width, lo[3], hi[3]) for box (t0,t1,u0,u1,v0,v1)."""
    X = _as_x(X)
    b = np.ascontiguousarray(np.asarray(box, dtype=np.float64))
    e = np.ascontiguousarray(np.asarray(eps, dtype=np.float64))
    col, ins = ctypes.c_int(), ctypes.c_int()
    w = np.zeros(1)
    lo, hi = np.zeros(3), np.zeros(3)
    lib().oracle_box_check(kind, _dptr(X), _dptr(b), _dptr(e), min_sep, ctypes.byref(col),
                           ctypes.byref(ins), _dptr(w), _dptr(lo), _dptr(hi))
    return bool(col.value), bool(ins.value), float(w[0]), lo, hi


def validate(X, delta: float, max_iter: int, min_sep: float = 0.0) -> bool:
    X = _as_x(X)
    return lib().oracle_validate(_dptr(X), delta, max_iter, min_sep) == 0


def solve(kind: int, X, delta: float = 1e-6, max_iter: int = 1_000_000, min_sep: float = 0.0,
          literal: bool = False, t_max: float = 1.0, gamma=None) -> OracleResult:
    """Algorithm 2 on one query over I = [0, t_max] x [0,1]^2; raises ValueError on
    invalid input.  gamma: scene-wide gamma per axis (3 values) or None.  The
    result's box keeps the time axis normalized (t / t_max)."""
    X = _as_x(X)
    r = OracleResult()
    g = None if gamma is None else np.ascontiguousarray(np.asarray(gamma, dtype=np.float64))
    rc = lib().oracle_solve_full(kind, _dptr(X), delta, int(max_iter), min_sep, float(t_max),
                                 None if g is None else _dptr(g), int(literal), ctypes.byref(r))
    if rc != 0:
        raise ValueError("invalid CCD query")
    return r


def solve_batch(pos: np.ndarray, kind=None, default_kind: int = 0, delta=1e-6,
                max_iter=1_000_000, min_sep=0.0, literal: bool = False, t_max: float = 1.0,
                gamma=None):
    """Batch over SoA positions pos[24, n]. delta/max_iter/min_sep may be scalars
    or per-query arrays. Returns a dict of numpy arrays."""
    pos = np.ascontiguousarray(np.asarray(pos, dtype=np.float64))
    assert pos.ndim == 2 and pos.shape[0] == 24
    n = pos.shape[1]
    kind_a = None if kind is None else np.ascontiguousarray(np.asarray(kind, dtype=np.uint8))

    def _arr(v, dt):
        if np.ndim(v) == 0:
            return None, v
        return np.ascontiguousarray(np.asarray(v, dtype=dt)), 0

    dq, ds = _arr(delta, np.float64)
    mq, ms_ = _arr(max_iter, np.int64)
    sq, ss = _arr(min_sep, np.float64)
    g = None if gamma is None else np.ascontiguousarray(np.asarray(gamma, dtype=np.float64))
    toi = np.empty(n)
    tw = np.empty(n)
    hit = np.empty(n, np.uint8)
    nc = np.empty(n, np.uint64)
    st = np.empty(n, np.uint8)
    u8 = ctypes.POINTER(ctypes.c_uint8)
    bad = lib().oracle_solve_batch(
        n, _dptr(pos), None if kind_a is None else kind_a.ctypes.data_as(u8), default_kind,
        None if dq is None else _dptr(dq), float(ds),
        None if mq is None else mq.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(ms_),
        None if sq is None else _dptr(sq), float(ss), float(t_max),
        None if g is None else _dptr(g), int(literal),
        _dptr(toi), _dptr(tw), hit.ctypes.data_as(u8),
        nc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), st.ctypes.data_as(u8))
    return {"toi": toi, "t_width": tw, "hit": hit, "n_checks": nc, "status": st,
            "invalid": int(bad)}
