"""CPU oracle for the exact 2D convex hull and the gScan method model.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the product path never does.  It shares
no code with the GPU library (see ``oracle.h`` for what each function
computes and which passage of the paper it follows).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, NONFINITE, RANGE, BADARG, NOMEM, CAPACITY = range(6)


class OracleError(RuntimeError):
    def __init__(self, status: int):
        super().__init__(f"oracle status {status}")
        self.status = status


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc, contraction off."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
            "-o", tmp, os.path.join(_HERE, "oracle.c"), "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _ModelResult(ctypes.Structure):
    _fields_ = [
        ("extremes", ctypes.c_int32 * 4),
        ("n_corners", ctypes.c_int32),
        ("m1", ctypes.c_int64),
        ("round1_keep", ctypes.POINTER(ctypes.c_uint8)),
        ("pivot", ctypes.c_int32),
        ("n_sorted", ctypes.c_int64),
        ("sorted", ctypes.POINTER(ctypes.c_int32)),
        ("longest", ctypes.c_int32),
        ("l", ctypes.c_int64),
        ("m2", ctypes.c_int64),
        ("round2", ctypes.POINTER(ctypes.c_int32)),
        ("h", ctypes.c_int64),
        ("hull", ctypes.POINTER(ctypes.c_int32)),
    ]


class _ChainResult(ctypes.Structure):
    _fields_ = [
        ("extremes", ctypes.c_int32 * 4),
        ("m1", ctypes.c_int64),
        ("region", ctypes.POINTER(ctypes.c_int8)),
        ("n_region", ctypes.c_int64 * 4),
        ("n_kept", ctypes.c_int64 * 4),
        ("kept", ctypes.POINTER(ctypes.c_int32)),
        ("m2", ctypes.c_int64),
        ("h", ctypes.c_int64),
        ("hull", ctypes.POINTER(ctypes.c_int32)),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        d = ctypes.c_double
        lib.oracle_orient.argtypes = [d, d, d, d, d, d]
        lib.oracle_orient.restype = ctypes.c_int
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_validate.argtypes = [dp, ctypes.c_int64]
        lib.oracle_validate.restype = ctypes.c_int
        lib.oracle_hull.argtypes = [dp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_hull.restype = ctypes.c_int
        lib.oracle_model.argtypes = [dp, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.POINTER(_ModelResult)]
        lib.oracle_model.restype = ctypes.c_int
        lib.oracle_learned_round1.argtypes = [dp, ctypes.c_int64, dp, ctypes.c_int32,
                                              ctypes.POINTER(ctypes.c_uint8),
                                              ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_learned_round1.restype = ctypes.c_int
        lib.oracle_round2.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_uint8)]
        lib.oracle_round2.restype = ctypes.c_int
        lib.oracle_chain.argtypes = [dp, ctypes.c_int64, ctypes.POINTER(_ChainResult)]
        lib.oracle_chain.restype = ctypes.c_int
        _lib = lib
    return _lib


def _points(xy) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(xy, dtype=np.float64).reshape(-1, 2))
    return a


def orient(a, b, c) -> int:
    """Exact sign of (b - a) x (c - a)."""
    return int(_load().oracle_orient(float(a[0]), float(a[1]), float(b[0]),
                                     float(b[1]), float(c[0]), float(c[1])))


def validate(xy) -> int:
    a = _points(xy)
    return int(_load().oracle_validate(
        a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), a.shape[0]))


def hull(xy) -> np.ndarray:
    """Canonical hull indices (int32): CCW from the lexicographic minimum,
    collinear points and duplicates dropped, smallest index per vertex."""
    a = _points(xy)
    n = a.shape[0]
    out = np.empty(max(n, 1), dtype=np.int32)
    h = ctypes.c_int64(0)
    st = _load().oracle_hull(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n,
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             out.shape[0], ctypes.byref(h))
    if st != OK:
        raise OracleError(st)
    return out[:h.value].copy()


def round2(q, l: int, chunk: int = 0) -> np.ndarray:
    """Step 7 alone on points already in angular order (q[0] = P_0,
    q[l] = P_longest); returns the keep mask."""
    a = _points(q)
    keep = np.zeros(max(a.shape[0], 1), dtype=np.uint8)
    st = _load().oracle_round2(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               a.shape[0], int(l), int(chunk),
                               keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if st != OK:
        raise OracleError(st)
    return keep[:a.shape[0]].astype(bool)


def model(xy, chunk: int = 0) -> dict:
    """Every stage of the method model (Steps 1-8).  ``chunk``: 0 = one walk
    per region, -1 = 1024 subsets per region, c > 0 = subsets of c points."""
    a = _points(xy)
    n = a.shape[0]
    m = max(n, 1)
    keep1 = np.zeros(m, dtype=np.uint8)
    srt = np.empty(m, dtype=np.int32)
    r2 = np.empty(m, dtype=np.int32)
    hl = np.empty(m, dtype=np.int32)
    r = _ModelResult()
    r.round1_keep = keep1.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    r.sorted = srt.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    r.round2 = r2.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    r.hull = hl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    st = _load().oracle_model(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n,
                              int(chunk), ctypes.byref(r))
    if st != OK:
        raise OracleError(st)
    return {
        "extremes": list(r.extremes),
        "n_corners": int(r.n_corners),
        "m1": int(r.m1),
        "round1_keep": keep1[:n].astype(bool),
        "pivot": int(r.pivot),
        "sorted": srt[:r.n_sorted].copy(),
        "longest": int(r.longest),
        "l": int(r.l),
        "m2": int(r.m2),
        "round2": r2[:r.m2].copy(),
        "hull": hl[:r.h].copy(),
    }


def learned_round1(xy, dirs) -> dict:
    """First round with the learned discard polygon (see oracle.h): the
    survivors (bool [n]), the candidate indices (the four Step-1 extremes, then
    one per direction) and the survivor count."""
    a = _points(xy)
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 2)
    n, k = a.shape[0], d.shape[0]
    keep = np.zeros(max(n, 1), dtype=np.uint8)
    cand = np.zeros(k + 4, dtype=np.int32)
    m1 = ctypes.c_int64(0)
    dp = ctypes.POINTER(ctypes.c_double)
    st = _load().oracle_learned_round1(a.ctypes.data_as(dp), n, d.ctypes.data_as(dp), k,
                                       keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                       cand.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       ctypes.byref(m1))
    if st != OK:
        raise OracleError(st)
    return {"keep": keep[:n].astype(bool), "cand": cand, "m1": int(m1.value)}


def chain(xy) -> dict:
    """The four-region variant (see oracle.h): extremes, the region of every
    point (-1 discarded by round 1, 4 on the quadrilateral's boundary), the
    kept points per region in walking order, and the canonical hull."""
    a = _points(xy)
    n = a.shape[0]
    m = max(n, 1)
    reg = np.zeros(m, dtype=np.int8)
    kept = np.zeros(m, dtype=np.int32)
    hl = np.zeros(m, dtype=np.int32)
    r = _ChainResult()
    r.region = reg.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
    r.kept = kept.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    r.hull = hl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    st = _load().oracle_chain(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n, ctypes.byref(r))
    if st != OK:
        raise OracleError(st)
    nk = list(r.n_kept)
    offs = np.cumsum([0] + nk)
    return {
        "extremes": list(r.extremes),
        "m1": int(r.m1),
        "region": reg[:n].copy(),
        "n_region": list(r.n_region),
        "kept": [kept[offs[k]:offs[k + 1]].copy() for k in range(4)],
        "m2": int(r.m2),
        "hull": hl[:r.h].copy(),
    }
