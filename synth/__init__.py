"""Seeded synthetic point sets for the exact 2D hull workloads.

This package holds only random-number draws and point placement (see
``synth.h``); it contains none of the hull method's arithmetic.  The CPU
oracle tests and the GPU path read their inputs from here, so both sides see
the same bytes.

Named workloads mirror the paper's test groups (Section 4: uniform points in
a square and in a circle, read as the unit disk) at its sizes, plus the
adversarial, batched and mixture workloads used to stress the exact
predicates:

=====================  =====================================================
``square_100k``        100,000 points uniform in [0,1)^2, seed (1, 1)
``square_20M``         20,000,000 points uniform in [0,1)^2, seed (2, 1)
``disk_20M``           20,000,000 points uniform in the unit disk, seed (3, 1)
``annulus_ngon_20M``   10M annulus r in [0.999, 1] (seed 4) + 10M vertices of
                       a 2^20-gon with repetition (seed 5), shuffled (seed 6)
``grid_500x4``         500x500 integer grid, each cell 4 times, shuffled
                       (seed 7): 1,000,000 points
``mixture_20M``        20,000,000 points from 1-8 anisotropic Gaussians (seed 9)
=====================  =====================================================
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``libsynth.so`` with gcc (no contraction, so the bytes are stable)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
            "-o", tmp, os.path.join(_HERE, "synth.c"), "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        i64, u64, c_int = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
        for name, args in {
            "synth_square": [dp, i64, u64, u64],
            "synth_disk": [dp, i64, u64, u64],
            "synth_annulus": [dp, i64, ctypes.c_double, u64, u64],
            "synth_gaussian": [dp, i64, ctypes.c_double, u64, u64],
            "synth_ngon": [dp, i64, c_int, u64, u64],
            "synth_shuffle": [dp, i64, u64, u64],
            "synth_grid": [dp, c_int, c_int, u64, u64],
            "synth_grid_draws": [dp, i64, c_int, u64, u64],
            "synth_mixture": [dp, i64, u64, u64],
            "synth_batch_sizes": [ctypes.POINTER(ctypes.c_int64), c_int,
                                  ctypes.c_double, ctypes.c_double, u64],
            "synth_batch_set": [dp, i64, u64, c_int],
        }.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = c_int
        lib.synth_hash.argtypes = [dp, i64]
        lib.synth_hash.restype = u64
        _lib = lib
    return _lib


def _buf(n: int) -> np.ndarray:
    return np.empty((int(n), 2), dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int) -> None:
    if rc < 0:
        raise ValueError("synth: bad argument")


def square(n: int, seed=(1, 1)) -> np.ndarray:
    a = _buf(n)
    _check(_load().synth_square(_ptr(a), n, seed[0], seed[1]))
    return a


def disk(n: int, seed=(3, 1)) -> np.ndarray:
    a = _buf(n)
    _check(_load().synth_disk(_ptr(a), n, seed[0], seed[1]))
    return a


def annulus(n: int, r_in: float = 0.999, seed=(4, 1)) -> np.ndarray:
    a = _buf(n)
    _check(_load().synth_annulus(_ptr(a), n, r_in, seed[0], seed[1]))
    return a


def gaussian(n: int, sigma: float = 1.0, seed=(10, 1)) -> np.ndarray:
    a = _buf(n)
    _check(_load().synth_gaussian(_ptr(a), n, sigma, seed[0], seed[1]))
    return a


def ngon(n: int, log2k: int, seed=(5, 1)) -> np.ndarray:
    a = _buf(n)
    _check(_load().synth_ngon(_ptr(a), n, log2k, seed[0], seed[1]))
    return a


def shuffle(a: np.ndarray, seed=(6, 1)) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    _check(_load().synth_shuffle(_ptr(a), a.shape[0], seed[0], seed[1]))
    return a


def grid(side: int, copies: int, seed=(7, 1)) -> np.ndarray:
    a = _buf(side * side * copies)
    _check(_load().synth_grid(_ptr(a), side, copies, seed[0], seed[1]))
    return a


def grid_draws(n: int, side: int, seed=(7, 2)) -> np.ndarray:
    a = _buf(n)
    _check(_load().synth_grid_draws(_ptr(a), n, side, seed[0], seed[1]))
    return a


def mixture(n: int, seed=(9, 1)) -> np.ndarray:
    a = _buf(n)
    _check(_load().synth_mixture(_ptr(a), n, seed[0], seed[1]))
    return a


def annulus_ngon(n_annulus: int, n_ngon: int, log2k: int = 20,
                 seeds=((4, 1), (5, 1), (6, 1))) -> np.ndarray:
    """Annulus points plus n-gon vertices with repetition, shuffled together."""
    a = np.concatenate([annulus(n_annulus, 0.999, seeds[0]),
                        ngon(n_ngon, log2k, seeds[1])])
    return shuffle(a, seeds[2])


def batch_sizes(S: int = 4096, lo: float = 64.0, hi: float = 200000.0,
                seed: int = 8) -> np.ndarray:
    s = np.empty(S, dtype=np.int64)
    _check(_load().synth_batch_sizes(
        s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), S, lo, hi, seed))
    return s


def batch_set(n: int, set_id: int, seed: int = 8):
    """Returns (points, kind) with kind 0 square, 1 disk, 2 Gaussian, 3 annulus."""
    a = _buf(n)
    kind = _load().synth_batch_set(_ptr(a), n, seed, set_id)
    _check(kind)
    return a, kind


def batch(S: int = 4096, lo: float = 64.0, hi: float = 200000.0, seed: int = 8):
    """Concatenated batch: (points [sum N, 2], offsets int64 [S+1], kinds)."""
    sizes = batch_sizes(S, lo, hi, seed)
    offs = np.zeros(S + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    pts = np.empty((int(offs[-1]), 2), dtype=np.float64)
    kinds = np.empty(S, dtype=np.int32)
    lib = _load()
    for s in range(S):
        view = pts[offs[s]:offs[s + 1]]
        k = lib.synth_batch_set(_ptr(view), int(sizes[s]), seed, s)
        _check(k)
        kinds[s] = k
    return pts, offs, kinds


def content_hash(a: np.ndarray) -> int:
    a = np.ascontiguousarray(a, dtype=np.float64)
    return int(_load().synth_hash(_ptr(a), a.shape[0]))


WORKLOADS = {
    "square_100k": lambda: square(100_000, (1, 1)),
    "square_20M": lambda: square(20_000_000, (2, 1)),
    "disk_20M": lambda: disk(20_000_000, (3, 1)),
    "annulus_ngon_20M": lambda: annulus_ngon(10_000_000, 10_000_000, 20),
    "grid_500x4": lambda: grid(500, 4, (7, 1)),
    "mixture_20M": lambda: mixture(20_000_000, (9, 1)),
}


def workload(name: str) -> np.ndarray:
    """The named workload's points as float64 [n, 2] (see the module docstring)."""
    return WORKLOADS[name]()
