"""Exact 2D convex hulls on AMD Instinct MI355X (gfx950).

Python binding of ``libhull2d.so`` (C ABI in ``include/hull2d.h``).  This
module only marshals arguments: every step of the hull path runs in the
library's HIP kernels and its host stack scan.  PyTorch provides device
memory and the stream.  There is no fallback: if the library is missing the
functions raise.
"""
from __future__ import annotations

import atexit
import ctypes
import json
import os
import sys
import weakref
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhull2d.so")

STATUS = {
    0: "ok", 1: "invalid argument", 2: "non-finite coordinate",
    3: "coordinate magnitude outside [2^-300, 2^300]", 4: "output capacity too small",
    5: "out of memory", 6: "device error", 7: "weights missing or corrupt",
    8: "not implemented", 9: "input larger than HULL2D_NOALLOC_MAX_POINTS",
}
(OK, INVALID_ARG, NONFINITE, RANGE, CAPACITY, OUT_OF_MEMORY, DEVICE, WEIGHTS, UNIMPLEMENTED,
 TOO_LARGE) = range(10)
NOALLOC_MAX_POINTS = 262144  # HULL2D_NOALLOC_MAX_POINTS

STAGES = ["extremes", "extremes_final", "filter1", "longest", "histogram", "sort0", "sort1",
          "sort2", "sort3", "ties", "ties_long", "buckets", "round2", "compact", "tail",
          "learned", "d2h", "host_scan", "scan"]

EXPORTED = ["hull2d_create", "hull2d_compute", "hull2d_compute_noalloc", "hull2d_batch", "hull2d_destroy",
            "hull2d_status_string", "hull2d_set_weights", "hull2d_load_weights",
            "hull2d_get_weights", "hull2d_histogram", "hull2d_mlp_infer", "hull2d_train_step",
            "hull2d_debug_learned", "hull2d_debug_orient", "hull2d_debug_angle_key",
            "hull2d_debug_stages", "hull2d_debug_round1", "hull2d_debug_chain"]

MLP_PARAMS = 336416  # HULL2D_MLP_PARAMS


class HullError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        super().__init__(f"{where}: {STATUS.get(status, status)} (status {status})")
        self.status = status


class _Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("round2_chunk", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("full_sort", ctypes.c_int32),
                ("filter", ctypes.c_int32), ("batch_blocks_per_cu", ctypes.c_int32),
                ("batch_order", ctypes.c_int32), ("batch_graph", ctypes.c_int32),
                ("method", ctypes.c_int32), ("reserve_noalloc", ctypes.c_int32),
                ("scan", ctypes.c_int32), ("workspace_limit_mib", ctypes.c_int32),
                ("batch_engine", ctypes.c_int32), ("batch_tile", ctypes.c_int32),
                ("batch_filter_bits", ctypes.c_int32), ("batch_sort_bits", ctypes.c_int32),
                ("batch_side_sets", ctypes.c_int32), ("batch_items", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_round1", ctypes.c_int64),
                ("n_sorted", ctypes.c_int64), ("n_round2", ctypes.c_int64),
                ("n_hull", ctypes.c_int64), ("n_candidates", ctypes.c_int64),
                ("ms_total", ctypes.c_double),
                ("ms_device", ctypes.c_double),
                ("ms_stage", ctypes.c_double * len(STAGES))]


_lib = None

# Every open context, so that the ones still open when the interpreter exits
# are destroyed while the HIP runtime is still up (see _close_all).
_live: "weakref.WeakSet[Hull2D]" = weakref.WeakSet()
_atexit_registered = False


def _close_all():
    """Destroys every context still open.  Registered with atexit when the
    first context is created, which is after torch (and with it the HIP
    runtime) has been loaded, so it runs before their teardown: destroying a
    context synchronises its stream and frees device and pinned memory, which
    must not happen once the runtime has been finalised."""
    for ctx in list(_live):
        try:
            ctx.close()
        except Exception:
            pass
    _default.clear()


def load_library():
    """Load ``libhull2d.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1508_05931_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.hull2d_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.POINTER(_Options)]
    lib.hull2d_create.restype = ctypes.c_int
    lib.hull2d_compute.argtypes = [vp, vp, i64, ctypes.POINTER(i32), i64, ctypes.POINTER(i64),
                                   ctypes.POINTER(_Stats)]
    lib.hull2d_compute.restype = ctypes.c_int
    lib.hull2d_compute_noalloc.argtypes = lib.hull2d_compute.argtypes
    lib.hull2d_compute_noalloc.restype = ctypes.c_int
    lib.hull2d_batch.argtypes = [vp, vp, ctypes.POINTER(i64), i32, ctypes.POINTER(i32), i64,
                                 ctypes.POINTER(i64), ctypes.POINTER(_Stats)]
    lib.hull2d_batch.restype = ctypes.c_int
    lib.hull2d_destroy.argtypes = [vp]
    lib.hull2d_destroy.restype = None
    lib.hull2d_status_string.argtypes = [ctypes.c_int]
    lib.hull2d_status_string.restype = ctypes.c_char_p
    lib.hull2d_debug_orient.argtypes = [vp, vp, i64, vp]
    lib.hull2d_debug_orient.restype = ctypes.c_int
    lib.hull2d_debug_angle_key.argtypes = [vp, vp, i64, ctypes.c_double, ctypes.c_double, vp]
    lib.hull2d_debug_angle_key.restype = ctypes.c_int
    lib.hull2d_debug_stages.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                        ctypes.POINTER(i32), i64, ctypes.POINTER(i64)]
    lib.hull2d_debug_stages.restype = ctypes.c_int
    lib.hull2d_debug_round1.argtypes = [vp, ctypes.POINTER(i32), i64, ctypes.POINTER(i64)]
    lib.hull2d_debug_round1.restype = ctypes.c_int
    lib.hull2d_debug_chain.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), i64]
    lib.hull2d_debug_chain.restype = ctypes.c_int
    fp = ctypes.POINTER(ctypes.c_float)
    lib.hull2d_set_weights.argtypes = [vp, fp, i64]
    lib.hull2d_set_weights.restype = ctypes.c_int
    lib.hull2d_load_weights.argtypes = [vp, ctypes.c_char_p]
    lib.hull2d_load_weights.restype = ctypes.c_int
    lib.hull2d_get_weights.argtypes = [vp, fp, i64]
    lib.hull2d_get_weights.restype = ctypes.c_int
    lib.hull2d_histogram.argtypes = [vp, vp, i64, vp]
    lib.hull2d_histogram.restype = ctypes.c_int
    lib.hull2d_mlp_infer.argtypes = [vp, vp, i32, vp]
    lib.hull2d_mlp_infer.restype = ctypes.c_int
    lib.hull2d_train_step.argtypes = [vp, vp, vp, i32, ctypes.c_float, i32, fp, fp]
    lib.hull2d_train_step.restype = ctypes.c_int
    lib.hull2d_debug_learned.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int32), fp,
                                         ctypes.POINTER(ctypes.c_int32)]
    lib.hull2d_debug_learned.restype = ctypes.c_int
    _lib = lib
    return lib


@dataclass
class Stats:
    n: int = 0
    n_round1: int = 0
    n_sorted: int = 0
    n_round2: int = 0
    n_hull: int = 0
    n_candidates: int = 0
    ms_total: float = 0.0
    ms_device: float = 0.0
    ms_stage: dict = field(default_factory=dict)

    @staticmethod
    def _from(s: _Stats) -> "Stats":
        return Stats(s.n, s.n_round1, s.n_sorted, s.n_round2, s.n_hull, s.n_candidates,
                     s.ms_total, s.ms_device,
                     {k: float(s.ms_stage[i]) for i, k in enumerate(STAGES)})


def _i32p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


TUNING = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "batch.json")


# The schedule knobs autotune.py may store (each 0 = the library default).
TUNED_KEYS = ("batch_blocks_per_cu", "batch_order", "batch_tile", "batch_filter_bits",
              "batch_sort_bits", "batch_side_sets", "batch_items")


def tuned_batch_schedule() -> dict:
    """The batched form's schedule chosen by autotune.py (empty: none)."""
    try:
        with open(TUNING) as f:
            t = json.load(f)
        return {k: int(t[k]) for k in TUNED_KEYS if k in t}
    except (OSError, ValueError, KeyError, TypeError):
        return {}


class Hull2D:
    """A library context bound to one device and one HIP stream.

    profile: 0 (or False) no stage times; 1 (or True) every stage's device
    time in last_stats.ms_stage (one HIP event per stage); 2 only Step 1 and
    Steps 2-3 (two events per call).

    batch_graph: capture and replay the batched form's device work in a HIP
    graph.  batch_engine: 0 tiled (passes over points share a large set among
    many workgroups), 1 one persistent workgroup per set.  batch_blocks_per_cu
    / batch_order: the persistent engine's schedule; batch_tile /
    batch_filter_bits / batch_sort_bits / batch_side_sets / batch_items: the
    tiled engine's
    (hull2d_options documents each).  None takes the values autotune.py stored
    in tuning/batch.json, else the library's defaults."""

    def __init__(self, device: int | None = None, stream=None, round2_chunk: int = 0,
                 profile: int = 0, full_sort: bool = False, learned: bool = False,
                 weights=None, batch_graph: bool = True, batch_blocks_per_cu: int | None = None,
                 batch_order: int | None = None, reserve_noalloc: bool = False, method: int = 0,
                 scan: int = 0, workspace_limit_mib: int = 0, batch_engine: int = 0,
                 batch_tile: int | None = None, batch_filter_bits: int | None = None,
                 batch_sort_bits: int | None = None, batch_side_sets: int | None = None,
                 batch_items: int | None = None):
        import torch
        lib = load_library()
        if device is None:
            device = torch.cuda.current_device()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = int(device)
        self.stream = stream
        tuned = tuned_batch_schedule()
        given = {"batch_blocks_per_cu": batch_blocks_per_cu, "batch_order": batch_order,
                 "batch_tile": batch_tile, "batch_filter_bits": batch_filter_bits,
                 "batch_sort_bits": batch_sort_bits, "batch_side_sets": batch_side_sets,
                 "batch_items": batch_items}
        sched = {k: int(v) if v is not None else tuned.get(k, 0) for k, v in given.items()}
        opt = _Options(ctypes.sizeof(_Options), int(round2_chunk), int(profile),
                       int(bool(full_sort)), int(bool(learned)), sched["batch_blocks_per_cu"],
                       sched["batch_order"], int(bool(batch_graph)), int(method),
                       int(bool(reserve_noalloc)), int(scan), int(workspace_limit_mib),
                       int(batch_engine), sched["batch_tile"], sched["batch_filter_bits"],
                       sched["batch_sort_bits"], sched["batch_side_sets"], sched["batch_items"])
        h = ctypes.c_void_p()
        st = lib.hull2d_create(ctypes.byref(h), self.device, ctypes.c_void_p(stream.cuda_stream),
                               ctypes.byref(opt))
        if st != OK:
            raise HullError(st, "hull2d_create")
        self._h = h
        self._lib = lib
        global _atexit_registered
        _live.add(self)
        if not _atexit_registered:
            atexit.register(_close_all)
            _atexit_registered = True
        self.last_stats: Stats | None = None
        self._out = np.empty(1024, dtype=np.int32)
        if weights is not None:
            if isinstance(weights, (str, os.PathLike)):
                self.load_weights(weights)
            else:
                self.set_weights(weights)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.hull2d_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # During interpreter shutdown the HIP runtime may already be gone:
        # contexts open at exit are destroyed by the atexit hook, never here.
        # The check is bound as a default argument because module globals
        # (sys among them) can already be None when a late __del__ runs.
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def compute(self, xy) -> np.ndarray:
        """Canonical hull (int32 input indices) of a float64 [n, 2] device tensor."""
        import torch
        if not (isinstance(xy, torch.Tensor) and xy.is_cuda and xy.dtype == torch.float64):
            raise TypeError("xy must be a float64 CUDA tensor of shape [n, 2]")
        if xy.dim() != 2 or xy.shape[1] != 2 or not xy.is_contiguous():
            raise ValueError("xy must be a contiguous [n, 2] tensor")
        n = xy.shape[0]
        stats = _Stats()
        hn = ctypes.c_int64(0)
        for _ in range(2):
            st = self._lib.hull2d_compute(self._h, ctypes.c_void_p(xy.data_ptr() if n else 0), n,
                                          _i32p(self._out), self._out.shape[0], ctypes.byref(hn),
                                          ctypes.byref(stats))
            if st == CAPACITY:
                self._out = np.empty(max(int(hn.value), 2 * self._out.shape[0]), dtype=np.int32)
                continue
            break
        if st != OK:
            raise HullError(st, "hull2d_compute")
        self.last_stats = Stats._from(stats)
        return self._out[:hn.value].copy()

    def compute_noalloc(self, xy, out: np.ndarray) -> np.ndarray:
        """hull2d_compute_noalloc: the hull written into the caller's int32
        array `out` (no allocation inside the library call; the context must
        be created with reserve_noalloc=True).  Returns the filled prefix."""
        import torch
        if not (isinstance(xy, torch.Tensor) and xy.is_cuda and xy.dtype == torch.float64):
            raise TypeError("xy must be a float64 CUDA tensor of shape [n, 2]")
        if xy.dim() != 2 or xy.shape[1] != 2 or not xy.is_contiguous():
            raise ValueError("xy must be a contiguous [n, 2] tensor")
        if out.dtype != np.int32 or not out.flags["C_CONTIGUOUS"]:
            raise TypeError("out must be a contiguous int32 array")
        n = xy.shape[0]
        stats = _Stats()
        hn = ctypes.c_int64(0)
        st = self._lib.hull2d_compute_noalloc(self._h, ctypes.c_void_p(xy.data_ptr() if n else 0), n,
                                              _i32p(out), out.shape[0], ctypes.byref(hn),
                                              ctypes.byref(stats))
        if st != OK:
            raise HullError(st, "hull2d_compute_noalloc")
        self.last_stats = Stats._from(stats)
        return out[:hn.value]

    def batch(self, xy, offsets) -> "tuple[np.ndarray, np.ndarray]":
        """Hulls of the sets xy[offsets[s]:offsets[s+1]] of a float64 [N, 2]
        device tensor: (int32 set-local indices, int64 offsets [S+1])."""
        import torch
        if not (isinstance(xy, torch.Tensor) and xy.is_cuda and xy.dtype == torch.float64):
            raise TypeError("xy must be a float64 CUDA tensor of shape [N, 2]")
        if xy.dim() != 2 or xy.shape[1] != 2 or not xy.is_contiguous():
            raise ValueError("xy must be a contiguous [N, 2] tensor")
        offs = np.ascontiguousarray(offsets, dtype=np.int64)
        S = offs.shape[0] - 1
        if S < 0 or offs[-1] != xy.shape[0]:
            raise ValueError("offsets must have S+1 entries ending at N")
        out_offs = np.zeros(S + 1, dtype=np.int64)
        stats = _Stats()
        i64p = ctypes.POINTER(ctypes.c_int64)
        cap = max(getattr(self, "_bcap", 0), 1024)
        for _ in range(2):
            out = np.empty(cap, dtype=np.int32)
            st = self._lib.hull2d_batch(self._h, ctypes.c_void_p(xy.data_ptr() if xy.shape[0] else 0),
                                        offs.ctypes.data_as(i64p), S, _i32p(out), cap,
                                        out_offs.ctypes.data_as(i64p), ctypes.byref(stats))
            if st == CAPACITY:
                cap = int(out_offs[-1])
                self._bcap = cap
                continue
            break
        if st != OK:
            raise HullError(st, "hull2d_batch")
        self.last_stats = Stats._from(stats)
        return out[:out_offs[-1]].copy(), out_offs

    # ---- learned filter ------------------------------------------------
    def set_weights(self, params) -> None:
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        st = self._lib.hull2d_set_weights(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                          p.size)
        if st != OK:
            raise HullError(st, "hull2d_set_weights")

    def load_weights(self, path) -> None:
        st = self._lib.hull2d_load_weights(self._h, os.fsencode(os.fspath(path)))
        if st != OK:
            raise HullError(st, "hull2d_load_weights")

    def get_weights(self) -> np.ndarray:
        p = np.empty(MLP_PARAMS, dtype=np.float32)
        st = self._lib.hull2d_get_weights(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                          p.size)
        if st != OK:
            raise HullError(st, "hull2d_get_weights")
        return p

    def histogram(self, xy):
        """The network input of a float64 [n, 2] CUDA tensor (float32 [1024] tensor)."""
        import torch
        out = torch.empty(1024, dtype=torch.float32, device=xy.device)
        st = self._lib.hull2d_histogram(self._h, ctypes.c_void_p(xy.data_ptr() if xy.shape[0] else 0),
                                        xy.shape[0], ctypes.c_void_p(out.data_ptr()))
        if st != OK:
            raise HullError(st, "hull2d_histogram")
        return out

    def mlp_infer(self, x):
        """Network outputs [rows, 32] of a float32 [rows, 1024] CUDA tensor."""
        import torch
        x = x.contiguous()
        y = torch.empty((x.shape[0], 32), dtype=torch.float32, device=x.device)
        st = self._lib.hull2d_mlp_infer(self._h, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                        ctypes.c_void_p(y.data_ptr()))
        if st != OK:
            raise HullError(st, "hull2d_mlp_infer")
        return y

    def train_step(self, x, t, lr: float = 1e-3, apply: bool = True, want_grad: bool = False):
        """One step on float32 CUDA tensors x [B, 1024], t [B, 32]: (loss, grad or None)."""
        x = x.contiguous()
        t = t.contiguous()
        loss = ctypes.c_float(0.0)
        g = np.empty(MLP_PARAMS, dtype=np.float32) if want_grad else None
        st = self._lib.hull2d_train_step(
            self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()), x.shape[0],
            float(lr), int(bool(apply)), ctypes.byref(loss),
            g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if g is not None else None)
        if st != OK:
            raise HullError(st, "hull2d_train_step")
        return float(loss.value), g

    def learned_info(self) -> dict:
        """Directions, candidates, raw outputs and polygon size of the last
        learned-filter call."""
        d = np.empty(32, dtype=np.float64)
        c = np.empty(20, dtype=np.int32)
        y = np.empty(32, dtype=np.float32)
        nv = ctypes.c_int32(0)
        st = self._lib.hull2d_debug_learned(self._h, d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            y.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                            ctypes.byref(nv))
        if st != OK:
            raise HullError(st, "hull2d_debug_learned")
        return {"dirs": d.reshape(16, 2), "cand": c, "y": y, "nv": int(nv.value)}

    def stages(self, cap: int) -> dict:
        """Stage results of the last compute (for checking against the model)."""
        ext = np.zeros(4, dtype=np.int32)
        srt = np.zeros(max(cap, 1), dtype=np.int32)
        r2 = np.zeros(max(cap, 1), dtype=np.int32)
        counts = np.zeros(6, dtype=np.int64)
        st = self._lib.hull2d_debug_stages(self._h, _i32p(ext), _i32p(srt), _i32p(r2), cap,
                                           counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        if st != OK:
            raise HullError(st, "hull2d_debug_stages")
        ns, l, m2, longest, have_sorted, ncand = (int(v) for v in counts)
        return {"extremes": ext.tolist(), "sorted": srt[:ns].copy() if have_sorted else None,
                "l": l, "round2": r2[:m2].copy(), "longest": longest, "m2": m2,
                "n_sorted": ns, "n_candidates": ncand}

    def round1_survivors(self) -> np.ndarray:
        """Input indices (ascending) of the last compute's round-1 survivors,
        copies of the pivot excluded."""
        cap = max(int(self.last_stats.n) if self.last_stats else 0, 1)
        out = np.empty(cap, dtype=np.int32)
        n = ctypes.c_int64(0)
        st = self._lib.hull2d_debug_round1(self._h, _i32p(out), cap, ctypes.byref(n))
        if st != OK:
            raise HullError(st, "hull2d_debug_round1")
        return out[:n.value].copy()

    def chain_info(self) -> dict:
        """Counts and kept lists of the last compute with method=1 (the
        four-region variant)."""
        counts = np.zeros(14, dtype=np.int64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        st = self._lib.hull2d_debug_chain(self._h, counts.ctypes.data_as(i64p), None, 0)
        if st != OK:
            raise HullError(st, "hull2d_debug_chain")
        nk = [int(v) for v in counts[9:13]]
        kept = np.zeros(max(sum(nk), 1), dtype=np.int32)
        st = self._lib.hull2d_debug_chain(self._h, None, _i32p(kept), kept.shape[0])
        if st != OK:
            raise HullError(st, "hull2d_debug_chain")
        offs = np.cumsum([0] + nk)
        return {"m1": int(counts[0]), "n_region": [int(v) for v in counts[1:5]],
                "n_cand": [int(v) for v in counts[5:9]], "n_kept": nk, "m2": int(counts[13]),
                "kept": [kept[offs[k]:offs[k + 1]].copy() for k in range(4)]}

    def debug_orient(self, abc) -> "np.ndarray":
        import torch
        abc = abc.contiguous()
        out = torch.empty(abc.shape[0], dtype=torch.int32, device=abc.device)
        st = self._lib.hull2d_debug_orient(self._h, ctypes.c_void_p(abc.data_ptr()),
                                           abc.shape[0], ctypes.c_void_p(out.data_ptr()))
        if st != OK:
            raise HullError(st, "hull2d_debug_orient")
        return out.cpu().numpy()

    def debug_angle_key(self, xy, x0: float, y0: float) -> "np.ndarray":
        import torch
        xy = xy.contiguous()
        out = torch.empty(xy.shape[0], dtype=torch.int32, device=xy.device)
        st = self._lib.hull2d_debug_angle_key(self._h, ctypes.c_void_p(xy.data_ptr()),
                                              xy.shape[0], float(x0), float(y0),
                                              ctypes.c_void_p(out.data_ptr()))
        if st != OK:
            raise HullError(st, "hull2d_debug_angle_key")
        return out.cpu().numpy().view(np.uint32)


_default: dict = {}


def compute(xy) -> np.ndarray:
    """Hull of a float64 [n, 2] CUDA tensor on the current device and stream."""
    import torch
    dev = xy.device.index if xy.device.index is not None else torch.cuda.current_device()
    stream = torch.cuda.current_stream(dev)
    key = (dev, stream.cuda_stream)
    ctx = _default.get(key)
    if ctx is None:
        ctx = Hull2D(dev, stream)
        _default[key] = ctx
    return ctx.compute(xy)
