"""The no-allocation entry point, hull2d_compute_noalloc, through the C ABI:
its hulls equal hull2d_compute's (and the oracle's) bit for bit, on calls in
a row with shrinking inputs, from two contexts sharing the device's fixed
workspace, on the tail and the multi-kernel paths; inputs above the limit and
contexts created without the reservation are refused."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    return torch


@pytest.fixture(scope="module")
def hx(torch_dev):
    import paper_1508_05931_amd as hx
    return hx


def _noalloc(hx, ctx, d, cap):
    """One hull2d_compute_noalloc call: (status, hull indices)."""
    lib = hx.load_library()
    out = np.full(max(cap, 1), -7, dtype=np.int32)
    n_out = ctypes.c_int64(-1)
    st = lib.hull2d_compute_noalloc(ctx._h, ctypes.c_void_p(d.data_ptr() if d.shape[0] else 0),
                                    d.shape[0], out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    cap, ctypes.byref(n_out), None)
    return st, out[:max(n_out.value, 0)].copy()


def _cases():
    t = np.arange(10_000, dtype=np.float64)
    return [
        ("square_max", synth.square(262_144, (90, 1))),
        ("disk_100k", synth.disk(100_000, (91, 1))),
        ("collinear_10k", np.stack([t, 0.5 * t + 3.0], 1)[np.random.default_rng(5).permutation(10_000)]),
        ("annulus_262k", synth.annulus(262_144, 0.99999, (92, 1))),
        ("grid_draws_200k", synth.grid_draws(200_000, 64, (93, 1))),
        ("three", np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])),
    ]


def test_noalloc_equals_compute(torch_dev, hx):
    ref = hx.Hull2D()
    a = hx.Hull2D(reserve_noalloc=True)
    b = hx.Hull2D(reserve_noalloc=True)
    for k, (name, pts) in enumerate(_cases()):
        say(f"noalloc {name} n={len(pts)}")
        d = torch_dev.from_numpy(np.ascontiguousarray(pts)).cuda()
        want = ref.compute(d)
        assert want.tolist() == oracle.hull(pts).tolist()
        ctx = a if k % 2 == 0 else b
        st, got = _noalloc(hx, ctx, d, len(want) + 3)
        assert st == hx.OK, st
        assert got.tolist() == want.tolist()
        # the other context right after, then this one again: the shared
        # workspace keeps no state that changes a result
        other = b if ctx is a else a
        st, got2 = _noalloc(hx, other, d, len(want))
        assert st == hx.OK and got2.tolist() == want.tolist()
    for c in (ref, a, b):
        c.close()


def test_noalloc_two_calls_second_smaller(torch_dev, hx):
    ref = hx.Hull2D()
    c = hx.Hull2D(reserve_noalloc=True)
    big = synth.disk(250_000, (94, 1))
    small = synth.square(1_000, (95, 1))
    for pts in (big, small):
        d = torch_dev.from_numpy(pts).cuda()
        want = ref.compute(d)
        st, got = _noalloc(hx, c, d, 4096)
        assert st == hx.OK
        assert got.tolist() == want.tolist()
    ref.close()
    c.close()


def test_noalloc_limits_and_errors(torch_dev, hx):
    c = hx.Hull2D(reserve_noalloc=True)
    over = torch_dev.from_numpy(synth.square(hx.NOALLOC_MAX_POINTS + 1, (96, 1))).cuda()
    st, _ = _noalloc(hx, c, over, 64)
    assert st == hx.TOO_LARGE
    plain = hx.Hull2D()
    ok = torch_dev.from_numpy(synth.square(5_000, (97, 1))).cuda()
    st, _ = _noalloc(hx, plain, ok, 64)
    assert st == hx.INVALID_ARG
    # capacity: the required size comes back, the output is untouched
    want = oracle.hull(synth.square(5_000, (97, 1)))
    lib = hx.load_library()
    out = np.full(2, -7, dtype=np.int32)
    n_out = ctypes.c_int64(0)
    st = lib.hull2d_compute_noalloc(c._h, ctypes.c_void_p(ok.data_ptr()), ok.shape[0],
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 2,
                                    ctypes.byref(n_out), None)
    assert st == hx.CAPACITY and n_out.value == len(want) and (out == -7).all()
    st, got = _noalloc(hx, c, ok, len(want))
    assert st == hx.OK and got.tolist() == want.tolist()
    # empty input
    st, got = _noalloc(hx, c, torch_dev.zeros((0, 2), dtype=torch_dev.float64, device="cuda"), 0)
    assert st == hx.OK and len(got) == 0
    plain.close()
    c.close()
