"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

* device predicates (orientation, angle key) against exact rationals;
* every stage (extremes, sorted order, split, round-2 survivors) against the
  oracle's step-by-step model, for the single-walk and subset modes;
* the canonical hull against the monotone-chain oracle, bit for bit, on the
  small configuration, ragged sizes, degenerate and duplicate-heavy inputs;
* the full-size workloads against oracle-written golden hashes.
"""
import hashlib
import json
import math
import os
import random
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.exact_ref import orient_q

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden", "hulls.json")


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


@pytest.fixture(scope="module")
def ctx(hx):
    return hx.Hull2D()


def to_dev(torch, pts):
    return torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float64)).cuda()


def _walk(v, k):
    for _ in range(abs(k)):
        v = math.nextafter(v, math.inf if k > 0 else -math.inf)
    return v


# ---------------------------------------------------------------- predicates
def test_device_orient_vs_exact(torch_dev, ctx):
    rng = random.Random(41)
    rows = []
    for _ in range(20000):
        ax, ay, bx, by = (rng.uniform(-1, 1) for _ in range(4))
        t = rng.uniform(-2, 3)
        rows.append((ax, ay, bx, by, _walk(ax + t * (bx - ax), rng.randint(-3, 3)),
                     _walk(ay + t * (by - ay), rng.randint(-3, 3))))
    for _ in range(3000):
        s = math.ldexp(1.0, rng.choice([-300, -100, 100, 299]))
        a = (rng.uniform(1, 2) * s, rng.uniform(1, 2) * s)
        rows.append((*a, _walk(a[0], rng.randint(1, 4)), _walk(a[1], rng.randint(-4, 4)),
                     _walk(a[0], rng.randint(-4, 8)), _walk(a[1], rng.randint(-4, 8))))
    abc = np.array(rows, dtype=np.float64)
    say(f"device orient on {len(rows)} triples")
    got = ctx.debug_orient(to_dev(torch_dev, abc))
    want = np.array([oracle.orient(r[0:2], r[2:4], r[4:6]) for r in rows])
    assert (got == want).all()
    for r, g in list(zip(rows, got))[:: 97]:
        assert g == orient_q(r[0:2], r[2:4], r[4:6])


def test_device_orient_shared_coordinates(torch_dev, ctx):
    """Triples with repeated points or a shared x or y coordinate (exactly
    collinear or not), at several scales: the exact-zero shortcut of the
    predicate and the cases next to it."""
    rng = random.Random(43)
    rows = []
    for _ in range(4000):
        s = math.ldexp(1.0, rng.choice([-290, -40, 0, 40, 290]))
        a = (rng.uniform(-1, 1) * s, rng.uniform(-1, 1) * s)
        b = (rng.uniform(-1, 1) * s, rng.uniform(-1, 1) * s)
        y1 = rng.uniform(-1, 1) * s
        rows += [(*a, *a, *b), (*a, *b, *a), (*a, *b, *b), (*a, *a, *a),
                 (*a, a[0], b[1], *b), (a[0], y1, *a, a[0], b[1]), (y1, a[1], *a, b[0], a[1]),
                 (*a, a[0], b[1], b[0], a[1]), (*a, b[0], a[1], *b),
                 (*a, _walk(a[0], 1), a[1], a[0], _walk(a[1], 1))]
    abc = np.array(rows, dtype=np.float64)
    say(f"device orient on {len(rows)} degenerate triples")
    got = ctx.debug_orient(to_dev(torch_dev, abc))
    for r, g in zip(rows, got):
        assert g == orient_q(r[0:2], r[2:4], r[4:6]), r


def _key_q(x, y, x0, y0):
    from fractions import Fraction
    dx = Fraction(x) - Fraction(x0)
    dy = Fraction(y) - Fraction(y0)
    s = dy / (abs(dx) + dy)
    return math.floor((s if dx >= 0 else 2 - s) * 2 ** 31)


def test_device_angle_key_vs_exact(torch_dev, ctx):
    rng = random.Random(42)
    x0, y0 = 0.5, 0.25
    pts = []
    for _ in range(3000):
        k = rng.randrange(1, 2 ** 32 - 1)
        if k < 2 ** 31:
            dx, dy = float(2 ** 31 - k), float(k)
        else:
            dx, dy = -float(k - 2 ** 31), float(2 ** 32 - k)
        sc = math.ldexp(1.0, rng.randint(-30, 30))
        x, y = x0 + dx * sc, y0 + dy * sc
        for px, py in [(x, y), (_walk(x, 1), y), (_walk(x, -1), y), (x, _walk(y, -1))]:
            if py > y0 or (py == y0 and px > x0):
                pts.append((px, py))
    for _ in range(3000):
        pts.append((rng.uniform(-1, 2), y0 + rng.random()))
    arr = np.array(pts, dtype=np.float64)
    say(f"device angle key on {len(pts)} points")
    got = ctx.debug_angle_key(to_dev(torch_dev, arr), x0, y0)
    want = np.array([_key_q(p[0], p[1], x0, y0) for p in pts], dtype=np.uint64)
    assert (got.astype(np.uint64) == want).all()


# ------------------------------------------------------------- small inputs
def _cases():
    t = np.arange(-700, 800, dtype=np.float64)
    c = {
        "square_100k": synth.square(100_000, (1, 1)),
        "square_100003": synth.square(100_003, (51, 1)),
        "disk_100k": synth.disk(100_000, (52, 1)),
        "gauss_50k": synth.gaussian(50_000, 1.0, (53, 1)),
        "mixture_100k": synth.mixture(100_000, (54, 1)),
        "annulus_ngon_100k": synth.annulus_ngon(50_000, 50_000, 14, ((55, 1), (56, 1), (57, 1))),
        "grid_draws_100k": synth.grid_draws(100_000, 64, (58, 1)),
        "grid_200x3": synth.grid(200, 3, (59, 1)),
        "ngon_4096": synth.ngon(4096, 12, (60, 1)),
        "collinear_1500": np.stack([t, 2 * t - 5], axis=1)[np.random.default_rng(1).permutation(1500)],
        "collinear_dups": np.repeat(np.stack([t[:40], -t[:40]], axis=1), 3, axis=0),
        "collinear_10k": np.stack([np.arange(10_000.0), 0.5 * np.arange(10_000.0) + 3.0],
                                  axis=1)[np.random.default_rng(2).permutation(10_000)],
        "dup_heavy": np.concatenate([np.full((5000, 2), 0.25), synth.square(3000, (65, 1)),
                                     np.full((3000, 2), 1.0)])[np.random.default_rng(3).permutation(11_000)],
        "all_equal_1000": np.full((1000, 2), 0.375),
        "one": np.array([[0.25, -0.5]]),
        "two_same": np.array([[1.0, 1.0], [1.0, 1.0]]),
        "two": np.array([[1.0, 3.0], [-1.0, 2.0]]),
        "three_collinear": np.array([[0.0, 0.0], [2.0, 2.0], [1.0, 1.0]]),
        "triangle_interior": np.array([[0.0, 0.0], [4.0, 0.0], [0.0, 4.0], [1.0, 1.0], [-0.0, 0.0]]),
        "tiny_magnitudes": (1.0 + synth.square(5000, (61, 1))) * math.ldexp(1.0, -290),
        "huge_magnitudes": (synth.disk(5000, (62, 1)) - 0.5) * math.ldexp(1.0, 290),
    }
    return c


CASES = _cases()


@pytest.mark.parametrize("name", sorted(CASES))
def test_hull_equals_oracle(torch_dev, ctx, name):
    pts = CASES[name]
    say(f"hull {name} n={len(pts)}")
    got = ctx.compute(to_dev(torch_dev, pts))
    want = oracle.hull(pts)
    assert got.tolist() == want.tolist()
    st = ctx.last_stats
    assert st.n_hull == len(want)


@pytest.mark.parametrize("mode", ["bucketed", "full", "paper", "chunk5"])
@pytest.mark.parametrize("name", ["square_100k", "disk_100k", "grid_draws_100k", "annulus_ngon_100k",
                                  "collinear_1500", "grid_200x3", "mixture_100k", "collinear_10k",
                                  "dup_heavy"])
def test_stages_equal_model(torch_dev, hx, name, mode):
    chunk, full = {"bucketed": (0, False), "full": (0, True), "paper": (-1, True),
                   "chunk5": (5, True)}[mode]
    pts = CASES[name]
    say(f"stages {name} mode={mode}")
    c = hx.Hull2D(round2_chunk=chunk, full_sort=full)
    got = c.compute(to_dev(torch_dev, pts))
    m = oracle.model(pts, chunk)
    s = c.stages(len(pts) + 1)
    assert s["extremes"] == m["extremes"]
    assert s["n_sorted"] == len(m["sorted"])
    if mode != "bucketed":
        assert s["sorted"].tolist() == m["sorted"].tolist()
    else:
        assert s["sorted"] is None
        assert s["n_candidates"] <= max(len(m["sorted"]), 1)
    if len(m["sorted"]):
        assert s["l"] == m["l"]
        assert s["longest"] == m["longest"]
    assert s["round2"].tolist() == m["round2"].tolist()
    assert got.tolist() == m["hull"].tolist()
    st = c.last_stats
    assert st.n_round1 == m["m1"]
    assert st.n_round2 == m["m2"]
    c.close()


TAIL_SLOTS = 65536  # candidates the one-workgroup tail reads (16-bit slots)


@pytest.mark.parametrize("name", ["square_100k", "disk_100k", "dup_heavy", "collinear_10k",
                                  "annulus_ngon_100k", "grid_draws_100k", "annulus_400k"])
def test_tail_and_fallback_paths(torch_dev, hx, name):
    """The bucketed mode finishes small candidate sets in one workgroup and
    larger ones with the multi-kernel path; both match the oracle.  The
    candidates come from bucket maxima over a sample of the survivors, so
    they may include points the exact table would not select (the tail
    narrows them to those; the multi-kernel path walks them all)."""
    pts = synth.annulus(400_000, 0.9999, (66, 1)) if name == "annulus_400k" else CASES[name]
    say(f"tail/fallback {name}")
    c = hx.Hull2D(profile=True)
    got = c.compute(to_dev(torch_dev, pts))
    assert got.tolist() == oracle.hull(pts).tolist()
    st = c.last_stats
    tail_ran = st.ms_stage["tail"] > 0.0
    sort_ran = st.ms_stage["histogram"] > 0.0
    assert tail_ran or sort_ran
    if st.n_candidates > TAIL_SLOTS:
        assert sort_ran
    if name in ("square_100k", "disk_100k"):
        assert tail_ran and not sort_ran
    if name == "annulus_400k":
        assert st.n_candidates > TAIL_SLOTS
    c.close()


@pytest.mark.parametrize("side,n", [(2, 1000), (3, 100_000), (8, 100_003), (64, 100_000),
                                    (64, 1_000_003), (1000, 2_000_000)])
def test_extremes_tie_heavy(torch_dev, ctx, side, n):
    """Step 1 tie rules on inputs where every criterion has many ties."""
    pts = synth.grid_draws(n, side, (70 + side, n % 97))
    say(f"extremes grid draws side={side} n={n}")
    ctx.compute(to_dev(torch_dev, pts))
    x, y = pts[:, 0], pts[:, 1]
    idx = np.arange(n)
    want = [int(np.lexsort((idx, -y, x))[0]), int(np.lexsort((idx, x, y))[0]),
            int(np.lexsort((idx, y, -x))[0]), int(np.lexsort((idx, -x, -y))[0])]
    assert ctx.stages(n + 1)["extremes"] == want


def test_repeatable(torch_dev, ctx):
    pts = CASES["disk_100k"]
    d = to_dev(torch_dev, pts)
    a = ctx.compute(d)
    for _ in range(5):
        assert ctx.compute(d).tolist() == a.tolist()


def test_workspace_shrink_and_grow(torch_dev, ctx):
    for name in ["square_100k", "one", "annulus_ngon_100k", "two", "square_100003"]:
        pts = CASES[name]
        assert ctx.compute(to_dev(torch_dev, pts)).tolist() == oracle.hull(pts).tolist()


@pytest.mark.parametrize("bad,status", [(float("nan"), 2), (float("inf"), 2), (1e-310, 3),
                                        (math.ldexp(1.0, 301), 3)])
def test_domain_errors(torch_dev, hx, ctx, bad, status):
    pts = synth.square(10_000, (63, 1))
    pts[4321, 1] = bad
    with pytest.raises(hx.HullError) as e:
        ctx.compute(to_dev(torch_dev, pts))
    assert e.value.status == status
    # the context stays usable
    ok = synth.square(1000, (64, 1))
    assert ctx.compute(to_dev(torch_dev, ok)).tolist() == oracle.hull(ok).tolist()


def test_empty_and_capacity(torch_dev, hx, ctx):
    import ctypes
    import torch
    empty = torch.zeros((0, 2), dtype=torch.float64, device="cuda")
    assert ctx.compute(empty).tolist() == []
    pts = CASES["disk_100k"]
    want = oracle.hull(pts)
    d = to_dev(torch_dev, pts)
    lib = hx.load_library()
    out = np.zeros(4, dtype=np.int32)
    n_out = ctypes.c_int64(0)
    st = lib.hull2d_compute(ctx._h, ctypes.c_void_p(d.data_ptr()), len(pts),
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 4,
                            ctypes.byref(n_out), None)
    assert st == hx.CAPACITY
    assert n_out.value == len(want)
    assert (out == 0).all()


# ---------------------------------------------------------------- full size
def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["square_20M", "disk_20M", "annulus_ngon_20M", "grid_500x4",
                                  "mixture_20M"])
def test_full_size_matches_golden(torch_dev, ctx, name):
    g = _golden()[name]
    say(f"full size {name}: generating")
    pts = synth.workload(name)
    assert pts.shape[0] == g["n"]
    assert synth.content_hash(pts) == g["input_hash"]
    say(f"full size {name}: hull on GPU")
    got = ctx.compute(to_dev(torch_dev, pts))
    assert len(got) == g["h"]
    assert got[:16].tolist() == g["head"]
    assert hashlib.sha256(np.ascontiguousarray(got, dtype="<i4").tobytes()).hexdigest() == g["sha256"]
    st = ctx.last_stats
    say(f"  n={st.n} round1={st.n_round1} round2={st.n_round2} h={st.n_hull} "
        f"ms={st.ms_total:.3f}")


WEIGHTS = os.path.join(ROOT, "paper_1508_05931_amd", "weights", "filter16.f32")


@pytest.mark.parametrize("name,mode", [("square_20M", "full_sort"), ("disk_20M", "full_sort"),
                                       ("mixture_20M", "learned")])
def test_full_size_modes_match_golden(torch_dev, hx, name, mode):
    """The paper's Step 4 as printed (every round-1 survivor sorted) on the
    20M square and disk, and the learned filter with the shipped weights on
    its own 20M mixture: the same oracle-written hulls as the default path."""
    if mode == "learned" and not os.path.exists(WEIGHTS):
        pytest.skip("no trained weights in the tree")
    g = _golden()[name]
    say(f"full size {name} ({mode}): generating")
    pts = synth.workload(name)
    assert synth.content_hash(pts) == g["input_hash"]
    c = hx.Hull2D(full_sort=True) if mode == "full_sort" else hx.Hull2D(learned=True, weights=WEIGHTS)
    say(f"full size {name} ({mode}): hull on GPU")
    got = c.compute(to_dev(torch_dev, pts))
    assert len(got) == g["h"]
    assert got[:16].tolist() == g["head"]
    assert hashlib.sha256(np.ascontiguousarray(got, dtype="<i4").tobytes()).hexdigest() == g["sha256"]
    st = c.last_stats
    if mode == "full_sort":
        assert st.n_candidates == st.n_sorted
    say(f"  n={st.n} round1={st.n_round1} round2={st.n_round2} h={st.n_hull}")
    c.close()


def _without_pivot_copies(pts, keep, pivot):
    px, py = pts[pivot]
    return np.flatnonzero(keep & ~((pts[:, 0] == px) & (pts[:, 1] == py))).astype(np.int32)


@pytest.mark.parametrize("mode", ["bucketed", "full_sort", "learned"])
def test_round1_survivors_element_by_element(torch_dev, hx, mode):
    """Step 2's survivors, index by index, on sets of over a million points:
    the quadrilateral's against the oracle's model (the bucketed and the
    full-sort modes share Step 2 but not what follows), the learned polygon's
    against the oracle's learned first round for the directions the device
    used."""
    if mode == "learned":
        if not os.path.exists(WEIGHTS):
            pytest.skip("no trained weights in the tree")
        pts = synth.mixture(1_500_007, (81, 1))
        c = hx.Hull2D(learned=True, weights=WEIGHTS)
    else:
        pts = synth.disk(1_000_003, (80, 1)) if mode == "bucketed" else synth.square(1_200_001, (82, 1))
        c = hx.Hull2D(full_sort=(mode == "full_sort"))
    say(f"round-1 survivors {mode} n={len(pts)}")
    c.compute(to_dev(torch_dev, pts))
    got = c.round1_survivors()
    m = oracle.model(pts)
    if mode == "learned":
        keep = oracle.learned_round1(pts, c.learned_info()["dirs"])["keep"]
    else:
        keep = m["round1_keep"]
    want = _without_pivot_copies(pts, keep, m["pivot"])
    assert got.shape == want.shape
    assert np.array_equal(got, want)
    assert c.last_stats.n_sorted == len(want)
    c.close()


def _ngon(k, seed):
    """k vertices of a regular k-gon (every point a hull vertex), shuffled."""
    return synth.ngon(k, int(math.log2(k)), seed)


@pytest.mark.parametrize("name,full,where", [
    ("square_100k", False, "device"),       # one part
    ("disk_100k", False, "device"),
    ("grid_200x3", False, "device"),        # collinear and repeated kept points
    ("dup_heavy", False, "device"),
    ("ngon_16384", False, "host"),          # three parts whose chains overflow one workgroup
    ("disk_100k", True, "device"),          # list form (multi-kernel path)
    ("collinear_10k", True, "device"),
    ("ngon_131072", True, "host"),          # list form, chains overflow
])
def test_step8_device_and_host_fallback(torch_dev, hx, name, full, where):
    """Step 8 on the device (options.scan = 1: chunk scans joined at common
    tangents) falls back to the host scan when the parts' chains do not fit
    one workgroup; the hull equals the oracle's either way."""
    pts = {"ngon_16384": lambda: _ngon(16384, (98, 1)),
           "ngon_131072": lambda: _ngon(131072, (99, 1))}.get(name, lambda: CASES[name])()
    say(f"step 8 {name} full={full}")
    c = hx.Hull2D(profile=True, full_sort=full, scan=1)
    got = c.compute(to_dev(torch_dev, pts))
    assert got.tolist() == oracle.hull(pts).tolist()
    st = c.last_stats
    if where == "device":
        assert st.ms_stage["host_scan"] == 0.0 and st.ms_stage["scan"] > 0.0
    else:
        assert st.ms_stage["host_scan"] > 0.0
    m = oracle.model(pts)
    s = c.stages(len(pts) + 1)
    assert s["round2"].tolist() == m["round2"].tolist()
    c.close()


@pytest.mark.parametrize("name,full,where", [
    ("disk_100k", False, "host"),           # the tail's kept points: host by default
    ("annulus_400k", False, "device"),      # over 65,536 kept points by the multi-kernel path
])
def test_step8_default_placement(torch_dev, hx, name, full, where):
    pts = synth.annulus(400_000, 0.9999, (66, 1)) if name == "annulus_400k" else CASES[name]
    c = hx.Hull2D(profile=True, full_sort=full)
    got = c.compute(to_dev(torch_dev, pts))
    assert got.tolist() == oracle.hull(pts).tolist()
    st = c.last_stats
    say(f"step 8 default {name}: kept {st.n_round2} host {st.ms_stage['host_scan']:.3f} "
        f"device {st.ms_stage['scan']:.3f}")
    if where == "host":
        assert st.ms_stage["scan"] == 0.0 and st.ms_stage["host_scan"] > 0.0
    elif st.n_round2 > 65536:
        assert st.ms_stage["scan"] > 0.0


def test_out_of_memory_path(torch_dev, hx):
    """A workspace limit makes the allocation fail: OUT_OF_MEMORY, nothing
    written, and the context still computes inputs that fit."""
    c = hx.Hull2D(workspace_limit_mib=16)
    big = synth.square(1_000_000, (83, 1))
    with pytest.raises(hx.HullError) as e:
        c.compute(to_dev(torch_dev, big))
    assert e.value.status == hx.OUT_OF_MEMORY
    small = synth.disk(50_000, (84, 1))
    assert c.compute(to_dev(torch_dev, small)).tolist() == oracle.hull(small).tolist()
    with pytest.raises(hx.HullError) as e:
        c.compute(to_dev(torch_dev, big))
    assert e.value.status == hx.OUT_OF_MEMORY
    c.close()
