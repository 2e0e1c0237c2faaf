"""GPU parity of the batched form (hull2d_batch) against the CPU oracle.

Every set's hull must equal the monotone-chain oracle's hull of that set, bit
for bit (set-local indices, canonical order).  Covers empty and one-point
sets, duplicates, collinear sets (including one whose equal-key run is too
long for the workgroup sorter, finished by the single-hull path), grids,
thin annuli whose second round keeps most points (the device Graham scan's
chunk reduction), and the 4096-set workload against an oracle-written hash.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden", "batch.json")


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


@pytest.fixture(scope="module", params=[0, 1], ids=["tiled", "persistent"])
def ctx(hx, request):
    """A context of each batch engine: tiled (the default) and persistent."""
    c = hx.Hull2D(batch_engine=request.param)
    yield c
    c.close()


def _mixed_sets():
    t = np.arange(-700, 800, dtype=np.float64)
    rng = np.random.default_rng(11)
    sets = [
        np.zeros((0, 2)),
        np.array([[0.25, -0.5]]),
        np.array([[1.0, 1.0], [1.0, 1.0]]),
        np.array([[1.0, 3.0], [-1.0, 2.0]]),
        np.array([[0.0, 0.0], [2.0, 2.0], [1.0, 1.0]]),
        np.full((300, 2), 0.375),
        np.stack([t, 2 * t - 5], axis=1)[rng.permutation(1500)],
        np.repeat(np.stack([t[:40], -t[:40]], axis=1), 3, axis=0),
        # one ray from the pivot holds 10,000 points: a run of equal keys
        # longer than the workgroup sorter takes
        np.stack([np.arange(10_000.0), 0.5 * np.arange(10_000.0) + 3.0], axis=1)[rng.permutation(10_000)],
        synth.grid(40, 3, (81, 1)),
        synth.grid_draws(20_000, 16, (82, 1)),
        np.concatenate([np.full((500, 2), 0.25), synth.square(300, (83, 1)),
                        np.full((300, 2), 1.0)])[rng.permutation(1100)],
        synth.ngon(2048, 9, (84, 1)),
    ]
    for i, n in enumerate([64, 100, 1000, 4097, 20_000, 70_000]):
        sets.append(synth.square(n, (90 + i, 1)))
        sets.append(synth.disk(n, (100 + i, 1)))
        sets.append(synth.gaussian(n, 1.0, (110 + i, 1)))
        sets.append(synth.annulus(n, 0.999, (120 + i, 1)))
    sets.append(synth.annulus(150_000, 0.999, (130, 1)))
    sets.append(synth.mixture(50_000, (131, 1)))
    return sets


def _concat(sets):
    offs = np.zeros(len(sets) + 1, dtype=np.int64)
    np.cumsum([len(s) for s in sets], out=offs[1:])
    pts = np.concatenate([np.asarray(s, dtype=np.float64).reshape(-1, 2) for s in sets])
    return np.ascontiguousarray(pts), offs


def _check_all(hulls, out_offs, sets):
    for i, s in enumerate(sets):
        got = hulls[out_offs[i]:out_offs[i + 1]]
        want = oracle.hull(np.ascontiguousarray(s, dtype=np.float64).reshape(-1, 2))
        assert got.tolist() == want.tolist(), f"set {i} (n={len(s)})"


def test_batch_mixed_sets(torch_dev, ctx):
    sets = _mixed_sets()
    pts, offs = _concat(sets)
    say(f"batch mixed S={len(sets)} N={len(pts)}")
    d = torch_dev.from_numpy(pts).cuda()
    hulls, out_offs = ctx.batch(d, offs)
    _check_all(hulls, out_offs, sets)
    assert ctx.last_stats.n_candidates >= 1  # the long collinear run went to the host


def test_batch_tile_boundaries(torch_dev, ctx):
    """Sets one point either side of the 4096-point tile and of two tiles,
    several distributions: the oracle's hulls."""
    sets = []
    for i, n in enumerate([1, 2, 3, 4095, 4096, 4097, 8191, 8192, 8193, 12_289]):
        sets.append(synth.square(n, (160 + i, 1)))
        sets.append(synth.annulus(n, 0.999, (170 + i, 1)))
        sets.append(synth.gaussian(n, 1.0, (180 + i, 1)))
    pts, offs = _concat(sets)
    say(f"batch tile boundaries S={len(sets)}")
    hulls, out_offs = ctx.batch(torch_dev.from_numpy(pts).cuda(), offs)
    _check_all(hulls, out_offs, sets)
    assert ctx.last_stats.n_candidates == 0


def _sliver(n, seed, angle):
    """n points in a thin triangle (height 1e-4 of its length) rotated by
    `angle`: seen from its lowest point nearly every point falls in one or
    two angle buckets."""
    rng = np.random.default_rng(seed)
    u, v = rng.random(n), rng.random(n)
    x, y = u, 1e-4 * u * v
    c, s = np.cos(angle), np.sin(angle)
    return np.stack([c * x - s * y, s * x + c * y], axis=1)


def test_batch_crowded_buckets(torch_dev, ctx):
    """Buckets holding more candidates than one walk tile (the tiled engine
    sorts such a region with the radix sort in HBM); no set needs the host."""
    sets = [_sliver(n, 190 + i, a) for i, (n, a) in
            enumerate([(20_000, 0.3), (9_000, 1.2), (30_000, 2.5), (5_000, -0.7), (60_000, 0.01)])]
    sets.append(synth.square(3000, (199, 1)))
    pts, offs = _concat(sets)
    say(f"batch crowded buckets S={len(sets)}")
    hulls, out_offs = ctx.batch(torch_dev.from_numpy(pts).cuda(), offs)
    _check_all(hulls, out_offs, sets)
    assert ctx.last_stats.n_candidates == 0


def test_batch_equals_compute(torch_dev, ctx):
    """The batched result equals hull2d_compute set by set."""
    sets = [synth.batch_set(int(n), 500 + i)[0] for i, n in enumerate([77, 3000, 12_345, 40_000])]
    pts, offs = _concat(sets)
    say("batch vs compute")
    d = torch_dev.from_numpy(pts).cuda()
    hulls, out_offs = ctx.batch(d, offs)
    for i, s in enumerate(sets):
        one = ctx.compute(torch_dev.from_numpy(np.ascontiguousarray(s)).cuda())
        assert hulls[out_offs[i]:out_offs[i + 1]].tolist() == one.tolist()


def test_batch_repeat_and_shrink(torch_dev, ctx):
    """Two calls in a row, the second smaller, give the oracle's hulls."""
    for S, seed in [(300, 1), (40, 2)]:
        sizes = synth.batch_sizes(S, 64.0, 20_000.0, 900 + seed)
        sets = [synth.batch_set(int(n), k, 900 + seed)[0] for k, n in enumerate(sizes)]
        pts, offs = _concat(sets)
        say(f"batch S={S}")
        hulls, out_offs = ctx.batch(torch_dev.from_numpy(pts).cuda(), offs)
        _check_all(hulls, out_offs, sets)


def test_batch_errors(torch_dev, ctx):
    import paper_1508_05931_amd as hx
    sets = [synth.square(100, (140, 1)), synth.square(100, (141, 1))]
    sets[1][7, 0] = np.nan
    pts, offs = _concat(sets)
    say("batch nonfinite")
    with pytest.raises(hx.HullError) as e:
        ctx.batch(torch_dev.from_numpy(pts).cuda(), offs)
    assert e.value.status == hx.NONFINITE
    sets[1][7, 0] = 2.0 ** 400
    pts, offs = _concat(sets)
    with pytest.raises(hx.HullError) as e:
        ctx.batch(torch_dev.from_numpy(pts).cuda(), offs)
    assert e.value.status == hx.RANGE
    # no sets at all
    h, o = ctx.batch(torch_dev.zeros((0, 2), dtype=torch_dev.float64, device="cuda"),
                     np.zeros(1, dtype=np.int64))
    assert len(h) == 0 and o.tolist() == [0]


def test_batch_capacity(torch_dev, hx):
    """A too-small output buffer: CAPACITY, offsets written, then a retry."""
    import ctypes
    c = hx.Hull2D()
    sets = [synth.disk(5000, (150, 1)), synth.square(3000, (151, 1))]
    pts, offs = _concat(sets)
    d = torch_dev.from_numpy(pts).cuda()
    out = np.empty(4, dtype=np.int32)
    oo = np.zeros(3, dtype=np.int64)
    i64p = ctypes.POINTER(ctypes.c_int64)
    st = c._lib.hull2d_batch(c._h, ctypes.c_void_p(d.data_ptr()), offs.ctypes.data_as(i64p), 2,
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 4,
                             oo.ctypes.data_as(i64p), None)
    assert st == hx.CAPACITY
    want = [oracle.hull(s) for s in sets]
    assert oo.tolist() == [0, len(want[0]), len(want[0]) + len(want[1])]
    hulls, out_offs = c.batch(d, offs)
    _check_all(hulls, out_offs, sets)
    c.close()


def test_batch_4096_sets_golden(torch_dev, ctx):
    """The 4096-set workload (sizes log-uniform in [64, 200000], four
    distributions): hash of all hulls against the oracle's, and a sample of
    sets compared one by one."""
    with open(GOLDEN) as f:
        g = json.load(f)["batch_4096"]
    pts, offs, kinds = synth.batch(4096)
    assert synth.content_hash(pts) == g["input_hash"]
    say(f"batch 4096 sets N={len(pts)}")
    d = torch_dev.from_numpy(pts).cuda()
    hulls, out_offs = ctx.batch(d, offs)
    assert out_offs.tolist()[-1] == g["total"]
    assert hashlib.sha256(np.ascontiguousarray(out_offs, dtype="<i8").tobytes()).hexdigest() == g["offsets_sha256"]
    assert hashlib.sha256(np.ascontiguousarray(hulls, dtype="<i4").tobytes()).hexdigest() == g["sha256"]
    rng = np.random.default_rng(5)
    sizes = np.diff(offs)
    pick = list(rng.choice(4096, 24, replace=False)) + list(np.argsort(sizes)[-4:])
    for i in pick:
        s = pts[offs[i]:offs[i + 1]]
        assert hulls[out_offs[i]:out_offs[i + 1]].tolist() == oracle.hull(s).tolist()


def _graph_sets(seed):
    sizes = synth.batch_sizes(200, 64.0, 20_000.0, 950)
    return [synth.batch_set(int(n), k, seed)[0] for k, n in enumerate(sizes)]


def test_batch_graph_replays_match_eager(torch_dev, hx):
    """The captured batch work, replayed several times with eager work and
    synchronisations between the replays, gives the eager result every time,
    also after new points are written into the same buffer."""
    sets = _graph_sets(951)
    pts, offs = _concat(sets)
    d = torch_dev.from_numpy(pts).cuda()
    cg = hx.Hull2D(batch_graph=True)
    ce = hx.Hull2D(batch_graph=False)
    want_h, want_o = ce.batch(d, offs)
    say("batch graph replays")
    for r in range(4):
        h, o = cg.batch(d, offs)
        assert o.tolist() == want_o.tolist() and h.tolist() == want_h.tolist(), f"replay {r}"
        one = cg.compute(d[offs[3]:offs[4]])
        assert one.tolist() == oracle.hull(sets[3]).tolist()
        torch_dev.cuda.synchronize()
    sets2 = _graph_sets(952)
    pts2, offs2 = _concat(sets2)
    assert offs2.tolist() == offs.tolist()
    d.copy_(torch_dev.from_numpy(pts2))
    torch_dev.cuda.synchronize()
    h2, o2 = cg.batch(d, offs)
    w2, wo2 = ce.batch(d, offs)
    assert o2.tolist() == wo2.tolist() and h2.tolist() == w2.tolist()
    _check_all(h2, o2, sets2)
    cg.close()
    ce.close()


def test_batch_graph_with_large_sets(torch_dev, hx):
    """Sets of 65,536 points and more run on a second stream beside the
    others; the captured graph (fork and join) replayed several times, with
    eager work between the replays, gives the eager result every time."""
    sizes = [70_000, 130_000, 66_000, 90_000] + [int(n) for n in synth.batch_sizes(60, 64.0, 20_000.0, 960)]
    sets = [synth.batch_set(n, k, 961)[0] for k, n in enumerate(sizes)]
    pts, offs = _concat(sets)
    d = torch_dev.from_numpy(pts).cuda()
    ce = hx.Hull2D(batch_graph=False)
    want_h, want_o = ce.batch(d, offs)
    _check_all(want_h, want_o, sets)
    cg = hx.Hull2D(batch_graph=True)
    say("batch graph with large sets")
    for r in range(3):
        h, o = cg.batch(d, offs)
        assert o.tolist() == want_o.tolist() and h.tolist() == want_h.tolist(), f"replay {r}"
        torch_dev.cuda.synchronize()
    cg.close()
    ce.close()


@pytest.mark.parametrize("blocks,order", [(1, 0), (1, 1), (1, 2), (2, 0), (2, 1), (2, 2)])
def test_batch_schedules_agree(torch_dev, hx, blocks, order):
    """Every schedule the autotuner chooses from gives the same hulls."""
    sets = _graph_sets(953)
    pts, offs = _concat(sets)
    d = torch_dev.from_numpy(pts).cuda()
    say(f"batch schedule blocks={blocks} order={order}")
    c = hx.Hull2D(batch_blocks_per_cu=blocks, batch_order=order, batch_engine=1)
    h, o = c.batch(d, offs)
    _check_all(h, o, sets)
    c.close()


@pytest.mark.parametrize("tile,fbits,sbits,side,items", [
    (1024, 0, 0, 0, 2), (65536, 0, 0, 0, 8), (0, 4, 4, 0, 0), (0, 9, 6, -1, 8), (2048, 13, 11, 1, 2),
    (8192, 14, 12, 4096, 4)])
def test_batch_tiled_schedules_agree(torch_dev, hx, tile, fbits, sbits, side, items):
    """Every schedule of the tiled engine (tile size, bucket bits of the
    filter and of the grouping, sets on the second stream, points per thread
    per round) gives the oracle's hulls, eager and replayed from a graph."""
    sizes = [70_000, 130_000, 66_000] + [int(n) for n in synth.batch_sizes(40, 64.0, 20_000.0, 962)]
    sets = [synth.batch_set(n, k, 963)[0] for k, n in enumerate(sizes)]
    sets += [_sliver(9_000, 964, 1.2), np.array([[0.5, 0.5]]), synth.annulus(4097, 0.999, (965, 1))]
    pts, offs = _concat(sets)
    d = torch_dev.from_numpy(pts).cuda()
    say(f"batch tiled schedule tile={tile} fbits={fbits} sbits={sbits} side={side} items={items}")
    kw = dict(batch_tile=tile, batch_filter_bits=fbits, batch_sort_bits=sbits, batch_side_sets=side,
              batch_items=items)
    ce = hx.Hull2D(batch_graph=False, **kw)
    h, o = ce.batch(d, offs)
    _check_all(h, o, sets)
    cg = hx.Hull2D(batch_graph=True, **kw)
    for r in range(2):
        hg, og = cg.batch(d, offs)
        assert og.tolist() == o.tolist() and hg.tolist() == h.tolist(), f"replay {r}"
        torch_dev.cuda.synchronize()
    cg.close()
    ce.close()


def test_batch_tiled_schedule_errors(hx):
    """Schedule values out of range are rejected by the batched call."""
    import torch
    d = torch.zeros((4, 2), dtype=torch.float64, device="cuda")
    offs = np.array([0, 4], dtype=np.int64)
    for kw in (dict(batch_tile=1000), dict(batch_tile=512), dict(batch_tile=131072),
               dict(batch_filter_bits=3), dict(batch_filter_bits=15), dict(batch_sort_bits=13),
               dict(batch_side_sets=-2), dict(batch_side_sets=4097), dict(batch_items=3),
               dict(batch_items=16)):
        c = hx.Hull2D(**kw)
        with pytest.raises(hx.HullError):
            c.batch(d, offs)
        c.close()


@pytest.mark.parametrize("tile,side", [(0, 0), (1024, -1), (65536, 1)])
def test_batch_large_sets(torch_dev, hx, tile, side):
    """Sets of 65,536 to 400,000 points (thin annuli, where every point
    survives Step 2, a disk, a square, a Gaussian) beside small ones, with
    several tile sizes and second-stream splits: the oracle's hulls, eager
    and from a graph."""
    sets = [synth.annulus(200_000, 0.999, (300, 1)), synth.annulus(70_000, 0.999, (301, 1)),
            synth.annulus(300_000, 0.999, (302, 1)), synth.disk(400_000, (303, 1)),
            synth.square(300_000, (304, 1)), synth.annulus(65_536, 0.999, (305, 1)),
            synth.annulus(40_000, 0.999, (306, 1)), synth.gaussian(100_000, 1.0, (307, 1))]
    sets += [synth.batch_set(int(n), k, 308)[0] for k, n in enumerate(synth.batch_sizes(30, 64.0, 30_000.0, 309))]
    pts, offs = _concat(sets)
    d = torch_dev.from_numpy(pts).cuda()
    say(f"batch large sets tile={tile} side={side}")
    kw = dict(batch_tile=tile, batch_side_sets=side)
    ce = hx.Hull2D(batch_graph=False, **kw)
    h, o = ce.batch(d, offs)
    _check_all(h, o, sets)
    assert ce.last_stats.n_candidates == 0
    cg = hx.Hull2D(batch_graph=True, **kw)
    for r in range(2):
        hg, og = cg.batch(d, offs)
        assert og.tolist() == o.tolist() and hg.tolist() == h.tolist(), f"replay {r}"
        torch_dev.cuda.synchronize()
    cg.close()
    ce.close()
