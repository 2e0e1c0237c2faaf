"""Pins of the learned-filter oracle and of the network reference.

The learned first round must keep every hull vertex, keep nothing the
quadrilateral discards, match a brute-force exact evaluation of its
definition on small integer inputs, take its direction candidates from the
network's sample only, discard between the quadrilateral and the
candidates' own hull, and give the closed-form survivor count on a regular
polygon.  The network reference's gradient must match central
finite differences, and its layers must reduce to the bias on zero weights.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp
from tests.exact_ref import brute_hull, orient_q


def _uniform_dirs(k=16, phase=0.0):
    return [(math.cos(phase + 2 * math.pi * j / k), math.sin(phase + 2 * math.pi * j / k))
            for j in range(k)]


@pytest.mark.parametrize("name,seed", [("mixture", 1), ("disk", 2), ("square", 3), ("gauss", 4)])
def test_learned_keeps_hull_and_is_inside_quad(name, seed):
    gen = {"mixture": lambda: synth.mixture(30_000, (300 + seed, 1)),
           "disk": lambda: synth.disk(30_000, (300 + seed, 1)),
           "square": lambda: synth.square(30_000, (300 + seed, 1)),
           "gauss": lambda: synth.gaussian(30_000, 1.0, (300 + seed, 1))}[name]
    pts = gen()
    rng = np.random.default_rng(seed)
    q = oracle.model(pts)
    h = oracle.hull(pts)
    for dirs in (_uniform_dirs(), rng.normal(size=(16, 2)), np.ones((16, 2))):
        r = oracle.learned_round1(pts, dirs)
        assert r["keep"][h].all()                         # hull vertices always survive
        assert np.all(~r["keep"] | q["round1_keep"])      # never more than the quadrilateral
        assert r["m1"] == int(r["keep"].sum())
        assert r["m1"] <= q["m1"]


def _inside_q(poly, p):
    return len(poly) >= 3 and all(orient_q(poly[e], poly[(e + 1) % len(poly)], p) > 0
                                  for e in range(len(poly)))


def test_learned_matches_brute_force_on_integer_points():
    """Integer points and directions: every product is exact, so the argmax,
    the hull of the candidates and the strict-inside tests can be evaluated in
    rational arithmetic independently.  Below 4096 points the sample is every
    point."""
    rng = np.random.default_rng(7)
    for trial in range(40):
        n = int(rng.integers(1, 60))
        pts = rng.integers(-20, 21, size=(n, 2)).astype(np.float64)
        k = int(rng.integers(0, 9))
        dirs = rng.integers(-5, 6, size=(k, 2)).astype(np.float64)
        r = oracle.learned_round1(pts, dirs)
        # candidates: Step-1 extremes with their tie rules, then exact argmax
        P = [(int(x), int(y)) for x, y in pts]
        idx = range(n)
        ext = [min(idx, key=lambda i: (P[i][0], -P[i][1], i)),
               min(idx, key=lambda i: (P[i][1], P[i][0], i)),
               min(idx, key=lambda i: (-P[i][0], P[i][1], i)),
               min(idx, key=lambda i: (-P[i][1], -P[i][0], i))]
        dc = [min(idx, key=lambda i: (-(P[i][0] * int(ux) + P[i][1] * int(uy)), i)) for ux, uy in dirs]
        assert r["cand"].tolist() == ext + dc
        cpts = np.array([P[i] for i in ext + dc], dtype=np.float64)
        ppts = [cpts[v] for v in brute_hull(cpts)]       # exact strict corners, CCW
        for i in range(n):
            assert r["keep"][i] == (not _inside_q(ppts, pts[i])), (trial, i)


def test_learned_directions_use_the_sample_only():
    """The direction candidates come from the network's sample (above 4096
    points: 16 blocks of 256, block b at floor(b n / 16)): a point far out
    along every direction placed outside the sample is never a candidate,
    while the same point inside it is the candidate of every direction it
    wins.  Checked against an independent integer argmax over the sample."""
    rng = np.random.default_rng(11)
    n = 3 * 4096 + 777                                   # blocks start at b * 816.56...
    pts = rng.integers(-1000, 1001, size=(n, 2)).astype(np.float64)
    dirs = rng.integers(-5, 6, size=(9, 2)).astype(np.float64)
    dirs[0] = (1.0, 1.0)
    sample = [(b * n) // 16 + j for b in range(16) for j in range(256)]
    assert sample == mlp.sample_index(n).tolist()        # the histogram's sample
    assert {0, 255, 816, 1071, 12248, 12503} <= set(sample)
    assert not {256, 815, 1072, 4500, 12247, 12504, n - 1} & set(sample)

    def expect(p):
        P = [(int(x), int(y)) for x, y in p]
        return [min(sample, key=lambda i: (-(P[i][0] * int(ux) + P[i][1] * int(uy)), i))
                for ux, uy in dirs]

    for far in (256, 815, 4500, 12504, n - 1):           # outside the sample
        p = pts.copy()
        p[far] = (10_000.0, 10_000.0)
        r = oracle.learned_round1(p, dirs)
        assert r["cand"][4:].tolist() == expect(p)
        assert far not in r["cand"][4:].tolist()
        assert r["keep"][far]                            # a Step-1 extreme: survives
    for far in (0, 255, 816 + 17, 12503):                # inside the sample
        p = pts.copy()
        p[far] = (10_000.0, 10_000.0)
        r = oracle.learned_round1(p, dirs)
        assert r["cand"][4:].tolist() == expect(p)
        assert r["cand"][4] == far


def test_learned_polygon_contains_the_quadrilateral():
    """The polygon is the hull of the direction candidates and the four
    Step-1 extremes: a point inside the quadrilateral but outside the
    candidates' own hull is discarded, and so is one between the two that
    neither holds alone."""
    ring = [(0.0, 5.0), (5.0, 0.0), (10.0, 5.0), (5.0, 10.0)]   # the Step-1 extremes
    tri = [(0.0, 0.0), (9.0, 0.0), (0.0, 9.0)]                   # sample candidates
    probe = [(5.0, 5.0), (1.0, 1.0), (7.0, 6.0), (9.0, 3.0), (9.9, 0.5)]
    pts = np.array(ring + tri + probe)
    dirs = [(-1.0, -1.0), (1.0, -10.0), (-10.0, 1.0)]
    r = oracle.learned_round1(pts, dirs)
    assert r["cand"][4:].tolist() == [4, 5, 6]
    # (5, 5) in both, (1, 1) only in the triangle, (7, 6) only in the
    # quadrilateral, (9, 3) in neither but inside their hull; (9.9, 0.5) outside
    assert r["keep"][7:].tolist() == [False, False, False, False, True]
    assert r["keep"][:7].all()


def test_learned_regular_polygon_closed_form():
    """64 vertices of a regular polygon plus interior points; the 16
    directions at multiples of 2 pi / 16 select every 4th vertex, the
    polygon is the inscribed 16-gon, which holds every interior point of
    radius below cos(pi/16): exactly the 64 vertices survive."""
    th = 2 * np.pi * np.arange(64) / 64
    ring = np.stack([np.cos(th), np.sin(th)], axis=1)
    inner = synth.disk(5000, (310, 1)) * 0.9
    pts = np.concatenate([ring, inner])
    r = oracle.learned_round1(pts, _uniform_dirs())
    assert sorted(r["cand"][4:].tolist()) == list(range(0, 64, 4))
    assert r["m1"] == 64 and r["keep"][:64].all()


def test_learned_degenerate_inputs():
    one = np.array([[0.5, 0.5]])
    assert oracle.learned_round1(one, _uniform_dirs())["m1"] == 1
    line = np.stack([np.arange(50.0), 2 * np.arange(50.0)], axis=1)
    assert oracle.learned_round1(line, _uniform_dirs())["m1"] == 50   # no polygon: keep all
    with pytest.raises(oracle.OracleError):
        oracle.learned_round1(one, [(float("nan"), 1.0)])


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    flat = rng.normal(scale=0.05, size=mlp.N_PARAMS)
    x = rng.random(size=(3, mlp.N_IN)) * 2
    t = rng.normal(size=(3, mlp.N_OUT))
    g = mlp.grad(flat, x, t)
    for j in rng.choice(mlp.N_PARAMS, 60, replace=False):
        e = np.zeros_like(flat)
        e[j] = 1e-6
        fd = (mlp.loss(flat + e, x, t) - mlp.loss(flat - e, x, t)) / 2e-6
        assert abs(fd - g[j]) <= 1e-6 + 1e-4 * abs(fd), (j, fd, g[j])


def test_mlp_zero_weights_give_bias_and_bf16_rounding():
    p = {name: np.zeros(shp) for name, shp in mlp.SHAPES}
    p["b3"] = np.arange(mlp.N_OUT, dtype=np.float64) - 7.5
    y, _ = mlp.forward(mlp.pack(p), np.ones((2, mlp.N_IN)))
    assert np.array_equal(y, np.tile(p["b3"], (2, 1)))
    # bfloat16: 8 significant bits, ties to even
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -3.140625], dtype=np.float32)
    assert mlp.bf16(v).tolist() == [1.0, 1.0, 1.0 + 2 ** -6, 1.0, -3.140625]


def test_histogram_definition():
    pts = synth.square(65_536, (320, 1))
    h = mlp.histogram(pts)
    assert h.shape == (1024,) and abs(float(h.sum()) - 1024.0) < 1e-2
    s = mlp.sample_index(65_536)
    assert s.size == 4096 and s[0] == 0 and s[255] == 255 and s[256] == 4096
    # every 16th block of 256 at this size
    i = np.arange(65_536)
    assert np.array_equal(s, i[((i >> 8) & 15) == 0])
    # 4096 points at any larger size, blocks at floor(b n / 16), inside [0, n)
    for n in (4097, 100_003, 20_000_000):
        t = mlp.sample_index(n)
        assert t.size == 4096 and np.all(np.diff(t) > 0) and t[-1] < n
        assert [int(t[256 * b]) for b in (1, 7, 15)] == [n // 16, 7 * n // 16, 15 * n // 16]
    assert np.array_equal(mlp.sample_index(4096), np.arange(4096))
    assert np.array_equal(mlp.sample_index(37), np.arange(37))
    # the sample's four extreme coordinates land in the corner cells' rows / columns
    q = pts[s]
    assert h.reshape(32, 32)[:, 0].sum() > 0 and h.reshape(32, 32)[:, 31].sum() > 0
    assert np.allclose(h.reshape(32, 32).sum(), 1024.0)
    assert mlp.histogram(np.zeros((0, 2))).sum() == 0



def _sparse_params():
    """A network whose only non-zero parameters are the few below, so every
    output can be worked out by hand (values are float32 and dyadic)."""
    p = {name: np.zeros(shp) for name, shp in mlp.SHAPES}
    # layer 1: unit 0 = x0 + 2^-9 (not a bfloat16 value: rounds down to 1
    # when x0 = 1); unit 1 = x1 + 2^-8 - 2 (for x1 = 3 a tie between 1 and
    # 1 + 2^-7 -> even -> 1)
    p["W1"][0, 0] = 1.0
    p["b1"][0] = 2.0 ** -9
    p["W1"][1, 1] = 1.0
    p["b1"][1] = 2.0 ** -8 - 2.0
    # layer 2: identity on units 0 and 1
    p["W2"][0, 0] = 1.0
    p["W2"][1, 1] = 1.0
    # layer 3: y0 = 3 h0 + 1/4; y1 = w h1 + b with w = 1 + 2^-9 (rounds to 1
    # in bfloat16) and b = 1 + 2^-12 (a float32 bias, not rounded)
    p["W3"][0, 0] = 3.0
    p["b3"][0] = 0.25
    p["W3"][1, 1] = 1.0 + 2.0 ** -9
    p["b3"][1] = 1.0 + 2.0 ** -12
    return mlp.pack(p)


def _sparse_input():
    x = np.zeros((1, mlp.N_IN))
    x[0, 0] = 1.0
    # 3 + 2^-7 is not a bfloat16 value either: the input rounds to 3 first
    x[0, 1] = 3.0 + 2.0 ** -7
    return x


def test_forward_bf16_hand_worked():
    """The inference reference on a hand-worked case: weights and layer inputs
    rounded to bfloat16 (nearest, ties to even), biases kept in float32, the
    last layer's output not rounded.  Expected values by hand, in exact
    rationals:
      x0 = 1 -> z = 1 + 2^-9 -> h1[0] = bf16(z) = 1 (2^-9 < half an ulp 2^-8);
      x1 = bf16(3 + 2^-7) = 3 (ulp at 2 is 2^-6, 2^-7 is a tie -> even 3)
        -> z = 3 + 2^-8 - 2 = 1 + 2^-8, a tie -> h1[1] = 1 (even);
        unrounded, x1 would give 1 + 3*2^-8, a tie -> 1 + 2^-6;
      h2 = h1 (identity, already bfloat16);
      y0 = 3 * 1 + 1/4; y1 = bf16(1 + 2^-9) * 1 + (1 + 2^-12) = 2 + 2^-12;
      every other output is 0."""
    y = mlp.forward_bf16(_sparse_params(), _sparse_input())
    want = np.zeros(mlp.N_OUT)
    want[0] = float(Fraction(3) + Fraction(1, 4))
    want[1] = float(Fraction(2) + Fraction(1, 4096))
    assert y.shape == (1, mlp.N_OUT)
    assert np.array_equal(y[0], want), (y[0][:2], want[:2])
    # the float64 network differs on both outputs (no rounding anywhere)
    y64, _ = mlp.forward(_sparse_params(), _sparse_input())
    assert y64[0, 0] == 3 * (1 + 2.0 ** -9) + 0.25
    assert y64[0, 0] != y[0, 0] and y64[0, 1] != y[0, 1]


def test_forward_bf16_pin_catches_plausible_mistakes(monkeypatch):
    """Each plausible misreading of the inference precision changes the
    hand-worked outputs above: hidden activations left unrounded, biases
    rounded, inputs unrounded, or ties rounded away from zero."""
    params, x = _sparse_params(), _sparse_input()
    want = mlp.forward_bf16(params, x)
    real = mlp.bf16

    def run(fake):
        monkeypatch.setattr(mlp, "bf16", fake)
        try:
            return mlp.forward_bf16(params, x)
        finally:
            monkeypatch.setattr(mlp, "bf16", real)

    calls = {"n": 0}

    def skip_hidden(a):            # 1st call rounds x, 2nd W1, 3rd h1 ...
        calls["n"] += 1
        return np.asarray(a, dtype=np.float64) if calls["n"] in (3, 5) else real(a)

    def skip_input(a):
        calls["n"] += 1
        return np.asarray(a, dtype=np.float64) if calls["n"] == 1 else real(a)

    def ties_away(a):
        f = np.ascontiguousarray(a, dtype=np.float32)
        u = f.view(np.uint32).astype(np.uint64)
        r = ((u + 0x8000) >> 16) << 16
        return r.astype(np.uint32).view(np.float32).astype(np.float64)

    for fake in (skip_hidden, skip_input, ties_away):
        calls["n"] = 0
        assert not np.array_equal(run(fake), want), fake.__name__
    # rounding the biases as well
    p = mlp.unpack(params)
    for k in ("b1", "b2", "b3"):
        p[k] = real(p[k])
    assert not np.array_equal(mlp.forward_bf16(mlp.pack(p), x), want)


def _cell(h, cx, cy):
    return float(h.reshape(32, 32)[cy, cx])


def test_histogram_cell_map_hand_placed():
    """Hand-placed points on a bounding box of 8 x 2 (x from -4 to 4, y from
    1 to 3): a cell is 1/4 wide and 1/16 high, every scale factor is exact,
    and a cell index is cy * 32 + cx with cx = floor((x + 4) * 4) and
    cy = floor((y - 1) * 16), clipped to 31 (the box maximum lands in cell
    31).  Eight points, so each count weighs 1024 / 8 = 128."""
    pts = np.array([
        (-4.0, 1.0),        # box minimum -> (0, 0)
        (4.0, 3.0),         # box maximum -> (31, 31) after clipping 32
        (-2.25, 1.0625),    # (7, 1): x + 4 = 1.75 -> 7; y - 1 = 1/16 -> 1
        (-2.2500000000000004, 1.0),  # one ulp left of the boundary -> (6, 0)
        (0.0, 2.5),         # (16, 24)
        (0.0, 2.5),         # same cell again
        (3.99, 1.01),       # (31, 0)
        (-3.9, 2.99),       # (0, 31)
    ])
    h = mlp.histogram(pts)
    want = {(0, 0): 1, (31, 31): 1, (7, 1): 1, (6, 0): 1, (16, 24): 2, (31, 0): 1, (0, 31): 1}
    for (cx, cy), k in want.items():
        assert _cell(h, cx, cy) == 128.0 * k, (cx, cy)
    assert float(h.sum()) == 128.0 * 8
    # x and y are not interchangeable: the transposed cells are empty
    assert _cell(h, 24, 16) == 0.0 and _cell(h, 1, 7) == 0.0
    # a flat box (all y equal) puts everything in row 0
    flat = np.array([(0.0, 5.0), (1.0, 5.0), (2.0, 5.0), (4.0, 5.0)])
    hf = mlp.histogram(flat)
    assert [_cell(hf, cx, 0) for cx in (0, 8, 16, 31)] == [256.0] * 4
