"""Pins for the oracle's canonical hull (monotone chain).

Checked against: O(n^3) exact brute force on tiny inputs (random, collinear,
duplicate-heavy, small grids); closed forms (points on a parabola, regular
2^k-gons, a full integer grid, collinear sets, all-equal sets, n = 0, 1, 2);
exact invariants on larger inputs (containment, strict convexity, smallest
index per vertex, lexicographic start); and scipy's Qhull on generic inputs.
"""
import random

import numpy as np
import pytest

import oracle
import synth
from tests.exact_ref import brute_hull, orient_q


def _check_invariants(pts, hull_idx):
    """Exact invariants of a canonical hull (independent of how it was built)."""
    h = len(hull_idx)
    P = [tuple(map(float, pts[i])) for i in hull_idx]
    # smallest index holding each vertex value, distinct vertices
    first = {}
    for i, p in enumerate(map(tuple, pts)):
        first.setdefault((float(p[0]), float(p[1])), i)
    assert len(set(P)) == h
    for i, p in zip(hull_idx, P):
        assert first[p] == i
    if h >= 1:
        assert P[0] == min(P)
    if h >= 3:
        for k in range(h):
            assert orient_q(P[k], P[(k + 1) % h], P[(k + 2) % h]) > 0
        # containment: every input point is left of or on every edge
        for q in pts:
            for k in range(h):
                assert orient_q(P[k], P[(k + 1) % h], q) >= 0
    elif h == 2:
        for q in pts:
            assert orient_q(P[0], P[1], q) == 0


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_tiny_random(seed):
    rng = random.Random(seed)
    n = rng.randint(1, 22)
    mode = seed % 4
    if mode == 0:
        pts = [(rng.random(), rng.random()) for _ in range(n)]
    elif mode == 1:   # small integer grid: many collinear and duplicate points
        pts = [(float(rng.randint(0, 3)), float(rng.randint(0, 3))) for _ in range(n)]
    elif mode == 2:   # points on two lines plus duplicates
        pts = []
        for _ in range(n):
            t = rng.randint(-3, 3)
            pts.append((float(t), float(2 * t + 1)) if rng.random() < 0.6 else (float(t), 0.0))
        pts += pts[: n // 3]
    else:             # near-degenerate: points on a segment moved by ulps
        import math
        pts = []
        for _ in range(n):
            t = rng.random()
            x, y = 0.1 + 0.3 * t, 0.7 - 0.2 * t
            for _ in range(rng.randint(0, 2)):
                x = math.nextafter(x, 2.0)
            pts.append((x, y))
    pts = np.array(pts, dtype=np.float64).reshape(-1, 2)
    got = oracle.hull(pts).tolist()
    assert got == brute_hull(pts.tolist())
    _check_invariants(pts, got)


def test_parabola_all_vertices_in_x_order():
    xs = np.arange(-300, 301, 7, dtype=np.float64)
    rng = np.random.default_rng(1)
    perm = rng.permutation(len(xs))
    pts = np.stack([xs[perm], xs[perm] ** 2], axis=1)
    got = oracle.hull(pts)
    assert got.tolist() == np.argsort(pts[:, 0]).tolist()


@pytest.mark.parametrize("log2k", [4, 8, 12, 16])
def test_regular_polygon_all_vertices(log2k):
    K = 1 << log2k
    pts = synth.ngon(K, log2k)
    got = oracle.hull(pts)
    assert len(got) == K
    start = min(range(K), key=lambda i: (pts[i, 0], pts[i, 1]))
    assert got.tolist() == [(start + j) % K for j in range(K)]


def test_full_grid_gives_four_corners():
    pts = synth.grid(30, 3, (7, 5))
    got = oracle.hull(pts)
    corners = [(0.0, 0.0), (29.0, 0.0), (29.0, 29.0), (0.0, 29.0)]
    want = []
    for c in corners:
        want.append(int(np.flatnonzero((pts[:, 0] == c[0]) & (pts[:, 1] == c[1]))[0]))
    assert got.tolist() == want


def test_collinear_gives_two_endpoints():
    rng = np.random.default_rng(2)
    t = rng.integers(-50, 50, size=200).astype(np.float64)
    pts = np.stack([t, 3 * t - 2], axis=1)
    got = oracle.hull(pts)
    lo = int(np.flatnonzero(t == t.min())[0])
    hi = int(np.flatnonzero(t == t.max())[0])
    assert got.tolist() == [lo, hi]


def test_all_equal_and_tiny():
    assert oracle.hull(np.zeros((0, 2))).tolist() == []
    assert oracle.hull(np.array([[0.5, 0.5]])).tolist() == [0]
    assert oracle.hull(np.full((7, 2), 0.25)).tolist() == [0]
    assert oracle.hull(np.array([[1.0, 2.0], [1.0, 2.0]])).tolist() == [0]
    assert oracle.hull(np.array([[3.0, 2.0], [1.0, 2.0]])).tolist() == [1, 0]
    assert oracle.hull(np.array([[0.0, 0.0], [-0.0, 0.0], [1.0, 0.0]])).tolist() == [0, 2]


def test_negative_zero_equals_zero():
    pts = np.array([[-0.0, -0.0], [1.0, 0.0], [0.0, 0.0], [0.0, 1.0]])
    assert oracle.hull(pts).tolist() == [0, 1, 3]


@pytest.mark.parametrize("gen", ["square", "disk", "gaussian"])
def test_invariants_medium(gen):
    pts = {"square": lambda: synth.square(1500, (11, 1)),
           "disk": lambda: synth.disk(1500, (12, 1)),
           "gaussian": lambda: synth.gaussian(1500, 1.0, (13, 1))}[gen]()
    got = oracle.hull(pts).tolist()
    _check_invariants(pts, got)


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_matches_qhull_on_generic_input(seed):
    from scipy.spatial import ConvexHull
    pts = synth.disk(50_000, (seed, 1))
    got = oracle.hull(pts)
    qh = ConvexHull(pts)
    assert sorted(got.tolist()) == sorted(qh.vertices.tolist())
