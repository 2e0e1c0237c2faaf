"""Pins for the oracle's model of the paper's Steps 1-8.

Each stage is checked against something other than itself:
  * Step 1 extremes against a numpy lexicographic sort with the tie rules;
  * Step 2 survivors against the exact (Fraction) strict-interior definition,
    against the conservativeness invariant, and against the area closed form
    E[m1/n] = 1 - area(quad)/area(disk) on the uniform disk;
  * Step 4 order by exact rational adjacent-pair comparisons and a
    permutation check;
  * Step 7 (Figure 2) against the constructed example of Section 2.2.1
    (the paper's coordinates are in a lost figure: parity unpinned, the
    relations the text states are checked), against the record
    characterisation of the single-walk filter (a point survives exactly when
    it is not strictly inside the triangle of P_0, P_l and any earlier point),
    and against the subset-containment and conservativeness invariants;
  * the whole model against the monotone-chain oracle and brute force.
"""
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from tests.exact_ref import brute_hull, orient_q


def _inputs():
    out = {
        "square_5k": synth.square(5000, (31, 1)),
        "disk_5k": synth.disk(5000, (32, 1)),
        "gauss_5k": synth.gaussian(5000, 1.0, (33, 1)),
        "grid_20x3": synth.grid(20, 3, (34, 1)),
        "gridraw_3k": synth.grid_draws(3000, 16, (35, 1)),
        "annulus_ngon": synth.annulus_ngon(1500, 1500, 10, ((36, 1), (37, 1), (38, 1))),
        "mixture_5k": synth.mixture(5000, (39, 1)),
    }
    t = np.arange(-40, 41, dtype=np.float64)
    out["collinear"] = np.stack([t, -2 * t + 3], axis=1)[np.random.default_rng(0).permutation(81)]
    out["ray_dups"] = np.concatenate([np.stack([t % 7, t % 7], axis=1), [[0.0, 0.0]] * 5])
    out["single"] = np.array([[0.25, 0.5]] * 4)
    return out


INPUTS = _inputs()


@pytest.mark.parametrize("name", sorted(INPUTS))
@pytest.mark.parametrize("chunk", [0, -1, 1, 7])
def test_model_hull_equals_oracle(name, chunk):
    pts = INPUTS[name]
    m = oracle.model(pts, chunk)
    assert m["hull"].tolist() == oracle.hull(pts).tolist()


@pytest.mark.parametrize("seed", range(25))
def test_model_hull_brute_force_tiny(seed):
    rng = random.Random(1000 + seed)
    n = rng.randint(1, 18)
    if seed % 2:
        pts = [(float(rng.randint(0, 4)), float(rng.randint(0, 4))) for _ in range(n)]
    else:
        pts = [(rng.random(), rng.random()) for _ in range(n)]
    for chunk in (0, -1, 1, 2):
        assert oracle.model(pts, chunk)["hull"].tolist() == brute_hull(pts)


@pytest.mark.parametrize("name", sorted(INPUTS))
def test_extremes_tie_rules(name):
    pts = INPUTS[name]
    x, y = pts[:, 0], pts[:, 1]
    idx = np.arange(len(pts))
    want = [
        int(np.lexsort((idx, -y, x))[0]),    # min x, then max y, then min index
        int(np.lexsort((idx, x, y))[0]),     # min y, then min x
        int(np.lexsort((idx, y, -x))[0]),    # max x, then min y
        int(np.lexsort((idx, -x, -y))[0]),   # max y, then max x
    ]
    assert oracle.model(pts)["extremes"] == want


@pytest.mark.parametrize("name", ["square_5k", "disk_5k", "grid_20x3", "collinear", "mixture_5k"])
def test_round1_is_strict_interior_of_distinct_corners(name):
    pts = INPUTS[name]
    m = oracle.model(pts)
    corners = []
    for e in m["extremes"]:
        c = (float(pts[e, 0]), float(pts[e, 1]))
        if c not in corners:
            corners.append(c)
    assert m["n_corners"] == len(corners)
    for i, p in enumerate(pts):
        inside = len(corners) >= 3 and all(
            orient_q(corners[j], corners[(j + 1) % len(corners)], p) > 0
            for j in range(len(corners)))
        assert m["round1_keep"][i] == (not inside)


@pytest.mark.parametrize("name", sorted(INPUTS))
@pytest.mark.parametrize("chunk", [0, -1, 3])
def test_filters_are_conservative(name, chunk):
    """No canonical vertex (at its smallest index) is discarded by either round."""
    pts = INPUTS[name]
    m = oracle.model(pts, chunk)
    hull = oracle.hull(pts)
    keep1 = m["round1_keep"]
    r2 = set(m["round2"].tolist())
    for v in hull:
        assert keep1[v]
        assert v in r2


def _shoelace(poly):
    s = Fraction(0)
    for i in range(len(poly)):
        x0, y0 = map(Fraction, poly[i])
        x1, y1 = map(Fraction, poly[(i + 1) % len(poly)])
        s += x0 * y1 - x1 * y0
    return float(s / 2)


def test_round1_fraction_matches_area_closed_form():
    pts = synth.disk(200_000, (40, 1))
    m = oracle.model(pts)
    quad = [tuple(pts[e]) for e in m["extremes"]]
    expect = 1.0 - _shoelace(quad) / np.pi
    got = m["m1"] / len(pts)
    assert abs(got - expect) < 0.006, (got, expect)
    assert abs(got - (1 - 2 / np.pi)) < 0.02


def _angle_before(p0, a, b):
    """Exact Step-4 comparison: angle, then distance along the ray, then index."""
    o = orient_q(p0, a[:2], b[:2])
    if o != 0:
        return o > 0
    return (a[1], a[0], a[2]) < (b[1], b[0], b[2])


@pytest.mark.parametrize("name", sorted(INPUTS))
def test_sorted_order_exact(name):
    pts = INPUTS[name]
    m = oracle.model(pts)
    p0 = tuple(pts[m["pivot"]])
    s = m["sorted"]
    want = [i for i in range(len(pts)) if m["round1_keep"][i] and tuple(pts[i]) != p0]
    assert sorted(s.tolist()) == want
    for a, b in zip(s[:-1], s[1:]):
        A = (pts[a, 0], pts[a, 1], a)
        B = (pts[b, 0], pts[b, 1], b)
        assert _angle_before(p0, A, B)


@pytest.mark.parametrize("name", sorted(INPUTS))
def test_longest_and_split(name):
    pts = INPUTS[name]
    m = oracle.model(pts)
    s = m["sorted"]
    if len(s) == 0:
        assert m["longest"] == -1
        return
    p0 = pts[m["pivot"]]
    d = pts[s] - p0
    d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]
    best = s[d2 == d2.max()].min()
    assert m["longest"] == best
    assert s[m["l"] - 1] == best


def test_section_2_2_example_relations():
    """Constructed 15-point instance of Figure 1(b): P_0 at the bottom, 14
    sorted points, l = 8.  The text states that P4 is decided by the line
    P3 -> P8 alone and P11 by the line P12 -> P8 alone; both are interior."""
    q = np.array([
        (0, 0),                                         # P0
        (60, 5), (60, 20), (55, 40), (20, 20), (40, 60), (25, 70), (10, 80),   # P1..P7
        (0, 100),                                       # P8 = P_longest
        (-10, 80), (-30, 65), (-20, 30), (-55, 45), (-60, 20), (-65, 3),        # P9..P14
    ], dtype=np.float64)
    keep = oracle.round2(q, 8)
    # P3 is the P_temp in force when P4 is tested, and P4 is left of P3 -> P8
    assert keep[3] and not keep[4]
    assert orient_q(q[3], q[8], q[4]) > 0
    # P12 is the P_temp when P11 is tested, and P11 is right of P12 -> P8
    assert keep[12] and not keep[11]
    assert orient_q(q[12], q[8], q[11]) < 0
    assert keep[0] and keep[8] and keep[14]


def _sorted_sequence(pts):
    """P_0 plus the other distinct... all points in exact Step-4 order (test side)."""
    import functools
    idx = list(range(len(pts)))
    p0i = min(idx, key=lambda i: (pts[i][1], pts[i][0], i))
    p0 = tuple(pts[p0i])
    rest = [i for i in idx if tuple(pts[i]) != p0]

    def cmp(a, b):
        A = (pts[a][0], pts[a][1], a)
        B = (pts[b][0], pts[b][1], b)
        return -1 if _angle_before(p0, A, B) else 1
    rest.sort(key=functools.cmp_to_key(cmp))
    return [p0i] + rest


@pytest.mark.parametrize("seed", range(30))
def test_single_walk_is_record_filter(seed):
    """With one walk per region, P_i (right region) survives exactly when it is
    not strictly left of X -> P_l for any earlier X in [P_0, P_i) -- i.e. when
    it is a running extreme of the direction from P_l.  Mirror image for the
    left region, walked from the end.  Checked by brute force over all pairs."""
    rng = random.Random(seed)
    n = rng.randint(3, 60)
    if seed % 3 == 0:
        pts = [(float(rng.randint(0, 6)), float(rng.randint(0, 6))) for _ in range(n)]
    else:
        pts = [(rng.random(), rng.random()) for _ in range(n)]
    order = _sorted_sequence(pts)
    q = np.array([pts[i] for i in order], dtype=np.float64)
    N = len(q)
    if N < 2:
        return
    p0 = q[0]
    d2 = [((x - p0[0]) ** 2 + (y - p0[1]) ** 2) for x, y in q]
    l = max(range(1, N), key=lambda i: (Fraction(float(q[i][0]) - float(p0[0])) ** 2 +
                                       Fraction(float(q[i][1]) - float(p0[1])) ** 2, -order[i]))
    keep = oracle.round2(q, l, 0)
    for i in range(1, l):
        interior = any(orient_q(q[t], q[l], q[i]) > 0 for t in range(0, i))
        assert keep[i] == (not interior)
    for i in range(l + 1, N - 1):
        interior = any(orient_q(q[t], q[l], q[i]) < 0 for t in range(i + 1, N))
        assert keep[i] == (not interior)
    assert keep[0] and keep[l] and keep[N - 1]


@pytest.mark.parametrize("name", ["square_5k", "disk_5k", "annulus_ngon", "mixture_5k"])
def test_subsets_only_add_survivors(name):
    pts = INPUTS[name]
    base = set(oracle.model(pts, 0)["round2"].tolist())
    for chunk in (-1, 2, 5, 64):
        assert base <= set(oracle.model(pts, chunk)["round2"].tolist())
    m1 = oracle.model(pts, 1)
    assert m1["m2"] == len(m1["sorted"]) + 1   # subsets of one point test nothing


# Round 2 on hand-made sequences.  P_0 = (0, 0) and P_l = (0, 1000); every
# other point has small integer coordinates (|x|, |y| <= 10); two points
# that are compared either differ in x or are the same point.  Then
# orient(T, P_l, P) =
# -T.x (P.y - T.y) - (1000 - T.y)(P.x - T.x), whose second term (at least
# 990 in magnitude) outweighs the first (at most 200): P is strictly left of
# T -> P_l exactly when P.x < T.x, strictly right exactly when P.x > T.x.
# So the right region discards P_i when P_i.x < P_temp.x, the left region
# when P_i.x > P_temp.x; a copy of P_temp (orientation 0) is kept.
def _r2_sequence(right_x, left_x):
    q = [(0.0, 0.0)] + [(float(x), 1.0) for x in right_x] + [(0.0, 1000.0)] + \
        [(float(x), 2.0) for x in left_x]
    return np.array(q), 1 + len(right_x)


def test_round2_subsets_hand_worked():
    """Section 3.4's subsets on a hand-worked sequence (positions 1..7 right
    of P_l at 8, positions 9..15 left).  Subsets restart P_temp at their first
    point in walking order, which is kept untested; the right region's first
    subset starts from P_0.  The right region is cut from position 1 upward,
    the left region from the last position downward (its walking order), so
    its last subset, next to P_l, is the short one.  Expected masks worked
    out by hand from the x rule above."""
    rx = [5, 3, 7, 2, 6, 9, 1]
    lx = [4, 8, 2, 6, 3, 9, 5]
    q, l = _r2_sequence(rx, lx)
    assert l == 8 and len(q) == 16
    # one walk per region (Figure 2): right keeps running maxima of x from 0
    # (5, 7, 9); left walks 15 -> 9 from x = 5 keeping running minima (3, 2)
    one = oracle.round2(q, l, 0)
    assert one[1:8].tolist() == [1, 0, 1, 0, 0, 1, 0]
    assert one[9:16].tolist() == [0, 0, 1, 0, 1, 0, 1]
    # subsets of 3.  Right: [1,2,3] from P_0 -> 5 keep, 3 drop, 7 keep;
    # [4,5,6] from x=2 (kept) -> 6 keep, 9 keep; [7] alone (kept).
    # Left, cut from the top: [15,14,13] from x=5 -> 9 drop, 3 keep;
    # [12,11,10] from x=6 (kept) -> 2 keep, 8 drop; [9] alone (kept).
    three = oracle.round2(q, l, 3)
    assert three[1:8].tolist() == [1, 0, 1, 1, 1, 1, 1]
    assert three[9:16].tolist() == [1, 0, 1, 1, 1, 0, 1]
    # cut from the bottom instead, the left region would keep 12 (x=6 after
    # 13's x=3 in subset [14,13,12]) and drop 9: the layout is pinned
    assert three[12] and three[9]
    assert three[0] and three[l]
    # the right region's first subset starts from P_0, so its first point is
    # tested: x = -1 is strictly left of P_0 -> P_l and dropped
    q2, l2 = _r2_sequence([-1, 4, 2, 6], [3])
    # (one walk: 4 keep, 2 drop, 6 keep; subsets of 3: [1,2,3] likewise, [4]
    # alone is kept)
    for c in (0, 3):
        assert oracle.round2(q2, l2, c)[1:l2].tolist() == [0, 1, 0, 1]


def test_round2_paper_subsets_hand_worked():
    """The paper's division: 1024 subsets of ceil(m/1024) points per region.
    With m = 2053 points the subsets hold 3 points; the x pattern (5, 3, 7)
    repeated makes every subset, the first one from P_0 and the others from
    their own first point (x = 5), keep 5, drop 3, keep 7; the last subset
    holds the leftover 2053 - 684*3 = 1 point, kept.  The left region
    mirrors it with the pattern (5, 7, 3) read from the top: each subset
    starts at x = 5 (kept), drops 7, keeps 3 -- and its leftover point, at
    position l + 1, starts a subset of its own."""
    m = 2053
    rx = [(5, 3, 7)[i % 3] for i in range(m)]
    lx = [None] * m
    for k in range(m):                  # k counts from the top (walking order)
        lx[m - 1 - k] = (5, 7, 3)[k % 3]
    q, l = _r2_sequence(rx, lx)
    keep = oracle.round2(q, l, -1)
    right = keep[1:l]
    assert right[:-1].tolist() == [1, 0, 1] * 684 and right[-1]
    left_walk = keep[l + 1:][::-1]     # in walking order, from the top
    assert left_walk[:-1].tolist() == [1, 0, 1] * 684 and left_walk[-1]
    # one walk instead: the right region keeps the first 5 and every copy
    # of the running maximum 7 (684 of them); the left region the first 5
    # and every copy of the running minimum 3 (684)
    one = oracle.round2(q, l, 0)
    assert one[1] and int(one[1:l].sum()) == 685
    assert all(one[1 + i] == (i == 0 or rx[i] == 7) for i in range(m))
    assert int(one[l + 1:].sum()) == 685
