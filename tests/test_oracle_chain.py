"""Pins of the oracle of the four-region variant (Section 5.1, Table 8).

Each part is checked against something other than itself:
  * the final hull against the monotone-chain oracle and O(n^3) brute force;
  * the first round against the gScan model's (the same Steps 1-2);
  * the region of every survivor against exact rational orientations of the
    quadrilateral's edges;
  * each region's kept points against the plain definition by brute force:
    no other point of the region lies at least as far towards the region's
    corner on both axes (a copy with a smaller index counts), in walking
    order (u rising, v falling);
  * closed forms: a full integer grid keeps only its four corners, the
    vertices of a regular polygon are all kept;
  * a 90-degree rotation of the input moves every region to the next one
    and keeps the same points in the same order;
  * a hand-worked example.
"""
import random

import numpy as np
import pytest

import oracle
import synth
from tests.exact_ref import brute_hull, orient_q


def _uv(k, x, y):
    return [(x, y), (y, -x), (-x, -y), (-y, x)][k]


def _inputs():
    t = np.arange(-30, 31, dtype=np.float64)
    rng = np.random.default_rng(5)
    return {
        "square_5k": synth.square(5000, (61, 1)),
        "disk_5k": synth.disk(5000, (62, 1)),
        "gauss_5k": synth.gaussian(5000, 1.0, (63, 1)),
        "mixture_5k": synth.mixture(5000, (64, 1)),
        "annulus_ngon": synth.annulus_ngon(1500, 1500, 10, ((65, 1), (66, 1), (67, 1))),
        "grid_20x3": synth.grid(20, 3, (68, 1)),
        "gridraw_3k": synth.grid_draws(3000, 16, (69, 1)),
        "int_dups": rng.integers(-6, 7, size=(400, 2)).astype(np.float64),
        "collinear": np.stack([t, -2 * t + 3], axis=1)[rng.permutation(61)],
        "vertical": np.stack([np.zeros(61), t], axis=1)[rng.permutation(61)],
        "horizontal": np.stack([t, np.full(61, 2.0)], axis=1)[rng.permutation(61)],
        "single": np.array([[0.25, 0.5]] * 4),
        "two": np.array([[1.0, 2.0], [3.0, -1.0]]),
        "three": np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]),
    }


INPUTS = _inputs()


@pytest.mark.parametrize("name", sorted(INPUTS))
def test_chain_hull_equals_oracle(name):
    pts = INPUTS[name]
    c = oracle.chain(pts)
    assert c["hull"].tolist() == oracle.hull(pts).tolist()


@pytest.mark.parametrize("seed", range(25))
def test_chain_brute_force_tiny(seed):
    rng = random.Random(seed)
    n = rng.randint(1, 40)
    if seed % 2:
        pts = np.array([(rng.randint(0, 5), rng.randint(0, 5)) for _ in range(n)], dtype=np.float64)
    else:
        pts = np.array([(rng.random(), rng.random()) for _ in range(n)])
    c = oracle.chain(pts)
    assert c["hull"].tolist() == brute_hull(pts)


@pytest.mark.parametrize("name", sorted(INPUTS))
def test_chain_first_round_and_regions(name):
    pts = INPUTS[name]
    c = oracle.chain(pts)
    m = oracle.model(pts)
    assert c["extremes"] == m["extremes"]
    survived = c["region"] >= 0
    assert np.array_equal(survived, m["round1_keep"])
    assert c["m1"] == m["m1"]
    corners = [pts[i] for i in c["extremes"]]
    for i in np.flatnonzero(survived):
        want = 4
        for k in range(4):
            if orient_q(corners[k], corners[(k + 1) % 4], pts[i]) < 0:
                want = k
                break
        assert c["region"][i] == want, (i, want)
    assert [int((c["region"] == k).sum()) for k in range(4)] == c["n_region"]


def _kept_by_definition(pts, region, k):
    """Region k's points that no other point of the region dominates: q
    dominates p when q.u <= p.u and q.v <= p.v and q differs from p or is a
    copy with a smaller index.  Returned in walking order (u ascending)."""
    members = [i for i in range(len(pts)) if region[i] == k]
    uv = {i: _uv(k, float(pts[i][0]), float(pts[i][1])) for i in members}
    kept = []
    for p in members:
        pu, pv = uv[p]
        dominated = False
        for q in members:
            if q == p:
                continue
            qu, qv = uv[q]
            if qu <= pu and qv <= pv and ((qu, qv) != (pu, pv) or q < p):
                dominated = True
                break
        if not dominated:
            kept.append(p)
    return sorted(kept, key=lambda i: uv[i])


@pytest.mark.parametrize("name", ["square_5k", "disk_5k", "gauss_5k", "annulus_ngon", "int_dups",
                                  "gridraw_3k", "mixture_5k"])
def test_chain_round2_is_the_dominance_definition(name):
    pts = INPUTS[name]
    if len(pts) > 3000:
        pts = pts[:3000]
    c = oracle.chain(pts)
    for k in range(4):
        want = _kept_by_definition(pts, c["region"], k)
        assert c["kept"][k].tolist() == want, k
        # walking order: u strictly rising, v strictly falling
        uv = [_uv(k, float(pts[i][0]), float(pts[i][1])) for i in c["kept"][k]]
        assert all(a[0] < b[0] and a[1] > b[1] for a, b in zip(uv, uv[1:]))
    distinct = {tuple(pts[i]) for i in c["extremes"]}
    assert c["m2"] == sum(len(k) for k in c["kept"]) + len(distinct)


@pytest.mark.parametrize("name", sorted(INPUTS))
def test_chain_keeps_every_hull_vertex(name):
    pts = INPUTS[name]
    c = oracle.chain(pts)
    kept = set(np.concatenate(c["kept"]).tolist()) | set(c["extremes"])
    assert set(oracle.hull(pts).tolist()) <= kept


def test_chain_closed_forms():
    g = synth.grid(50, 4, (70, 1))               # full 50 x 50 grid, every cell 4 times
    c = oracle.chain(g)
    assert c["n_region"] == [0, 0, 0, 0] and c["m2"] == 4
    k = 10
    t = 2 * np.pi * np.arange(2 ** k) / 2 ** k
    ring = np.stack([np.cos(t), np.sin(t)], axis=1)[np.random.default_rng(1).permutation(2 ** k)]
    c = oracle.chain(ring)
    assert c["m2"] == 2 ** k                      # every vertex reaches the final stage
    assert len(c["hull"]) == 2 ** k


@pytest.mark.parametrize("name", ["square_5k", "disk_5k", "mixture_5k", "annulus_ngon", "int_dups"])
def test_chain_rotation_moves_regions(name):
    """(x, y) -> (-y, x) is exact and turns P_minx, P_miny, P_maxx, P_maxy
    into P_miny', P_maxx', P_maxy', P_minx' (the tie rules rotate with the
    points), so region k becomes region k+1 with the same (u, v)."""
    pts = INPUTS[name]
    rot = np.stack([-pts[:, 1], pts[:, 0]], axis=1)
    a, b = oracle.chain(pts), oracle.chain(rot)
    assert b["extremes"] == [a["extremes"][3], a["extremes"][0], a["extremes"][1], a["extremes"][2]]
    for k in range(4):
        assert b["kept"][(k + 1) % 4].tolist() == a["kept"][k].tolist()


def test_chain_hand_worked():
    """Ten points.  Extremes: P_minx = (0, 5) (min x, the higher of the two
    at x = 0), P_miny = (4, 0), P_maxx = (10, 3), P_maxy = (6, 9).  Region 0
    (below the edge (0,5) -> (4,0)): (0, 2), (1, 1), (2, 2), (1, 3).  Walking
    by x: (0,2) keep (v=2), (1,1) keep (1 < 2), (1,3) drop, (2,2) drop.
    Region 1 (beyond (4,0) -> (10,3)): (8, 0.5) keep.  Region 2 (beyond
    (10,3) -> (6,9)): (9, 7) keep.  Region 3: none.  (5, 5) is inside."""
    pts = np.array([[0, 5], [4, 0], [10, 3], [6, 9], [0, 2], [1, 1], [2, 2], [1, 3],
                    [8, 0.5], [9, 7], [5, 5]], dtype=np.float64)
    c = oracle.chain(pts)
    assert c["extremes"] == [0, 1, 2, 3]
    assert c["region"].tolist() == [4, 4, 4, 4, 0, 0, 0, 0, 1, 2, -1]
    assert [k.tolist() for k in c["kept"]] == [[4, 5], [8], [9], []]
    assert c["hull"].tolist() == oracle.hull(pts).tolist()
    assert c["hull"].tolist() == [4, 5, 1, 8, 2, 9, 3, 0]
