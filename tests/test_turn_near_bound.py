"""A float32 model of turn_key_near (the bucket-maxima direction key of the
batched form's tiled engine) against the exact key in rational arithmetic.

The batched form drops a survivor only when its key plus kTurnSlack (4096)
stays below the largest key of an earlier bucket; that is safe when every
key is within kTurnSlack / 2 of the exact one.  The device code documents a
bound of kTurnSlack / 8 (512); this model (numpy float32 with a correctly
rounded division, where the device's fast division may be 2 ulp off) must
stay well inside it, on random directions, directions near the axes and the
quadrant diagonals, and coordinates from 2^-300 to 2^300."""
import math
import random
from fractions import Fraction

import numpy as np

SLACK = 4096


def turn_q(px, py, cx, cy) -> int:
    dx = Fraction(px) - Fraction(cx)
    dy = Fraction(py) - Fraction(cy)
    if dx > 0 and dy >= 0:
        q, a, b = 0, dx, dy
    elif dx <= 0 and dy > 0:
        q, a, b = 1, dy, -dx
    elif dx < 0 and dy <= 0:
        q, a, b = 2, -dx, -dy
    else:
        q, a, b = 3, -dy, dx
    return q * 2 ** 30 + math.floor(b / (a + b) * 2 ** 30)


def turn_near_model(px, py, cx, cy) -> int:
    dx, dy = px - cx, py - cy  # float64 differences, as on the device
    if dx > 0 and dy >= 0:
        q, a, b = 0, dx, dy
    elif dx <= 0 and dy > 0:
        q, a, b = 1, dy, -dx
    elif dx < 0 and dy <= 0:
        q, a, b = 2, -dx, -dy
    else:
        q, a, b = 3, -dy, dx
    e = math.frexp(max(a, b))[1]
    af = np.float32(math.ldexp(a, -e))
    bf = np.float32(math.ldexp(b, -e))
    t = np.float32(bf / np.float32(af + bf)) * np.float32(2.0 ** 30)
    k = 2 ** 30 if t >= np.float32(2.0 ** 30) else int(t)
    return q * 2 ** 30 + k


def _cases():
    rng = random.Random(41)
    for _ in range(3000):
        cx, cy = rng.uniform(-1, 1), rng.uniform(-1, 1)
        yield rng.uniform(-2, 2), rng.uniform(-2, 2), cx, cy
    for _ in range(1500):
        s = math.ldexp(1.0, rng.choice([-300, -150, 0, 150, 299]))
        cx, cy = rng.uniform(-1, 1) * s, rng.uniform(-1, 1) * s
        ang = rng.choice([0.0, math.pi / 4, math.pi / 2, math.pi, 1.5 * math.pi]) + rng.uniform(-1e-9, 1e-9)
        r = rng.uniform(1e-6, 1.0) * s
        yield cx + r * math.cos(ang), cy + r * math.sin(ang), cx, cy
    for _ in range(500):
        # one coordinate difference far below the other
        cx, cy = 0.0, 0.0
        yield rng.choice([1.0, -1.0]) * math.ldexp(1.0, 200), rng.uniform(-1, 1) * math.ldexp(1.0, -200), cx, cy


def test_turn_key_near_within_bound():
    worst = 0
    for px, py, cx, cy in _cases():
        if px == cx and py == cy:
            continue
        d = abs(turn_near_model(px, py, cx, cy) - turn_q(px, py, cx, cy))
        worst = max(worst, d)
    assert worst <= SLACK // 16, worst


def test_slack_covers_the_bound():
    # a dropped point has model key + SLACK < model key of an earlier one;
    # with both within SLACK / 8 of the exact keys, the exact keys differ
    assert SLACK - 2 * (SLACK // 8) > 0
