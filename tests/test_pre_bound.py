"""The learned pre-filter's float32 orientation bound (no GPU).

The pre-filter drops a point only when float32 arithmetic proves it strictly
inside the direction candidates' polygon: on coordinates relative to corner
0 (one float64 subtraction, one conversion), a determinant beyond
48 u M^2 (u = 2^-24, M the largest magnitude involved) is taken to have the
exact sign.  This reproduces that arithmetic in numpy float32 (round to
nearest, no fused multiply-add, as the kernels are built) on near-degenerate
triples and checks every sign it claims against the oracle's exact
orientation."""
import math

import numpy as np

import oracle


def _claims(a, b, p, c0):
    """Sign the float32 test claims for orient(a, b, p) (0: cannot tell),
    coordinates taken relative to c0 (the polygon's corner 0)."""
    f = np.float32
    ax = f(a[0] - c0[0]); ay = f(a[1] - c0[1])
    bx = f(b[0] - c0[0]); by = f(b[1] - c0[1])
    px = f(p[0] - c0[0]); py = f(p[1] - c0[1])
    M = max(abs(ax), abs(ay), abs(bx), abs(by), abs(px), abs(py))
    if not (2.0 ** -50 <= M <= 2.0 ** 50):
        return 0
    bound = f(f(f(f(48.0) * f(2.0 ** -24)) * M) * M) * f(1.0001)
    acx = f(ax - px); bcy = f(by - py); acy = f(ay - py); bcx = f(bx - px)
    det = f(f(acx * bcy) - f(acy * bcx))
    return 1 if det > bound else (-1 if -det > bound else 0)


def _walk(v, k):
    for _ in range(abs(k)):
        v = math.nextafter(v, math.inf if k > 0 else -math.inf)
    return v


def test_float32_claims_match_exact_orientation():
    rng = np.random.default_rng(7)
    claimed = 0
    for _ in range(20000):
        s = 10.0 ** rng.uniform(-6, 6)
        o = rng.uniform(-1, 1, 2) * s * rng.choice([1.0, 1e3])
        a = o + rng.uniform(-1, 1, 2) * s
        b = o + rng.uniform(-1, 1, 2) * s
        t = rng.uniform(-0.5, 1.5)
        # a point on the line through a and b, moved by a few float32-sized steps
        q = a + t * (b - a)
        eps = float(np.spacing(np.float32(max(abs(q[0]), abs(q[1]), 1e-30)))) * rng.uniform(-64, 64)
        p = (q[0] + eps * rng.uniform(-1, 1), q[1] + eps * rng.uniform(-1, 1))
        p = (_walk(p[0], int(rng.integers(-3, 4))), p[1])
        c0 = tuple(o + rng.uniform(-1, 1, 2) * s * rng.choice([0.0, 1.0, 5.0]))
        c = _claims(tuple(a), tuple(b), p, c0)
        if c != 0:
            claimed += 1
            assert c == oracle.orient(tuple(a), tuple(b), p), (a, b, p)
    assert claimed > 2000  # the test does decide most cases


def test_float32_claims_on_clear_cases():
    rng = np.random.default_rng(8)
    for _ in range(5000):
        a, b, p, c0 = (tuple(rng.uniform(-10, 10, 2)) for _ in range(4))
        c = _claims(a, b, p, c0)
        assert c in (0, oracle.orient(a, b, p))
