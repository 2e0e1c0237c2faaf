"""Exact rational references for the tests (stdlib ``fractions`` only).

These are independent of both the C oracle and the GPU library: every value
is computed with ``Fraction`` from the definitions, never with floating-point
expansions.
"""
from __future__ import annotations

from fractions import Fraction


def F(v) -> Fraction:
    return Fraction(float(v))


def orient_q(a, b, c) -> int:
    """Sign of (b - a) x (c - a), in exact rational arithmetic."""
    ax, ay, bx, by, cx, cy = (F(a[0]), F(a[1]), F(b[0]), F(b[1]), F(c[0]), F(c[1]))
    d = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)
    return (d > 0) - (d < 0)


def brute_hull(pts) -> list:
    """Canonical hull by O(n^3) edge tests, exact.

    A directed pair (a, b) of distinct values is a hull edge when every other
    value c is strictly left of a->b or on the closed segment [a, b].  The
    vertices are the edge tails; the cycle is followed from the
    lexicographically smallest vertex.  Each vertex is reported by its smallest
    input index.
    """
    first = {}
    for i, p in enumerate(pts):
        key = (float(p[0]), float(p[1]))
        if key not in first:
            first[key] = i
    vals = list(first.keys())
    k = len(vals)
    if k <= 2:
        return [first[v] for v in sorted(vals)]

    def on_segment(a, b, c):
        return (min(a[0], b[0]) <= c[0] <= max(a[0], b[0]) and
                min(a[1], b[1]) <= c[1] <= max(a[1], b[1]))

    nxt = {}
    for a in vals:
        for b in vals:
            if a == b:
                continue
            ok = True
            for c in vals:
                if c == a or c == b:
                    continue
                o = orient_q(a, b, c)
                if o < 0 or (o == 0 and not on_segment(a, b, c)):
                    ok = False
                    break
            if ok:
                nxt[a] = b
    if not nxt:   # all values collinear
        return [first[min(vals)], first[max(vals)]]
    start = min(nxt.keys())
    out = [start]
    cur = nxt[start]
    while cur != start:
        out.append(cur)
        cur = nxt[cur]
        if len(out) > k:
            raise AssertionError("edge cycle does not close")
    return [first[v] for v in out]
