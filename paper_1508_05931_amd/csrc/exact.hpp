// exact.hpp - exact geometric predicates for host and device (gfx950).
//
// Every geometric decision of the hull path goes through these functions:
//   orient()     sign of the orientation determinant (Section 2.2.1's
//                "left side of a directed line" test), adaptive: a float64
//                determinant with a forward error bound, and an exact
//                expansion when the bound cannot decide;
//   angle_key()  the exact 32-bit pseudo-angle key used to sort by angle
//                (Section 3.3), with an exact boundary test when the float64
//                estimate is too close to an integer.
//
// Exactness relies on the input domain of the library: coordinates are 0 or
// of magnitude in [2^-300, 2^300], so every difference, product and product
// error term below is a normal double and the error-free transformations are
// exact.  This file must be compiled without floating-point contraction
// (-ffp-contract=off); fma() is written out where it is meant.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace hx {

// unit roundoff of binary64
constexpr double kEps = 1.1102230246251565e-16;  // 2^-53
// Forward error bound of the float64 orientation determinant computed from
// four rounded differences, two rounded products and one rounded difference
// (Shewchuk, "Adaptive Precision Floating-Point Arithmetic and Fast Robust
// Geometric Predicates", 1997: (3 + 16 eps) eps times |left| + |right|).
constexpr double kOrientBound = (3.0 + 16.0 * kEps) * kEps;

// a + b = s + e exactly (branch-free two-sum, Knuth).
__host__ __device__ inline void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    double bv = s - a;
    double av = s - bv;
    e = (a - av) + (b - bv);
}

// a - b = d + e exactly.
__host__ __device__ inline void two_diff(double a, double b, double& d, double& e) {
    d = a - b;
    double bv = a - d;
    double av = d + bv;
    e = (a - av) + (bv - b);
}

// a * b = p + e exactly (fma returns the rounding error of the product).
__host__ __device__ inline void two_prod(double a, double b, double& p, double& e) {
    p = a * b;
    e = fma(a, b, -p);
}

// Exact sign of t[0] + ... + t[N-1].  The terms are folded one at a time into
// a non-overlapping expansion ordered by increasing magnitude (Shewchuk's
// grow-expansion); the largest non-zero component then outweighs the rest, so
// it carries the sign of the exact sum.  Fully unrolled: stays in registers.
template <int N>
__host__ __device__ inline int exact_sign(const double (&t)[N]) {
    double e[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double q = t[k];
#pragma unroll
        for (int i = 0; i < k; ++i) {
            double s, r;
            two_sum(q, e[i], s, r);
            e[i] = r;
            q = s;
        }
        e[k] = q;
    }
    int sign = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if (e[i] > 0.0) sign = 1;
        else if (e[i] < 0.0) sign = -1;
    }
    return sign;
}

// Exact sign of (a - c) x (b - c): the four differences split into exact
// two-term expansions, then the eight partial products into sixteen exact terms.
__host__ __device__ __noinline__ inline int orient_exact(double ax, double ay, double bx, double by,
                                                        double cx, double cy) {
    double p, pe, q, qe, r, re, s, se;
    two_diff(ax, cx, p, pe);  // a.x - c.x
    two_diff(by, cy, q, qe);  // b.y - c.y
    two_diff(ay, cy, r, re);  // a.y - c.y
    two_diff(bx, cx, s, se);  // b.x - c.x
    double t[16];
    two_prod(p, q, t[0], t[1]);
    two_prod(p, qe, t[2], t[3]);
    two_prod(pe, q, t[4], t[5]);
    two_prod(pe, qe, t[6], t[7]);
    two_prod(-r, s, t[8], t[9]);
    two_prod(-r, se, t[10], t[11]);
    two_prod(-re, s, t[12], t[13]);
    two_prod(-re, se, t[14], t[15]);
    return exact_sign<16>(t);
}

// Sign of the orientation of (a, b, c): +1 when a -> b -> c turns
// counter-clockwise (c strictly left of the directed line a -> b), -1 when
// clockwise, 0 when collinear.  Exact.
__host__ __device__ inline int orient(double ax, double ay, double bx, double by, double cx,
                                      double cy) {
    double acx = ax - cx, bcy = by - cy;
    double acy = ay - cy, bcx = bx - cx;
    double l = acx * bcy;
    double r = acy * bcx;
    double det = l - r;
    double bound = kOrientBound * (fabs(l) + fabs(r));
    if (det > bound) return 1;
    if (-det > bound) return -1;
    // A difference of two doubles rounds to zero only when they are equal,
    // so when each product has a zero factor the determinant is exactly
    // zero (repeated points, and the walk's own maximum compared with itself).
    if (((acx == 0.0) | (bcy == 0.0)) & ((acy == 0.0) | (bcx == 0.0))) return 0;
    return orient_exact(ax, ay, bx, by, cx, cy);
}

// Exact test 2^31 * phi(p) >= k for the pseudo-angle of p = (x, y) about the
// pivot (x0, y0), dx = x - x0, dy = y - y0 >= 0:
//   phi = dy / (dx + dy)              for dx >= 0   (0 <= phi <= 1)
//   phi = (2|dx| + dy) / (|dx| + dy)  for dx <  0   (1 <  phi <  2)
// Cleared of the positive denominator the test is linear in the exact
// differences with integer coefficients (exact doubles below 2^33):
//   dx >= 0:  (2^31 - k) dy - k dx            >= 0
//   dx <  0:  (2^32 - k) (x0 - x) + (2^31 - k) dy >= 0
__host__ __device__ __noinline__ inline bool key_at_least(double x, double y, double x0, double y0,
                                                          bool right, double k) {
    double t[8];
    if (right) {
        double a = 2147483648.0 - k;
        two_prod(a, y, t[0], t[1]);
        two_prod(-a, y0, t[2], t[3]);
        two_prod(-k, x, t[4], t[5]);
        two_prod(k, x0, t[6], t[7]);
    } else {
        double b = 4294967296.0 - k;
        double c = 2147483648.0 - k;
        two_prod(b, x0, t[0], t[1]);
        two_prod(-b, x, t[2], t[3]);
        two_prod(c, y, t[4], t[5]);
        two_prod(-c, y0, t[6], t[7]);
    }
    return exact_sign<8>(t) >= 0;
}

// Exact key K(p) = floor(2^31 * phi(p)) in [0, 2^32): strictly increasing
// angle gives non-decreasing keys, and K(a) < K(b) implies that a comes
// strictly before b in angle.  Requires y >= y0, and x > x0 when y == y0.
// The float64 estimate t has absolute error below 2^-19 (a handful of
// roundings, each of relative size 2^-53, on a value below 2^32); when t lies
// within 2^-10 of an integer the exact test above decides.
__host__ __device__ inline uint32_t angle_key(double x, double y, double x0, double y0) {
    double dx = x - x0;  // the signs of the rounded differences are exact
    double dy = y - y0;
    bool right = dx >= 0.0;
    double adx = fabs(dx);
    double s = dy / (adx + dy);
    double t = right ? s * 2147483648.0 : (2.0 - s) * 2147483648.0;
    double f = floor(t);
    double fr = t - f;
    if (fr > 0.0009765625 && fr < 0.9990234375 && f < 4294967296.0) return (uint32_t)f;
    double ks = rint(t);
    if (!(ks > 0.0)) return 0u;  // phi >= 0; also catches NaN
    if (ks >= 4294967296.0) return 4294967295u;  // phi < 2
    return key_at_least(x, y, x0, y0, right, ks) ? (uint32_t)ks : (uint32_t)ks - 1u;
}

// Exact key of the full-turn pseudo-angle of the direction d = p - c (d != 0):
// the quadrant q (exact signs of the rounded differences) and, after rotating d
// by -q quarter turns to (a, b) with a > 0, b >= 0, the fraction t = b/(a+b)
// in [0, 1); key = q*2^30 + floor(2^30 t).  Strictly increasing directions
// (counter-clockwise from the +x axis) give non-decreasing keys, a half turn
// adds exactly 2^31, and the floor is exact: near an integer the test
// (2^30 - k) b - k a >= 0 (a, b exact differences) decides.
__host__ __device__ __noinline__ inline bool turn_at_least(double a1, double a2, double b1, double b2,
                                                           double k) {
    // a = a1 - a2, b = b1 - b2
    double A = 1073741824.0 - k;
    double t[8];
    two_prod(A, b1, t[0], t[1]);
    two_prod(-A, b2, t[2], t[3]);
    two_prod(-k, a1, t[4], t[5]);
    two_prod(k, a2, t[6], t[7]);
    return exact_sign<8>(t) >= 0;
}

__host__ __device__ inline uint32_t turn_key(double px, double py, double cx, double cy) {
    double dx = px - cx, dy = py - cy;
    uint32_t q;
    double a, b, a1, a2, b1, b2;
    if (dx > 0.0 && dy >= 0.0) {
        q = 0; a = dx; b = dy; a1 = px; a2 = cx; b1 = py; b2 = cy;
    } else if (dx <= 0.0 && dy > 0.0) {
        q = 1; a = dy; b = -dx; a1 = py; a2 = cy; b1 = cx; b2 = px;
    } else if (dx < 0.0 && dy <= 0.0) {
        q = 2; a = -dx; b = -dy; a1 = cx; a2 = px; b1 = cy; b2 = py;
    } else {
        q = 3; a = -dy; b = dx; a1 = cy; a2 = py; b1 = px; b2 = cx;
    }
    double t = b / (a + b) * 1073741824.0;
    double f = floor(t);
    double fr = t - f;
    uint32_t k;
    if (fr > 0.0009765625 && fr < 0.9990234375 && f < 1073741824.0) {
        k = (uint32_t)f;
    } else {
        double ks = rint(t);
        if (!(ks > 0.0)) k = 0u;
        else if (ks >= 1073741824.0) k = 1073741823u;
        else k = turn_at_least(a1, a2, b1, b2, ks) ? (uint32_t)ks : (uint32_t)ks - 1u;
    }
    return (q << 30) | k;
}

// Step 4's total order on round-1 survivors (the pivot's copies excluded):
// ascending angle about the pivot, then ascending distance along a common
// ray (larger y is farther; on the horizontal ray larger x), then ascending
// input index.  Returns true when a precedes b.  Exact.
__host__ __device__ inline bool angle_less(double ax, double ay, uint32_t ai, double bx, double by,
                                           uint32_t bi, double x0, double y0) {
    int o = orient(x0, y0, ax, ay, bx, by);
    if (o != 0) return o > 0;
    if (ay != by) return ay < by;
    if (ax != bx) return ax < bx;
    return ai < bi;
}

}  // namespace hx
