// steps.hpp - per-point pieces of Steps 1-3 and 5-7 shared by the
// single-hull kernels and the batched kernel.
#pragma once

#include <float.h>

#include "common.hpp"
#include "exact.hpp"

namespace hx {

// ---------------------------------------------------------------------------
// Step 1
// ---------------------------------------------------------------------------
// Strict total orders of the four extreme criteria (ties: P_minx -> larger y,
// P_miny -> smaller x, P_maxx -> smaller y, P_maxy -> larger x, then smaller
// index), so every reduction order returns the same candidates.
//
// These comparisons and the selections that use them are written with
// bitwise operators and explicit per-field selects: with short-circuit
// conditions guarding a whole-struct copy, the gfx950 code generator of this
// toolchain kept the old index on the tie path (wrong Step-1 corners on
// grid inputs).  Straight-line code avoids that shape.
template <int C>
__device__ inline bool better(const Cand& a, const Cand& b) {
    const double a1 = (C == 0 || C == 2) ? a.x : a.y, b1 = (C == 0 || C == 2) ? b.x : b.y;
    const double a2 = (C == 0 || C == 2) ? a.y : a.x, b2 = (C == 0 || C == 2) ? b.y : b.x;
    // primary: smaller for P_minx / P_miny, larger for P_maxx / P_maxy;
    // secondary: larger for P_minx / P_maxy, smaller for P_miny / P_maxx
    const bool p_win = (C <= 1) ? (a1 < b1) : (a1 > b1);
    const bool s_win = (C == 0 || C == 3) ? (a2 > b2) : (a2 < b2);
    const bool p_eq = a1 == b1, s_eq = a2 == b2, i_win = a.i < b.i;
    return p_win | (p_eq & (s_win | (s_eq & i_win)));
}

__device__ inline Cand sentinel(int c) {
    Cand s;
    s.i = INT32_MAX;
    s.pad = 0;
    s.x = (c == 0 || c == 1) ? INFINITY : -INFINITY;
    s.y = (c == 1 || c == 2) ? INFINITY : -INFINITY;
    return s;
}

__device__ inline Cand shfl_xor_cand(const Cand& c, int m) {
    Cand r;
    r.x = __shfl_xor(c.x, m);
    r.y = __shfl_xor(c.y, m);
    r.i = __shfl_xor(c.i, m);
    r.pad = 0;
    return r;
}

template <int C>
__device__ inline void take_better(Cand& c, const Cand& o) {
    const bool t = better<C>(o, c);
    c.x = t ? o.x : c.x;
    c.y = t ? o.y : c.y;
    c.i = t ? o.i : c.i;
}

__device__ inline void reduce4_wave(Cand (&c)[4]) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        take_better<0>(c[0], shfl_xor_cand(c[0], m));
        take_better<1>(c[1], shfl_xor_cand(c[1], m));
        take_better<2>(c[2], shfl_xor_cand(c[2], m));
        take_better<3>(c[3], shfl_xor_cand(c[3], m));
    }
}

// Input domain from the exponent bits alone (integer operations): NaN and
// infinity have the all-ones exponent; 0 < |v| < 2^-300 has a biased
// exponent below 723 (subnormals included); |v| > 2^300 has exponent 1324 or
// more, or exponent 1323 with a non-zero mantissa.
__device__ inline uint32_t domain_flags(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v) & 0x7FFFFFFFFFFFFFFFull;
    const uint32_t hi = (uint32_t)(b >> 32);
    const uint32_t e = hi >> 20;
    const bool nonfinite = e == 0x7FFu;
    const bool tiny = (b != 0) & (e < 723u);
    const bool huge = (b > 0x52B0000000000000ull) & !nonfinite;  // 2^300 = 0x52B0000000000000
    return (nonfinite ? kFlagNonfinite : 0u) | ((tiny | huge) ? kFlagRange : 0u);
}

__device__ inline void offer(Cand (&c)[4], double x, double y, int32_t i) {
    Cand p;
    p.x = x;
    p.y = y;
    p.i = i;
    p.pad = 0;
    take_better<0>(c[0], p);
    take_better<1>(c[1], p);
    take_better<2>(c[2], p);
    take_better<3>(c[3], p);
}

// The quadrilateral of Step 2 and the pivot from the four extreme points:
// distinct corners in the order P_minx -> P_miny -> P_maxx -> P_maxy
// (counter-clockwise), their edge vectors and one error bound for every edge
// test.  Step-5 fields start empty.
__device__ inline void make_params(Params& P, const Cand (&e)[4], uint32_t flags) {
    for (int k = 0; k < 4; ++k) {
        P.ext[k] = e[k];
        P.ext[k].pad = 0;
    }
    int nc = 0;
    for (int k = 0; k < 4; ++k) {
        bool dup = false;
        for (int j = 0; j < nc; ++j) dup |= (P.qx[j] == e[k].x && P.qy[j] == e[k].y);
        if (!dup) {
            P.qx[nc] = e[k].x;
            P.qy[nc] = e[k].y;
            ++nc;
        }
    }
    for (int j = nc; j < 4; ++j) {
        P.qx[j] = P.qx[0];
        P.qy[j] = P.qy[0];
    }
    for (int j = 0; j < 4; ++j) {
        int j1 = (j + 1) % (nc > 0 ? nc : 1);
        P.ex[j] = P.qx[j1] - P.qx[j];
        P.ey[j] = P.qy[j1] - P.qy[j];
    }
    // Every point and corner lies in the bounding box W x H, so for an edge
    // test ex*dy - ey*dx (four rounded differences, two rounded products, one
    // rounded difference) |ex dy| + |ey dx| <= 2WH and the rounding error is
    // below 4.01 eps * 2WH; 9 eps W H also covers the rounding of W and H.
    double W = e[2].x - e[0].x, H = e[3].y - e[1].y;
    P.qbound = 9.0 * kEps * W * H;
    P.ncorner = nc;
    P.x0 = e[1].x;
    P.y0 = e[1].y;
    P.p0_idx = e[1].i;
    P.flags = flags;
    P.pad = 0;
    P.lx = P.x0;
    P.ly = P.y0;
    P.l_idx = -1;
    P.kl = 0;
    P.turn_u = P.turn_v = 0;
    P.pad2[0] = P.pad2[1] = 0;
}

// ---------------------------------------------------------------------------
// Step 2: strictly inside the quadrilateral (strictly left of every edge of
// the distinct corners; fewer than 3 distinct corners: never).  The float64
// edge test is decided by the common bound qbound, else exactly.
// ---------------------------------------------------------------------------
__device__ inline bool quad_inside(const double (&qx)[4], const double (&qy)[4],
                                   const double (&ex)[4], const double (&ey)[4], double qb,
                                   int nc, double px, double py) {
    bool inside = nc >= 3;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (inside && j < nc) {
            double dx = px - qx[j], dy = py - qy[j];
            double l = ex[j] * dy;
            double r = ey[j] * dx;
            double det = l - r;
            int o = det > qb ? 1 : (-det > qb ? -1 : 0);
            if (o == 0) {
                int j1 = (j + 1) % nc;
                o = orient(qx[j], qy[j], qx[j1], qy[j1], px, py);
            }
            inside = o > 0;
        }
    }
    return inside;
}

// The learned discard polygon (learned-filter variant of Step 2): the exact
// convex hull of the candidate points, strict corners counter-clockwise.
constexpr int kPolyMax = 20;  // four Step-1 extremes + 16 directions
struct Poly {
    int32_t nv;  // corners (fewer than 3: discard nothing)
    int32_t pad;
    double qb;   // error bound of the float64 edge test (as for the quadrilateral)
    double px[kPolyMax], py[kPolyMax], ex[kPolyMax], ey[kPolyMax];
};

// Orientation of (a, b, p) with the float64 fast test against the common
// bound (every segment and point lies in the Step-1 bounding box), else exact.
__device__ inline int poly_orient(double ax, double ay, double bx, double by, double qb, double x,
                                  double y) {
    const double l = (bx - ax) * (y - ay);
    const double r = (by - ay) * (x - ax);
    const double det = l - r;
    if (det > qb) return 1;
    if (-det > qb) return -1;
    return orient(ax, ay, bx, by, x, y);
}

// Strictly inside the polygon (strictly left of every edge), by a binary
// search over the fan of diagonals from corner 0: p must lie strictly inside
// the angle at corner 0, then in the wedge between the diagonals to corners
// j and j+1, and strictly left of the edge j -> j+1.  A point on a diagonal
// strictly before its far end is inside (the diagonal's interior lies in the
// polygon's), which the last test decides as well.
// kOwnBound: every test takes the adaptive orient's own error bound (for
// points outside any known bounding box), not the common bound Q.qb.
template <bool kOwnBound = false>
__device__ inline bool poly_inside(const Poly& Q, double x, double y) {
    const int m = Q.nv;
    if (m < 3) return false;
    const double x0 = Q.px[0], y0 = Q.py[0], qb = Q.qb;
    auto side = [&](double ax, double ay, double bx, double by) {
        return kOwnBound ? orient(ax, ay, bx, by, x, y) : poly_orient(ax, ay, bx, by, qb, x, y);
    };
    if (side(x0, y0, Q.px[1], Q.py[1]) <= 0) return false;
    if (side(x0, y0, Q.px[m - 1], Q.py[m - 1]) >= 0) return false;
    // invariant: p is left of (or on) diagonal lo, strictly right of diagonal hi
    int lo = 1, hi = m - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (side(x0, y0, Q.px[mid], Q.py[mid]) >= 0) lo = mid;
        else hi = mid;
    }
    return side(Q.px[lo], Q.py[lo], Q.px[hi], Q.py[hi]) > 0;
}

// Conservative polygon test for a pre-filter: true only when float64
// arithmetic alone proves p strictly inside (every orientation it relies on
// clears the forward error bound); "cannot tell" counts as not inside, so a
// point it drops is one the exact test drops too.  A wedge chosen wrongly
// next to a diagonal is harmless: a convex polygon's inside points lie left
// of every edge, and points beyond a corner lie right of both its edges.
__device__ inline int sure_side(double ax, double ay, double bx, double by, double x, double y) {
    const double acx = ax - x, bcy = by - y, acy = ay - y, bcx = bx - x;
    const double l = acx * bcy, r = acy * bcx;
    const double det = l - r, bound = kOrientBound * (fabs(l) + fabs(r));
    return det > bound ? 1 : (-det > bound ? -1 : 0);
}
__device__ inline bool poly_surely_inside(const Poly& Q, double x, double y) {
    const int m = Q.nv;
    if (m < 3) return false;
    const double x0 = Q.px[0], y0 = Q.py[0];
    if (sure_side(x0, y0, Q.px[1], Q.py[1], x, y) <= 0) return false;
    if (sure_side(x0, y0, Q.px[m - 1], Q.py[m - 1], x, y) >= 0) return false;
    int lo = 1, hi = m - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sure_side(x0, y0, Q.px[mid], Q.py[mid], x, y) >= 0) lo = mid;
        else hi = mid;
    }
    return sure_side(Q.px[lo], Q.py[lo], Q.px[hi], Q.py[hi], x, y) > 0;
}

// The same test in float32 on coordinates relative to corner 0 (faster; for
// the pre-filter only).  Corners and point enter as float32 differences from
// corner 0, each within a relative 2^-24 (one float64 subtraction, one
// conversion); with M the largest magnitude among them, every difference of
// two of them is off by at most 3.01 u M, every product by 16.04 u M^2, a
// determinant by 40.1 u M^2 (u = 2^-24), so a determinant beyond
// 48 u M^2 has the exact sign.  Magnitudes outside [2^-50, 2^50] (or not
// finite) settle nothing.
struct PolyF {
    int32_t nv;
    float m;                     // largest corner magnitude (relative to corner 0)
    double x0, y0;               // corner 0
    float px[kPolyMax], py[kPolyMax];
};

__device__ inline void make_polyf(const Poly& Q, PolyF& F) {
    F.nv = Q.nv;
    F.x0 = Q.px[0];
    F.y0 = Q.py[0];
    float m = 0.f;
    for (int j = 0; j < kPolyMax; ++j) {
        F.px[j] = j < Q.nv ? (float)(Q.px[j] - Q.px[0]) : 0.f;
        F.py[j] = j < Q.nv ? (float)(Q.py[j] - Q.py[0]) : 0.f;
        m = fmaxf(m, fmaxf(fabsf(F.px[j]), fabsf(F.py[j])));
    }
    F.m = m;
}

__device__ inline int sure_side_f(float ax, float ay, float bx, float by, float x, float y, float bound) {
    const float acx = ax - x, bcy = by - y, acy = ay - y, bcx = bx - x;
    const float det = acx * bcy - acy * bcx;
    return det > bound ? 1 : (-det > bound ? -1 : 0);
}

__device__ inline bool poly_surely_inside_f32(const PolyF& F, double x, double y) {
    const int m = F.nv;
    if (m < 3) return false;
    const float px = (float)(x - F.x0), py = (float)(y - F.y0);
    const float M = fmaxf(F.m, fmaxf(fabsf(px), fabsf(py)));
    if (!(M >= 0x1p-50f && M <= 0x1p50f)) return false;
    const float bound = 48.0f * 0x1p-24f * M * M * 1.0001f;
    if (sure_side_f(0.f, 0.f, F.px[1], F.py[1], px, py, bound) <= 0) return false;
    if (sure_side_f(0.f, 0.f, F.px[m - 1], F.py[m - 1], px, py, bound) >= 0) return false;
    int lo = 1, hi = m - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sure_side_f(0.f, 0.f, F.px[mid], F.py[mid], px, py, bound) >= 0) lo = mid;
        else hi = mid;
    }
    return sure_side_f(F.px[lo], F.py[lo], F.px[hi], F.py[hi], px, py, bound) > 0;
}

// The exact convex hull of kC candidate points (s_x, s_y; s_use[j] = 0: no
// point) into Q (px, py, ex, ey, nv; not qb), by every thread of a block of
// at least kC * kC threads; s_use is overwritten.  One thread per ordered
// pair (a, b) of distinct points decides whether a -> b is a
// counter-clockwise hull edge between strict corners: every other point lies
// strictly left of it or on the open segment (a, b).  A strict corner has
// exactly one such successor.  The corners are then placed in the order of
// Andrew's monotone chain, counter-clockwise from the smallest (x, y): a
// corner's position is the number of corners u with orient(start, u, v) > 0
// (strict convexity makes that the angular order around the start).  Fewer
// than three corners give no polygon (nv = 0).
template <int kC>
__device__ inline void hull_of_points(const double* s_x, const double* s_y, int32_t* s_use, Poly& Q) {
    static_assert(kC <= kPolyMax, "corners fit the polygon");
    __shared__ int32_t s_next[kC];
    __shared__ int32_t s_start, s_nv;
    const int t = (int)threadIdx.x;
    // each distinct point once: the first candidate with its coordinates
    int use = 0;
    if (t < kC && s_use[t]) {
        use = 1;
        for (int u = 0; u < t; ++u) use &= !(s_use[u] && s_x[u] == s_x[t] && s_y[u] == s_y[t]);
    }
    if (t == 0) {
        s_start = -1;
        s_nv = 0;
    }
    __syncthreads();
    if (t < kC) {
        s_use[t] = use;
        s_next[t] = -1;
    }
    __syncthreads();
    if (t < kC * kC) {
        const int a = t / kC, b = t % kC;
        if (a != b && s_use[a] && s_use[b]) {
            const double ax = s_x[a], ay = s_y[a], bx = s_x[b], by = s_y[b];
            const double lx = fmin(ax, bx), hx = fmax(ax, bx), ly = fmin(ay, by), hy = fmax(ay, by);
            bool edge = true;
            for (int p = 0; p < kC && edge; ++p) {
                if (p == a || p == b || !s_use[p]) continue;
                const double x = s_x[p], y = s_y[p];
                const int o = orient(ax, ay, bx, by, x, y);
                // collinear with a and b: on the open segment iff inside their box
                edge = o > 0 || (o == 0 && x >= lx && x <= hx && y >= ly && y <= hy);
            }
            if (edge) s_next[a] = b;
        }
    }
    __syncthreads();
    const bool corner = t < kC && s_use[t] && s_next[t] >= 0;
    if (corner) {
        bool least = true;  // the smallest (x, y) of the distinct points
        for (int u = 0; u < kC; ++u)
            least &= !(s_use[u] && (s_x[u] < s_x[t] || (s_x[u] == s_x[t] && s_y[u] < s_y[t])));
        if (least) s_start = t;
        atomicAdd(&s_nv, 1);
    }
    __syncthreads();
    const int start = s_start, nv = s_nv >= 3 && start >= 0 ? s_nv : 0;
    int pos = -1;
    if (corner && nv > 0) {
        pos = 0;
        if (t != start) {
            const double sx = s_x[start], sy = s_y[start];
            pos = 1;
            for (int u = 0; u < kC; ++u)
                if (u != start && u != t && s_use[u] && s_next[u] >= 0)
                    pos += orient(sx, sy, s_x[u], s_y[u], s_x[t], s_y[t]) > 0;
        }
    }
    if (t < kPolyMax && t >= nv) {
        Q.px[t] = 0.0;
        Q.py[t] = 0.0;
        Q.ex[t] = 0.0;
        Q.ey[t] = 0.0;
    }
    if (pos >= 0 && pos < kPolyMax) {
        const int nx = s_next[t];
        Q.px[pos] = s_x[t];
        Q.py[pos] = s_y[t];
        Q.ex[pos] = s_x[nx] - s_x[t];
        Q.ey[pos] = s_y[nx] - s_y[t];
    }
    if (t == 0) {
        Q.pad = 0;
        Q.nv = nv;
        Q.qb = 0.0;
    }
    __syncthreads();
}

// Larger value wins, then the smaller index (extreme point along a direction).
__device__ inline void dir_take(double& bv, int32_t& bi, double v, int32_t i) {
    const bool tk = (v > bv) | ((v == bv) & (i < bi));
    bv = tk ? v : bv;
    bi = tk ? i : bi;
}

// Step 5's distance (a heuristic choice; only needs to be reproducible):
// fl(fl(dx*dx) + fl(dy*dy)) with dx = fl(x - x0), dy = fl(y - y0).
__device__ inline double dist2(double px, double py, double x0, double y0) {
    double dx = px - x0, dy = py - y0;
    double dxx = dx * dx;
    double dyy = dy * dy;
    return dxx + dyy;
}

// ---------------------------------------------------------------------------
// Steps 6-7, bucketed: region and direction key of a round-1 survivor
// ---------------------------------------------------------------------------
struct Cls {
    int region;      // 0 right of P_l, 1 left of P_l, 2 P_l or a copy of it
    uint32_t kappa;  // direction key in the region's order (larger follows)
    uint32_t bucket;
};

// Region by the exact angular order (angle key first, orientation on equal
// keys, distance along the ray on the same ray), then the direction key;
// from the fields it reads (P_0, P_l, its key and both turn keys).
__device__ inline Cls classify_at(double x, double y, uint32_t key, double x0, double y0, double lx,
                                  double ly, uint32_t kl, uint32_t turn_u, uint32_t turn_v) {
    Cls c;
    c.bucket = key >> (32 - kBucketBits);
    c.kappa = 0;
    if (x == lx && y == ly) {
        c.region = 2;
        return c;
    }
    int region;
    if (key < kl) {
        region = 0;
    } else if (key > kl) {
        region = 1;
    } else {
        int o = orient(x0, y0, lx, ly, x, y);
        if (o != 0) region = o < 0 ? 0 : 1;
        else region = (y < ly || (y == ly && x < lx)) ? 0 : 1;
    }
    uint32_t F = turn_key(x, y, lx, ly);
    // right region: counter-clockwise from P_0 - P_l; left region: clockwise
    // from P_l - P_0 (the key is reversed so that larger always follows)
    c.kappa = region == 0 ? F - turn_u : 0xFFFFFFFFu - (F - turn_v);
    c.region = region;
    return c;
}

// A direction key within kTurnSlack / 8 of turn_key(px, py, cx, cy) (p != c):
// the same quadrant rule on the exact signs, then the fraction b / (a + b)
// in float32 after scaling a and b by one power of two (exact), so that
// nothing overflows.  The rounded differences (2^-53), the two conversions,
// the sum and the fast division (2 ulp) leave a relative error below
// 9 * 2^-24 in a fraction below 1, under 600 units of 2^-30; the truncation
// adds one.
constexpr uint32_t kTurnSlack = 4096;
__device__ inline uint32_t turn_key_near(double px, double py, double cx, double cy) {
    const double dx = px - cx, dy = py - cy;
    const bool q0 = (dx > 0.0) & (dy >= 0.0), q1 = (dx <= 0.0) & (dy > 0.0), q2 = (dx < 0.0) & (dy <= 0.0);
    const uint32_t q = q0 ? 0u : q1 ? 1u : q2 ? 2u : 3u;
    const double a = q0 ? dx : q1 ? dy : q2 ? -dx : -dy;
    const double b = q0 ? dy : q1 ? -dx : q2 ? -dy : dx;
    int e;
    (void)frexp(a > b ? a : b, &e);
    const float af = (float)ldexp(a, -e), bf = (float)ldexp(b, -e);
    const float t = __fdividef(bf, af + bf) * 1073741824.0f;
    const uint32_t k = t >= 1073741824.0f ? 1073741824u : (uint32_t)t;
    return (q << 30) + k;
}

// classify_at with the direction key from turn_key_near: the region is
// exact, kappa within kTurnSlack / 8 of classify_at's (the true kappa of
// either region lies in [0, 2^31] or [2^31 - 1, 2^32 - 1]; a difference
// that wrapped below zero is taken as zero).
__device__ inline Cls classify_near(double x, double y, uint32_t key, double x0, double y0, double lx,
                                    double ly, uint32_t kl, uint32_t turn_u, uint32_t turn_v) {
    Cls c;
    c.bucket = key >> (32 - kBucketBits);
    c.kappa = 0;
    if (x == lx && y == ly) {
        c.region = 2;
        return c;
    }
    int region;
    if (key < kl) {
        region = 0;
    } else if (key > kl) {
        region = 1;
    } else {
        int o = orient(x0, y0, lx, ly, x, y);
        if (o != 0) region = o < 0 ? 0 : 1;
        else region = (y < ly || (y == ly && x < lx)) ? 0 : 1;
    }
    const uint32_t F = turn_key_near(x, y, lx, ly);
    uint32_t d = F - (region == 0 ? turn_u : turn_v);
    d = d > 0xC0000000u ? 0u : d;
    c.kappa = region == 0 ? d : 0xFFFFFFFFu - d;
    c.region = region;
    return c;
}

// The same with the fields taken from the call's parameters.
__device__ inline Cls classify(double x, double y, uint32_t key, const Params& P) {
    return classify_at(x, y, key, P.x0, P.y0, P.lx, P.ly, P.kl, P.turn_u, P.turn_v);
}

// Exclusive prefix maxima of one region's bucket maxima in walking order:
// ascending buckets for the right region (starting from kappa(P_0) = 0),
// descending for the left region (identity 0).  Called by all kT threads of
// a workgroup; `in` and `out` may be the same array (every read precedes
// the first barrier, every write follows the last); `s_w` holds kT / 64
// words of LDS.
template <int kT>
__device__ inline void bucket_prefix(const uint32_t* in, uint32_t* out, int region, uint32_t* s_w) {
    constexpr int PER = kBuckets / kT;
    static_assert(kBuckets % kT == 0, "whole buckets per thread");
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    uint32_t v[PER];
    uint32_t tmax = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int w = (int)threadIdx.x * PER + k;  // walking position
        v[k] = in[region == 0 ? w : kBuckets - 1 - w];
        tmax = max(tmax, v[k]);
    }
    uint32_t inc = tmax;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d);
        if (lane >= d) inc = max(inc, o);
    }
    uint32_t ex = __shfl_up(inc, 1);
    if (lane == 0) ex = 0;
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    for (int w = 0; w < wave; ++w) ex = max(ex, s_w[w]);
    __syncthreads();
    uint32_t run = ex;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int w = (int)threadIdx.x * PER + k;
        out[region == 0 ? w : kBuckets - 1 - w] = run;
        run = max(run, v[k]);
    }
}

}  // namespace hx
