/*
 * oracle.c - CPU oracle for the exact 2D hull and the gScan method model.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h): never part of the product path.
 * Compiled with contraction off so every a*b+c rounds twice unless fma() is
 * written out.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Exact arithmetic: error-free transformations and expansions.             */
/* ------------------------------------------------------------------------ */

/* s + e == a + b exactly, |e| <= ulp(s)/2 (Knuth's branch-free two-sum). */
static void two_sum(double a, double b, double* s, double* e) {
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    *e = (a - av) + (b - bv);
    *s = x;
}

/* p + e == a * b exactly (fma gives the rounding error of the product). */
static void two_prod(double a, double b, double* p, double* e) {
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* Adds b to the expansion e[0..m) (non-overlapping, increasing magnitude) in
 * place; the result has m+1 components with the same two properties. */
static int grow(double* e, int m, double b) {
    double q = b;
    for (int i = 0; i < m; ++i) {
        double s, err;
        two_sum(q, e[i], &s, &err);
        e[i] = err;
        q = s;
    }
    e[m] = q;
    return m + 1;
}

/* The largest non-zero component of a non-overlapping expansion outweighs
 * all the others together, so it carries the sign of the exact sum. */
static int expansion_sign(const double* e, int m) {
    for (int i = m - 1; i >= 0; --i)
        if (e[i] != 0.0) return e[i] > 0.0 ? 1 : -1;
    return 0;
}

int oracle_orient(double ax, double ay, double bx, double by, double cx, double cy) {
    /* (b-a) x (c-a) = bx*cy - bx*ay - ax*cy - by*cx + by*ax + ay*cx
     * (the two ax*ay terms of the expansion cancel). */
    const double f[6] = {bx, -bx, -ax, -by, by, ay};
    const double g[6] = {cy, ay, cy, cx, ax, cx};
    double e[12];
    int m = 0;
    for (int k = 0; k < 6; ++k) {
        double p, q;
        two_prod(f[k], g[k], &p, &q);
        m = grow(e, m, q);
        m = grow(e, m, p);
    }
    return expansion_sign(e, m);
}

/* ------------------------------------------------------------------------ */
/* Input domain.                                                            */
/* ------------------------------------------------------------------------ */

int oracle_validate(const double* xy, int64_t n) {
    if (n < 0 || (n > 0 && !xy)) return ORACLE_BADARG;
    if (n > INT32_MAX) return ORACLE_BADARG;
    const double lo = ldexp(1.0, -300), hi = ldexp(1.0, 300);
    int range = 0;
    for (int64_t i = 0; i < 2 * n; ++i) {
        double v = xy[i];
        if (!isfinite(v)) return ORACLE_NONFINITE;
        double a = fabs(v);
        if (a != 0.0 && (a < lo || a > hi)) range = 1;
    }
    return range ? ORACLE_RANGE : ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Canonical hull: Andrew's monotone chain.                                 */
/* ------------------------------------------------------------------------ */

static const double* g_xy;   /* comparator context (the oracle is single-threaded) */

static int cmp_lex(const void* pa, const void* pb) {
    int32_t a = *(const int32_t*)pa, b = *(const int32_t*)pb;
    double ax = g_xy[2 * (int64_t)a], ay = g_xy[2 * (int64_t)a + 1];
    double bx = g_xy[2 * (int64_t)b], by = g_xy[2 * (int64_t)b + 1];
    if (ax != bx) return ax < bx ? -1 : 1;
    if (ay != by) return ay < by ? -1 : 1;
    return (a > b) - (a < b);
}

static int orient_idx(const double* xy, int32_t a, int32_t b, int32_t c) {
    return oracle_orient(xy[2 * (int64_t)a], xy[2 * (int64_t)a + 1],
                         xy[2 * (int64_t)b], xy[2 * (int64_t)b + 1],
                         xy[2 * (int64_t)c], xy[2 * (int64_t)c + 1]);
}

static int same_point(const double* xy, int32_t a, int32_t b) {
    return xy[2 * (int64_t)a] == xy[2 * (int64_t)b] &&
           xy[2 * (int64_t)a + 1] == xy[2 * (int64_t)b + 1];
}

int oracle_hull(const double* xy, int64_t n, int32_t* out, int64_t cap, int64_t* h) {
    int st = oracle_validate(xy, n);
    if (st != ORACLE_OK) return st;
    if (!h || (cap > 0 && !out)) return ORACLE_BADARG;
    *h = 0;
    if (n == 0) return ORACLE_OK;

    int32_t* u = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* chain = (int32_t*)malloc((size_t)(2 * n + 2) * sizeof(int32_t));
    if (!u || !chain) { free(u); free(chain); return ORACLE_NOMEM; }
    for (int64_t i = 0; i < n; ++i) u[i] = (int32_t)i;
    g_xy = xy;
    qsort(u, (size_t)n, sizeof(int32_t), cmp_lex);

    /* Equal coordinates are adjacent; the first of each run has the smallest index. */
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i)
        if (k == 0 || !same_point(xy, u[k - 1], u[i])) u[k++] = u[i];

    int64_t hh = 0;
    if (k <= 2) {
        for (int64_t i = 0; i < k; ++i) chain[hh++] = u[i];
    } else {
        /* lower chain, left to right; a non-left turn pops (drops collinear) */
        for (int64_t i = 0; i < k; ++i) {
            while (hh >= 2 && orient_idx(xy, chain[hh - 2], chain[hh - 1], u[i]) <= 0) --hh;
            chain[hh++] = u[i];
        }
        /* upper chain, right to left, on top of the lower one */
        int64_t base = hh;
        for (int64_t i = k - 2; i >= 0; --i) {
            while (hh > base && orient_idx(xy, chain[hh - 2], chain[hh - 1], u[i]) <= 0) --hh;
            chain[hh++] = u[i];
        }
        --hh;  /* the last point repeats the first */
    }
    *h = hh;
    int st2 = ORACLE_OK;
    if (hh > cap) st2 = ORACLE_CAPACITY;
    else memcpy(out, chain, (size_t)hh * sizeof(int32_t));
    free(u);
    free(chain);
    return st2;
}

/* ------------------------------------------------------------------------ */
/* Method model: the paper's Steps 1-8 (Section 2.1).                        */
/* ------------------------------------------------------------------------ */

static double g_x0, g_y0;    /* pivot for the angular comparator */

/* Step 4's order: ascending angle about the pivot; points on one ray from the
 * pivot by ascending distance (larger y is farther, then larger x on the
 * horizontal ray); equal coordinates by ascending index.  All angles lie in
 * [0, pi) because the pivot is the lowest (then leftmost) point, so the sign
 * of the orientation compares two angles. */
static int cmp_angle(const void* pa, const void* pb) {
    int32_t a = *(const int32_t*)pa, b = *(const int32_t*)pb;
    double ax = g_xy[2 * (int64_t)a], ay = g_xy[2 * (int64_t)a + 1];
    double bx = g_xy[2 * (int64_t)b], by = g_xy[2 * (int64_t)b + 1];
    int o = oracle_orient(g_x0, g_y0, ax, ay, bx, by);
    if (o > 0) return -1;
    if (o < 0) return 1;
    if (ay != by) return ay < by ? -1 : 1;
    if (ax != bx) return ax < bx ? -1 : 1;
    return (a > b) - (a < b);
}

/* Step 1: the four extreme points.  Ties: P_minx takes the largest y,
 * P_miny the smallest x, P_maxx the smallest y, P_maxy the largest x, then
 * the smallest index; each is then a corner of the hull. */
static void extremes(const double* xy, int64_t n, int32_t ext[4]) {
    int32_t a = 0, b = 0, c = 0, d = 0;
    for (int64_t i = 1; i < n; ++i) {
        double x = xy[2 * i], y = xy[2 * i + 1];
        double ax = xy[2 * (int64_t)a], ay = xy[2 * (int64_t)a + 1];
        double bx = xy[2 * (int64_t)b], by = xy[2 * (int64_t)b + 1];
        double cx = xy[2 * (int64_t)c], cy = xy[2 * (int64_t)c + 1];
        double dx = xy[2 * (int64_t)d], dy = xy[2 * (int64_t)d + 1];
        if (x < ax || (x == ax && y > ay)) a = (int32_t)i;
        if (y < by || (y == by && x < bx)) b = (int32_t)i;
        if (x > cx || (x == cx && y < cy)) c = (int32_t)i;
        if (y > dy || (y == dy && x > dx)) d = (int32_t)i;
    }
    ext[0] = a; ext[1] = b; ext[2] = c; ext[3] = d;
}

static int64_t chunk_length(int64_t chunk, int64_t m) {
    if (m < 1) return 1;
    if (chunk == 0) return m;
    if (chunk < 0) return (m + 1023) / 1024;
    return chunk;
}

/* Step 7 (Section 2.2.1, Figure 2) on points already in angular order:
 * q[0] = P_0, q[l] = P_longest.  Right region q[1..l): walk forward from
 * P_temp = P_0; a point strictly left of the directed line P_temp -> P_l is
 * interior, otherwise it becomes P_temp.  Left region q(l..N-1]: walk
 * backward from P_temp = q[N-1]; a point strictly right of P_temp -> P_l is
 * interior.  With subsets (Section 3.4) every subset restarts P_temp at its
 * first point in walking order and keeps that point untested, except the right
 * region's first subset, which starts from P_0 as the figure does.  Subsets
 * are cut in walking order: the right region from q[1] upward, the left
 * region from q[N-1] downward, so each region's short leftover subset is the
 * one next to P_longest. */
int oracle_round2(const double* q, int64_t N, int64_t l, int64_t chunk, uint8_t* keep) {
    if (N < 1 || l < 0 || l >= N || !q || !keep || (l == 0 && N > 1)) return ORACLE_BADARG;
    for (int64_t i = 0; i < N; ++i) keep[i] = 1;
    const double lx = q[2 * l], ly = q[2 * l + 1];
    int64_t mR = l - 1;
    int64_t cR = chunk_length(chunk, mR);
    for (int64_t s = 1; s < l; s += cR) {
        int64_t e = s + cR < l ? s + cR : l;
        int64_t t = 0, i = s;
        if (s != 1) { t = s; i = s + 1; }
        for (; i < e; ++i) {
            if (oracle_orient(q[2 * t], q[2 * t + 1], lx, ly, q[2 * i], q[2 * i + 1]) > 0) keep[i] = 0;
            else t = i;
        }
    }
    int64_t mL = N - 1 - l;
    int64_t cL = chunk_length(chunk, mL);
    for (int64_t top = N - 1; top > l; top -= cL) {
        int64_t bot = top - cL + 1 > l + 1 ? top - cL + 1 : l + 1;
        int64_t t = top;
        for (int64_t i = top - 1; i >= bot; --i) {
            if (oracle_orient(q[2 * t], q[2 * t + 1], lx, ly, q[2 * i], q[2 * i + 1]) < 0) keep[i] = 0;
            else t = i;
        }
    }
    return ORACLE_OK;
}

int oracle_model(const double* xy, int64_t n, int64_t chunk, oracle_model_result* r) {
    int st = oracle_validate(xy, n);
    if (st != ORACLE_OK) return st;
    if (!r || (n > 0 && (!r->round1_keep || !r->sorted || !r->round2 || !r->hull)))
        return ORACLE_BADARG;
    r->n_corners = 0; r->m1 = 0; r->n_sorted = 0; r->l = 0; r->m2 = 0; r->h = 0;
    r->pivot = -1; r->longest = -1;
    for (int k = 0; k < 4; ++k) r->extremes[k] = -1;
    if (n == 0) return ORACLE_OK;

    /* Step 1 */
    extremes(xy, n, r->extremes);

    /* Step 2: the quadrilateral P_minx -> P_miny -> P_maxx -> P_maxy is
     * counter-clockwise; repeated corners are merged, and with fewer than three
     * distinct corners nothing is inside.  A point is discarded only when it is
     * strictly left of every edge (strictly inside). */
    int32_t corner[4];
    int nc = 0;
    for (int k = 0; k < 4; ++k) {
        int dup = 0;
        for (int j = 0; j < nc; ++j) dup |= same_point(xy, corner[j], r->extremes[k]);
        if (!dup) corner[nc++] = r->extremes[k];
    }
    r->n_corners = nc;
    int64_t m1 = 0;
    for (int64_t i = 0; i < n; ++i) {
        int inside = nc >= 3;
        for (int j = 0; j < nc && inside; ++j)
            inside = orient_idx(xy, corner[j], corner[(j + 1) % nc], (int32_t)i) > 0;
        r->round1_keep[i] = (uint8_t)!inside;
        m1 += !inside;
    }
    r->m1 = m1;

    /* Step 3/4: pivot P_0 = P_miny; its copies are not sorted (P_0 stands for them). */
    int32_t p0 = r->extremes[1];
    r->pivot = p0;
    g_x0 = xy[2 * (int64_t)p0];
    g_y0 = xy[2 * (int64_t)p0 + 1];
    int64_t ns = 0;
    for (int64_t i = 0; i < n; ++i)
        if (r->round1_keep[i] && !same_point(xy, (int32_t)i, p0)) r->sorted[ns++] = (int32_t)i;
    r->n_sorted = ns;
    g_xy = xy;
    qsort(r->sorted, (size_t)ns, sizeof(int32_t), cmp_angle);

    /* seq = [P_0, sorted...] */
    int64_t N = ns + 1;
    int32_t* seq = (int32_t*)malloc((size_t)N * sizeof(int32_t));
    uint8_t* keep = (uint8_t*)malloc((size_t)N);
    int32_t* stack = (int32_t*)malloc((size_t)N * sizeof(int32_t));
    double* sxy = (double*)malloc((size_t)N * 2 * sizeof(double));
    if (!seq || !keep || !stack || !sxy) {
        free(seq); free(keep); free(stack); free(sxy);
        return ORACLE_NOMEM;
    }
    seq[0] = p0;
    memcpy(seq + 1, r->sorted, (size_t)ns * sizeof(int32_t));
    memset(keep, 1, (size_t)N);

    if (ns > 0) {
        /* Step 5: longest squared distance from P_0, each operation rounded
         * once; ties go to the smallest index. */
        int32_t best = -1;
        double bestd = -1.0;
        for (int64_t i = 0; i < ns; ++i) {
            int32_t p = r->sorted[i];
            double dx = xy[2 * (int64_t)p] - g_x0;
            double dy = xy[2 * (int64_t)p + 1] - g_y0;
            double dxx = dx * dx;
            double dyy = dy * dy;
            double d2 = dxx + dyy;
            if (d2 > bestd || (d2 == bestd && p < best)) { bestd = d2; best = p; }
        }
        r->longest = best;
        /* Step 6: its position splits the sorted list into the right region
         * [1, l) and the left region (l, N-1]. */
        int64_t l = 0;
        for (int64_t i = 1; i < N; ++i)
            if (seq[i] == best) { l = i; break; }
        r->l = l;

        /* Step 7 on the coordinates in angular order */
        for (int64_t i = 0; i < N; ++i) {
            sxy[2 * i] = xy[2 * (int64_t)seq[i]];
            sxy[2 * i + 1] = xy[2 * (int64_t)seq[i] + 1];
        }
        oracle_round2(sxy, N, l, chunk, keep);
    }
    int64_t m2 = 0;
    for (int64_t i = 0; i < N; ++i)
        if (keep[i]) r->round2[m2++] = seq[i];
    r->m2 = m2;

    /* Step 8: Graham stack scan over the kept points in angular order; a
     * non-left turn pops, a repeat of the top point is skipped. */
    int64_t top = 0;
    for (int64_t i = 0; i < m2; ++i) {
        int32_t p = r->round2[i];
        if (top > 0 && same_point(xy, stack[top - 1], p)) continue;
        while (top >= 2 && orient_idx(xy, stack[top - 2], stack[top - 1], p) <= 0) --top;
        stack[top++] = p;
    }
    /* Canonical form: start at the lexicographically smallest vertex. */
    int64_t start = 0;
    for (int64_t i = 1; i < top; ++i) {
        double x = xy[2 * (int64_t)stack[i]], y = xy[2 * (int64_t)stack[i] + 1];
        double bx = xy[2 * (int64_t)stack[start]], by = xy[2 * (int64_t)stack[start] + 1];
        if (x < bx || (x == bx && y < by)) start = i;
    }
    for (int64_t i = 0; i < top; ++i) r->hull[i] = stack[(start + i) % top];
    r->h = top;
    free(seq);
    free(keep);
    free(stack);
    free(sxy);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Learned-filter variant of the first round (plain definition).            */
/* ------------------------------------------------------------------------ */

/* The network's sample: every point when n <= 4096, else 16 blocks of 256
 * consecutive points, block b starting at floor(b n / 16). */
static int64_t net_sample_size(int64_t n) { return n < 4096 ? n : 4096; }
static int64_t net_sample_point(int64_t s, int64_t n) {
    return n <= 4096 ? s : ((s >> 8) * n) / 16 + (s & 255);
}

int oracle_learned_round1(const double* xy, int64_t n, const double* dirs, int32_t k,
                          uint8_t* keep, int32_t* cand, int64_t* m1) {
    int st = oracle_validate(xy, n);
    if (st != ORACLE_OK) return st;
    if (!keep || !m1 || k < 0 || k > 64 || (k > 0 && !dirs)) return ORACLE_BADARG;
    for (int32_t j = 0; j < 2 * k; ++j)
        if (!(fabs(dirs[j]) <= DBL_MAX)) return ORACLE_BADARG;
    *m1 = 0;
    if (n == 0) return ORACLE_OK;

    /* the four extremes of Step 1, then per direction the farthest sample
     * point (ties: the smallest index; sample indices grow with s) */
    int32_t c[68];
    extremes(xy, n, c);
    const int64_t ns = net_sample_size(n);
    for (int32_t j = 0; j < k; ++j) {
        const double ux = dirs[2 * j], uy = dirs[2 * j + 1];
        int32_t best = -1;
        double bv = 0.0;
        for (int64_t s = 0; s < ns; ++s) {
            const int64_t i = net_sample_point(s, n);
            double v = fma(xy[2 * i], ux, xy[2 * i + 1] * uy);
            if (best < 0 || v > bv) { bv = v; best = (int32_t)i; }
        }
        c[4 + j] = best;
    }
    if (cand) memcpy(cand, c, (size_t)(4 + k) * sizeof(int32_t));

    /* the polygon: the exact convex hull of all the candidates, the four
     * extremes included, so that it contains the quadrilateral */
    const int32_t nc = 4 + k;
    double cxy[2 * 68];
    for (int32_t j = 0; j < nc; ++j) {
        cxy[2 * j] = xy[2 * (int64_t)c[j]];
        cxy[2 * j + 1] = xy[2 * (int64_t)c[j] + 1];
    }
    int32_t hv[68];
    int64_t h = 0;
    st = oracle_hull(cxy, nc, hv, 68, &h);
    if (st != ORACLE_OK) return st;

    /* discarded: strictly inside it (strictly left of every edge; fewer than
     * three corners: never) */
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        int inside = h >= 3;
        for (int64_t e = 0; e < h && inside; ++e) {
            const int32_t a = hv[e], b = hv[(e + 1) % h];
            inside = oracle_orient(cxy[2 * a], cxy[2 * a + 1], cxy[2 * b], cxy[2 * b + 1],
                                   xy[2 * i], xy[2 * i + 1]) > 0;
        }
        keep[i] = inside ? 0 : 1;
        cnt += keep[i];
    }
    *m1 = cnt;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* The four-region variant of Section 5.1 / Table 8 (CudaChain's design, the */
/* paper's comparison method): the same first round, then the survivors go   */
/* to four sub-regions, each sorted by one coordinate, and a second round    */
/* discards by comparing coordinates.                                        */
/* ------------------------------------------------------------------------ */

/* Region k holds the survivors strictly outside edge k of the cycle
 * P_minx -> P_miny -> P_maxx -> P_maxy -> P_minx (the first such edge; a
 * repeated corner makes its edge empty).  In region k the coordinates
 * rotated by -90 degrees k times, (u, v) = (x, y), (y, -x), (-x, -y), (-y, x)
 * (negation is exact), put every region in the lower-left position: its
 * hull chain runs from corner k to corner k+1 with u rising and v falling. */
static void rot_uv(int k, double x, double y, double* u, double* v) {
    switch (k & 3) {
        case 0: *u = x; *v = y; break;
        case 1: *u = y; *v = -x; break;
        case 2: *u = -x; *v = -y; break;
        default: *u = -y; *v = x; break;
    }
}

static int g_region;         /* comparator context: the region being sorted */

/* Sorting of one region: u ascending (R0 by x, R1 by y, R2 by x descending,
 * R3 by y descending), then v ascending, then index. */
static int cmp_region(const void* pa, const void* pb) {
    int32_t a = *(const int32_t*)pa, b = *(const int32_t*)pb;
    double au, av, bu, bv;
    rot_uv(g_region, g_xy[2 * (int64_t)a], g_xy[2 * (int64_t)a + 1], &au, &av);
    rot_uv(g_region, g_xy[2 * (int64_t)b], g_xy[2 * (int64_t)b + 1], &bu, &bv);
    if (au != bu) return au < bu ? -1 : 1;
    if (av != bv) return av < bv ? -1 : 1;
    return (a > b) - (a < b);
}

int oracle_chain(const double* xy, int64_t n, oracle_chain_result* r) {
    int st = oracle_validate(xy, n);
    if (st != ORACLE_OK) return st;
    if (!r || (n > 0 && (!r->region || !r->kept || !r->hull))) return ORACLE_BADARG;
    r->m1 = 0; r->m2 = 0; r->h = 0;
    for (int k = 0; k < 4; ++k) { r->extremes[k] = -1; r->n_region[k] = 0; r->n_kept[k] = 0; }
    if (n == 0) return ORACLE_OK;

    /* first round: Steps 1-2, the same as gScan's */
    int32_t c[4];
    extremes(xy, n, c);
    memcpy(r->extremes, c, sizeof(c));
    int32_t corner[4];
    int nc = 0;
    for (int k = 0; k < 4; ++k) {
        int dup = 0;
        for (int j = 0; j < nc; ++j) dup |= same_point(xy, corner[j], c[k]);
        if (!dup) corner[nc++] = c[k];
    }

    /* distribution into the four sub-regions (-1: discarded by round 1,
     * 4: on the quadrilateral's boundary, not strictly outside any edge) */
    int32_t* lists = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* stack = (int32_t*)malloc((size_t)(n + 8) * sizeof(int32_t));
    if (!lists || !stack) { free(lists); free(stack); return ORACLE_NOMEM; }
    int64_t m1 = 0;
    for (int64_t i = 0; i < n; ++i) {
        int inside = nc >= 3;
        for (int j = 0; j < nc && inside; ++j)
            inside = orient_idx(xy, corner[j], corner[(j + 1) % nc], (int32_t)i) > 0;
        int reg = -1;
        if (!inside) {
            ++m1;
            reg = 4;
            for (int k = 0; k < 4 && reg == 4; ++k)
                if (orient_idx(xy, c[k], c[(k + 1) & 3], (int32_t)i) < 0) reg = k;
        }
        r->region[i] = (int8_t)reg;
    }
    r->m1 = m1;

    /* per region: sort by the region's coordinate, then walk it keeping the
     * running minimum of v; a point is kept only when its v is strictly
     * below every v before it (a point before it with v no larger lies
     * towards the region's corner on both axes, so this one is not a
     * vertex of the region's chain) */
    int64_t nk = 0;
    for (int k = 0; k < 4; ++k) {
        int64_t m = 0;
        for (int64_t i = 0; i < n; ++i)
            if (r->region[i] == k) lists[m++] = (int32_t)i;
        r->n_region[k] = m;
        g_xy = xy;
        g_region = k;
        qsort(lists, (size_t)m, sizeof(int32_t), cmp_region);
        double vmin = INFINITY;
        int64_t kept = 0;
        for (int64_t j = 0; j < m; ++j) {
            double u, v;
            rot_uv(k, xy[2 * (int64_t)lists[j]], xy[2 * (int64_t)lists[j] + 1], &u, &v);
            if (v < vmin) {
                r->kept[nk++] = lists[j];
                ++kept;
                vmin = v;
            }
        }
        r->n_kept[k] = kept;
    }
    r->m2 = nk + nc;

    /* the final hull (the paper's second stage, on the host): per region a
     * stack scan of corner k, the kept points in walking order and corner
     * k+1 (a non-left turn pops, a repeat of the top is skipped): the hull's
     * chain from corner k to corner k+1.  The chains, each without its last
     * point (the next chain's first), form the hull from P_minx on. */
    int64_t h = 0;
    int64_t at = 0;
    for (int k = 0; k < 4; ++k) {
        const int64_t beg = h;
        for (int64_t j = -1; j <= r->n_kept[k]; ++j) {
            const int32_t p = j < 0 ? c[k] : j == r->n_kept[k] ? c[(k + 1) & 3] : r->kept[at + j];
            if (h > beg && same_point(xy, stack[h - 1], p)) continue;
            while (h - beg >= 2 && orient_idx(xy, stack[h - 2], stack[h - 1], p) <= 0) --h;
            stack[h++] = p;
        }
        at += r->n_kept[k];
        --h;  /* corner k+1: the next chain starts with it */
    }
    if (h == 0) stack[h++] = c[0];  /* one distinct point */
    /* canonical start: the lexicographically smallest vertex */
    int64_t start = 0;
    for (int64_t i = 1; i < h; ++i) {
        double x = xy[2 * (int64_t)stack[i]], y = xy[2 * (int64_t)stack[i] + 1];
        double bx = xy[2 * (int64_t)stack[start]], by = xy[2 * (int64_t)stack[start] + 1];
        if (x < bx || (x == bx && y < by)) start = i;
    }
    for (int64_t i = 0; i < h; ++i) r->hull[i] = stack[(start + i) % h];
    r->h = h;
    free(lists);
    free(stack);
    return ORACLE_OK;
}
