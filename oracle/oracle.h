/*
 * oracle.h - CPU oracle for the exact 2D convex hull and for the stages of
 * the gScan method (G. Mei, "gScan: Accelerating Graham Scan on the GPU").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code with the GPU library.
 *
 * Plain, single-threaded, slow on purpose:
 *   - oracle_orient: exact sign of the orientation determinant, from the six
 *     products of its expanded form summed as an exact floating-point
 *     expansion (error-free products by fma, Knuth two-sum, grow-expansion).
 *     No fast filter.
 *   - oracle_hull: Andrew's monotone chain over a lexicographic sort; the
 *     plain definition of the canonical hull (Section 1's problem statement:
 *     the smallest polygon containing all points), with collinear points and
 *     duplicates dropped, counter-clockwise from the lexicographically
 *     smallest vertex, each vertex reported by the smallest input index
 *     holding its coordinates.
 *   - oracle_model: the paper's Steps 1-8 (Section 2.1) in order, with the
 *     second-round filter of Section 2.2 / Figure 2 and its subset division
 *     of Section 3.4, exposing every stage's result.
 *
 * Input domain: every coordinate finite, and either 0 or of magnitude in
 * [2^-300, 2^300]; then every difference, product and error term used by the
 * exact arithmetic is a normal double.  Status codes: 0 ok, 1 non-finite
 * coordinate, 2 magnitude outside the domain, 3 bad argument, 4 no memory,
 * 5 output capacity too small.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_OK = 0, ORACLE_NONFINITE = 1, ORACLE_RANGE = 2, ORACLE_BADARG = 3,
       ORACLE_NOMEM = 4, ORACLE_CAPACITY = 5 };

/* Sign (-1, 0, +1) of (b - a) x (c - a): +1 when a, b, c turn counter-clockwise. */
int oracle_orient(double ax, double ay, double bx, double by, double cx, double cy);

/* Domain check of n points; returns a status code. */
int oracle_validate(const double* xy, int64_t n);

/* Canonical hull of n points (row-major [n][2]).  Writes the vertex indices to
 * out (capacity cap) and their count to *h.  Returns a status code. */
int oracle_hull(const double* xy, int64_t n, int32_t* out, int64_t cap, int64_t* h);

/* Stage results of the method model.  Arrays are caller-owned with the
 * capacities noted; counts are written back. */
typedef struct {
    int32_t extremes[4];      /* P_minx, P_miny, P_maxx, P_maxy (Step 1)        */
    int32_t n_corners;        /* distinct quadrilateral corners (Step 2)        */
    int64_t m1;               /* points surviving the first round               */
    uint8_t* round1_keep;     /* [n]: 1 = survived round 1                      */
    int32_t pivot;            /* P_0 = P_miny                                   */
    int64_t n_sorted;         /* survivors other than copies of P_0             */
    int32_t* sorted;          /* [n]: input indices in angular order (Step 4)   */
    int32_t longest;          /* input index of P_longest (Step 5)              */
    int64_t l;                /* position of P_longest in [P_0, sorted...]      */
    int64_t m2;               /* points kept by round 2, P_0 included           */
    int32_t* round2;          /* [n]: kept points in angular order, P_0 first   */
    int64_t h;                /* hull size                                      */
    int32_t* hull;            /* [n]: canonical hull (Step 8)                   */
} oracle_model_result;

/* Step 7 alone on coordinates already in angular order: q is [N][2] with
 * q[0] = P_0 and q[l] = P_longest; keep[N] receives 1 for kept points.  The
 * chunk argument is as for oracle_model. */
int oracle_round2(const double* q, int64_t N, int64_t l, int64_t chunk, uint8_t* keep);

/* chunk: 0 = each region walked as one sequence (Figure 2 as printed);
 *       -1 = each region divided into 1024 subsets of ceil(m/1024) points
 *            (Section 3.4); c > 0 = subsets of c points. */
int oracle_model(const double* xy, int64_t n, int64_t chunk, oracle_model_result* r);

/* First round with a learned discard polygon instead of the quadrilateral
 * (the learned-filter variant; not in the paper).  dirs is [k][2]: for each
 * direction u the candidate is the point of the network's sample (every point
 * when n <= 4096, else 16 blocks of 256 points, block b starting at
 * floor(b n / 16)) maximising fma(x, ux, y * uy) (ties: smallest index).  The
 * candidates are these k points and the four Step-1 extremes; the polygon is
 * their exact convex hull (strict corners), which contains the
 * quadrilateral, and a point is discarded when it is strictly inside it (a
 * polygon of fewer than three corners discards nothing).  keep[n] receives 1
 * for survivors; cand[k+4] (may be NULL) the candidate indices (extremes
 * first); *m1 the survivor count.  Directions need not be normalised; they
 * must be finite. */
int oracle_learned_round1(const double* xy, int64_t n, const double* dirs, int32_t k,
                          uint8_t* keep, int32_t* cand, int64_t* m1);

/* The four-region variant (Section 5.1, Table 8: the comparison method
 * CudaChain's design, built on Akl and Toussaint's heuristic): Steps 1-2 as
 * above; every survivor strictly outside edge k of the cycle P_minx ->
 * P_miny -> P_maxx -> P_maxy goes to region k (the first such edge), the
 * others (on the quadrilateral's boundary) to none; each region is sorted by
 * x or y (region k in the coordinates (u, v) rotated by -90 degrees k times:
 * u ascending, then v, then index) and walked keeping a point only when its
 * v is strictly below every v before it; the final hull is one stack scan
 * per region from corner k to corner k+1 over the kept points. */
typedef struct {
    int32_t extremes[4];      /* P_minx, P_miny, P_maxx, P_maxy                 */
    int64_t m1;               /* first-round survivors                          */
    int8_t* region;           /* [n]: 0..3, 4 = on the boundary, -1 = discarded */
    int64_t n_region[4];      /* points per region                              */
    int64_t n_kept[4];        /* points each region keeps                       */
    int32_t* kept;            /* [n]: kept points, region 0 first, each in its
                                 walking order                                 */
    int64_t m2;               /* points given to the final stage: the kept
                                 points and the distinct corners              */
    int64_t h;
    int32_t* hull;            /* [n]: canonical hull                            */
} oracle_chain_result;

int oracle_chain(const double* xy, int64_t n, oracle_chain_result* r);

#ifdef __cplusplus
}
#endif
#endif
