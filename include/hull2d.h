/*
 * hull2d.h - exact 2D convex hulls on AMD Instinct MI355X (gfx950).
 *
 * The data-parallel first stage of gScan (G. Mei, "gScan: Accelerating
 * Graham Scan on the GPU", Sections 2 and 3) as hand-written HIP kernels,
 * followed by the paper's final stack scan (Step 8, on the host or on the
 * device, options.scan):
 *
 *   Step 1  four extreme points by parallel reduction           (Section 3.1)
 *   Step 2  discard points strictly inside their quadrilateral  (Section 3.1)
 *   Step 3  exact angle keys about the pivot and farthest point (Section 3.2)
 *   Step 4  sort of the survivors by exact angle                 (Section 3.3)
 *   Step 5-6 farthest point P_l splits the sorted list          (Section 2.1)
 *   Step 7  second-round filter per region (Figure 2)           (Section 3.4)
 *   Step 8  stack scan of the kept points, as chains of pieces
 *           joined at their common tangents                      (Section 3)
 *
 * Input: n points as float64 [n][2] (x, y interleaved) in device memory.
 * Output: the canonical hull as int32 input indices in host memory:
 * counter-clockwise, starting at the lexicographically smallest vertex
 * (smallest x, then smallest y), collinear points and duplicates dropped,
 * each vertex reported by the smallest index holding its coordinates.
 * All geometric decisions are exact (float64 error-free products with an
 * adaptive expansion fallback), so the output is a deterministic function of
 * the input bytes.
 *
 * Input domain: every coordinate finite, and either 0 or of magnitude in
 * [2^-300, 2^300] (then the exact arithmetic never leaves the normal range);
 * -0.0 equals +0.0.  At most 2^31 - 1 points per set.
 *
 * Ownership and threading: the caller owns every input and output buffer;
 * inputs are never written.  A context owns a device workspace that grows on
 * demand and is freed by hull2d_destroy.  A context is bound to one device
 * and one HIP stream and is not thread-safe: use one context per stream.
 * Calls return after the host output is written (they synchronise the
 * context's stream).  Nothing throws across this interface.
 */
#ifndef HULL2D_H
#define HULL2D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hull2d_ctx hull2d_ctx;

typedef enum {
    HULL2D_OK = 0,
    HULL2D_ERR_INVALID_ARG = 1,  /* null pointer, negative size, bad option       */
    HULL2D_ERR_NONFINITE = 2,    /* a coordinate is NaN or infinite                */
    HULL2D_ERR_RANGE = 3,        /* a non-zero coordinate outside [2^-300, 2^300]  */
    HULL2D_ERR_CAPACITY = 4,     /* output too small; required size written back  */
    HULL2D_ERR_OUT_OF_MEMORY = 5,/* device or pinned host allocation failed        */
    HULL2D_ERR_DEVICE = 6,       /* a HIP call failed; the context is unusable     */
    HULL2D_ERR_WEIGHTS = 7,      /* learned-filter weights missing or corrupt      */
    HULL2D_ERR_UNIMPLEMENTED = 8,
    HULL2D_ERR_TOO_LARGE = 9     /* n above HULL2D_NOALLOC_MAX_POINTS (no-allocation entry point) */
} hull2d_status;

/* Largest input of hull2d_compute_noalloc (2^18 points). */
#define HULL2D_NOALLOC_MAX_POINTS 262144

/* Options.  Zero-initialise, then set struct_size = sizeof(hull2d_options). */
typedef struct {
    uint32_t struct_size;
    /* Round-2 subsets (Section 3.4).  0: each region is filtered as one
     * sequence, exactly as Figure 2 prints it (computed in parallel as a
     * prefix scan; the default).  -1: the paper's division of each region into
     * 1024 subsets of ceil(m/1024) points, each subset walked by one thread.
     * c > 0: subsets of c points.  The hull is identical in every mode; only
     * the number of round-2 survivors and the time change. */
    int32_t round2_chunk;
    /* 1: record per-kernel device times (HIP events) into hull2d_stats.
     * 2: record only Step 1 and Steps 2-3 (the two streaming passes over the
     * input), two events per call; the other stage times stay 0. */
    int32_t profile;
    /* Only for round2_chunk = 0.  0 (default): sort only the round-1 survivors
     * that can still be running maxima of the walk (coarse angle buckets and
     * an exclusive prefix of exact direction keys decide which; the kept set
     * is identical).  1: sort every round-1 survivor, as Step 4 prints it. */
    int32_t full_sort;
    /* First-round filter.  0 (default): the quadrilateral of Steps 1-2.
     * 1: the learned discard polygon (not in the paper): a network proposes 16
     * directions from a 32 x 32 occupancy histogram of a sample (every point
     * when n <= 4096, else 16 blocks of 256 points, block b starting at
     * floor(b n / 16)); the exact hull of the sample points extreme in those
     * directions and of the four Step-1 extremes is the discard polygon, and
     * a point is discarded strictly inside it.  It contains the
     * quadrilateral, so it discards at least as much, and never a hull
     * vertex (its corners are input points).  Needs weights
     * (hull2d_set_weights / hull2d_load_weights), else hull2d_compute
     * returns HULL2D_ERR_WEIGHTS. */
    int32_t filter;
    /* Schedule of the batched form (hull2d_batch); 0 keeps each default.
     * batch_blocks_per_cu: workgroups per compute unit of the persistent
     * launch (1 or 2; 0: as many as fit).  batch_order: the order in which
     * workgroups take the sets: 0 by size class (powers of two), largest
     * first; 1 by exact size, largest first; 2 input order.
     * paper_1508_05931_amd/autotune.py picks both by timing. */
    int32_t batch_blocks_per_cu;
    int32_t batch_order;
    /* 1: hull2d_batch captures its device work (the uploads of the offsets
     * and the schedule, the persistent launch, the download of the per-set
     * counts) in a HIP graph on the first call and replays it while the
     * set count, the points' address and the workspace stay the same;
     * 0: plain stream work every call.  The results are identical. */
    int32_t batch_graph;
    /* 0 (default): gScan, Steps 1-8 as above.  1: the four-region variant of
     * Section 5.1 (Table 8's comparison method): Steps 1-2, then every
     * survivor strictly outside edge k of the cycle P_minx -> P_miny -> P_maxx
     * -> P_maxy (the first such edge) goes to region k, which is ordered by
     * one coordinate (x, y, -x, -y for k = 0..3; ties by the other, negated
     * for k = 1, 2: (u, v) = (x, y), (y, -x), (-x, -y), (-y, x), then index)
     * and walked keeping a point only when its v is strictly below every v
     * before it; the hull is one stack scan per region from corner k over the
     * kept points to corner k+1 (on the host, as the variant's second stage).
     * Same canonical output.  Only the candidates (v below the minimum of
     * every earlier one of 65,536 buckets of u) are sorted and walked, which
     * keeps the same points.  round2_chunk, full_sort and filter do not
     * apply. */
    int32_t method;
    /* 1: hull2d_create also reserves the host buffers of
     * hull2d_compute_noalloc for its largest input (about 5 MB of pinned and
     * 3 MB of pageable host memory); required by that entry point. */
    int32_t reserve_noalloc;
    /* Where Step 8 runs.  0 (default): on the device when at least 65,536
     * points are kept by round 2 and the one-workgroup tail did not take
     * them, else on the host (faster for fewer kept points); 1: on the
     * device whenever possible; 2: on the host.  Same output either way;
     * the device falls back to the host when the chains of its parts exceed
     * one workgroup's LDS. */
    int32_t scan;
    /* Largest device workspace the context may allocate for one hull, in
     * MiB (0: no limit).  A call that needs more returns
     * HULL2D_ERR_OUT_OF_MEMORY and leaves the context usable. */
    int32_t workspace_limit_mib;
    /* How hull2d_batch spreads the sets over the device.  0 (default): tiled
     * -- every pass over points runs over tiles of 4,096 points of all sets
     * at once (so a large set is shared by many workgroups), the passes over
     * a whole set (reductions, bucket prefixes, the sort and walk of each
     * region, Step 8) take one workgroup per set or region; the candidates
     * are grouped by angle bucket and sorted bucket by bucket in LDS.  1: one
     * persistent launch, each workgroup computing whole sets start to end
     * (batch_blocks_per_cu and batch_order apply to it only).  Same output. */
    int32_t batch_engine;
    /* Schedule of the tiled engine; 0 keeps each default, other values give
     * the same output.  batch_tile: points per tile of the passes over
     * points (a power of two, 1,024 to 65,536; default 4,096).
     * batch_filter_bits: at most 2^batch_filter_bits buckets per region for
     * the bucket maxima of Steps 6-7 (4 to 14; default 14; a set gets about
     * one bucket per four points up to that).  batch_sort_bits: at most
     * 2^batch_sort_bits angle buckets per region for the grouping before the
     * sort (4 to 12; default 12).  batch_side_sets: how many of the largest
     * sets (those of at least 65,536 points) run on a second stream beside
     * the others (1 to 4,096; -1 none, one stream; default 128).
     * batch_items: points each thread takes per round in the passes over
     * points (2, 4 or 8; default 4).
     * paper_1508_05931_amd/autotune.py picks them by timing. */
    int32_t batch_tile;
    int32_t batch_filter_bits;
    int32_t batch_sort_bits;
    int32_t batch_side_sets;
    int32_t batch_items;
} hull2d_options;

/* Per-kernel stage indices of hull2d_stats.ms_stage. */
enum {
    HULL2D_STAGE_EXTREMES = 0,   /* Step 1 partial reduction                       */
    HULL2D_STAGE_EXTREMES_FINAL, /* Step 1 final reduction and quadrilateral        */
    HULL2D_STAGE_FILTER1,        /* Step 2 discard + Step 3 keys + compaction       */
    HULL2D_STAGE_LONGEST,        /* Step 5 farthest point                           */
    HULL2D_STAGE_HISTOGRAM,      /* Step 4 digit histograms                         */
    HULL2D_STAGE_SORT0,          /* Step 4 radix passes (bits 0-7 ... 24-31)        */
    HULL2D_STAGE_SORT1,
    HULL2D_STAGE_SORT2,
    HULL2D_STAGE_SORT3,
    HULL2D_STAGE_TIES,           /* Step 4 exact order inside equal-key runs        */
    HULL2D_STAGE_TIES_LONG,
    HULL2D_STAGE_BUCKETS,        /* Steps 6-7 bucket maxima, prefix, candidates     */
    HULL2D_STAGE_ROUND2,         /* Steps 6-7 second-round filter                   */
    HULL2D_STAGE_COMPACT,        /* Step 7 stable removal of interior points        */
    HULL2D_STAGE_TAIL,           /* Steps 4, 6-7 on a small candidate set, one workgroup */
    HULL2D_STAGE_LEARNED,        /* learned filter: histogram, network, polygon     */
    HULL2D_STAGE_D2H,            /* copy of the kept points to the host             */
    HULL2D_STAGE_HOST_SCAN,      /* Step 8 on the host (wall clock; 0 when the device finished it) */
    HULL2D_STAGE_SCAN,           /* Step 8 on the device                            */
    HULL2D_NUM_STAGES
};

typedef struct {
    int64_t n;            /* points in                                             */
    int64_t n_round1;     /* points that survived round 1 (Step 2)                 */
    int64_t n_sorted;     /* round-1 survivors other than copies of the pivot      */
    int64_t n_round2;     /* points kept by round 2, the pivot included            */
    int64_t n_hull;       /* hull vertices                                          */
    int64_t n_candidates; /* points sorted for round 2 (= n_sorted with full_sort)  */
    double ms_total;      /* host wall clock of the whole call                     */
    double ms_device;     /* first kernel start to end of the host copy (events)   */
    double ms_stage[HULL2D_NUM_STAGES]; /* filled when options.profile = 1 (2: two) */
} hull2d_stats;

/* Create a context on HIP device `device` using stream `hip_stream`
 * (a hipStream_t; NULL = the default stream).  opt may be NULL (defaults).
 * Errors: INVALID_ARG, DEVICE. */
hull2d_status hull2d_create(hull2d_ctx** out, int device, void* hip_stream,
                            const hull2d_options* opt);

/* Hull of n points at d_xy (device, float64 [n][2], 8-byte aligned).
 * Writes at most `cap` indices to h_out (host) and the hull size to *n_out.
 * CAPACITY: *n_out holds the required size and h_out is untouched.
 * NONFINITE / RANGE: input outside the domain; *n_out = 0.
 * stats may be NULL. */
hull2d_status hull2d_compute(hull2d_ctx* ctx, const double* d_xy, int64_t n,
                             int32_t* h_out, int64_t cap, int64_t* n_out,
                             hull2d_stats* stats);

/* hull2d_compute for callers that cannot allocate memory during the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same result, with no hipMalloc, hipFree, pinned or heap
 * allocation inside the call.  The device workspace is a fixed array of the
 * library (about 23 MB on each device the library runs on, held until the
 * process ends) sized for HULL2D_NOALLOC_MAX_POINTS points; the context must
 * have been created with options.reserve_noalloc = 1 (else INVALID_ARG),
 * which reserves the host buffers at creation.  Every call on a device
 * shares that device's array, so calls that overlap on one device (from any
 * context or thread) race; calls on one context are serialised by its
 * stream as usual.  The array keeps the last call's contents; the call
 * itself initialises everything it reads.
 * TOO_LARGE: n > HULL2D_NOALLOC_MAX_POINTS (nothing is computed).  Other
 * errors as hull2d_compute. */
hull2d_status hull2d_compute_noalloc(hull2d_ctx* ctx, const double* d_xy, int64_t n,
                                     int32_t* h_out, int64_t cap, int64_t* n_out,
                                     hull2d_stats* stats);

/* Hulls of S independent sets stored back to back at d_xy: set s is points
 * [h_offsets[s], h_offsets[s+1]) (host array of S+1 non-decreasing int64,
 * h_offsets[0] = 0).  Each set's hull (indices local to the set, canonical as
 * above) is written to h_out at [h_out_offsets[s], h_out_offsets[s+1]).
 * One persistent launch computes every set (Steps 1-8 on the device, one
 * workgroup per set at a time, largest sets first); a set whose equal-key
 * runs exceed the workgroup sorter is finished with hull2d_compute.
 * CAPACITY: the offsets are still written, with h_out_offsets[S] the
 * required size, and h_out is untouched.  NONFINITE / RANGE: some set is
 * outside the domain.  stats (may be NULL): n = total points, n_hull = total
 * hull vertices, n_candidates = sets finished by hull2d_compute, ms_device,
 * ms_total; the other fields are 0. */
hull2d_status hull2d_batch(hull2d_ctx* ctx, const double* d_xy,
                           const int64_t* h_offsets, int32_t S,
                           int32_t* h_out, int64_t cap, int64_t* h_out_offsets,
                           hull2d_stats* stats);

void hull2d_destroy(hull2d_ctx* ctx);

const char* hull2d_status_string(hull2d_status s);

/* ---- Learned filter: network weights and training ---------------------- */

/* The network: 1024 inputs (the occupancy histogram), two hidden layers of
 * 256 ReLU units, 32 outputs read as 16 directions (y[2j], y[2j+1]).
 * Parameters are one float32 vector, W1 [256][1024], b1 [256], W2 [256][256],
 * b2 [256], W3 [32][256], b3 [32] (row = output unit), HULL2D_MLP_PARAMS
 * values.  Inference uses bfloat16 weights and layer inputs with float32
 * sums; training keeps float32 weights. */
#define HULL2D_MLP_PARAMS 336416

/* Copy parameters from host memory (count = HULL2D_MLP_PARAMS) to the
 * context: they become the inference weights and the training start point
 * (the optimiser state is reset).  Errors: INVALID_ARG, WEIGHTS (a
 * non-finite value), OUT_OF_MEMORY, DEVICE. */
hull2d_status hull2d_set_weights(hull2d_ctx* ctx, const float* h_params, int64_t count);

/* The same from a file of HULL2D_MLP_PARAMS little-endian float32 values
 * (no header; the shapes are fixed).  WEIGHTS: missing, short or non-finite. */
hull2d_status hull2d_load_weights(hull2d_ctx* ctx, const char* path);

/* The current float32 parameters to host memory (count = HULL2D_MLP_PARAMS). */
hull2d_status hull2d_get_weights(hull2d_ctx* ctx, float* h_params, int64_t count);

/* The network input of a point set: 32 x 32 occupancy histogram of the
 * sample (all points when n <= 4096, else 16 blocks of 256 consecutive points,
 * block b starting at floor(b n / 16)) over the sample's bounding box,
 * cell (cy * 32 + cx), each count times 1024 / (sample size).  d_xy device
 * float64 [n][2]; d_x device float32 [1024].  Synchronous. */
hull2d_status hull2d_histogram(hull2d_ctx* ctx, const double* d_xy, int64_t n, float* d_x);

/* Inference (the filter's precision) on `rows` inputs: d_x device float32
 * [rows][1024], d_y device float32 [rows][32].  WEIGHTS if none are set. */
hull2d_status hull2d_mlp_infer(hull2d_ctx* ctx, const float* d_x, int32_t rows, float* d_y);

/* One training step on a batch (1 <= B <= 4096): float32 forward pass, mean
 * squared error against d_t [B][32] (device), gradient by backpropagation;
 * apply = 1 then takes an Adam step (beta 0.9 / 0.999, eps 1e-8, rate lr).
 * h_loss (may be NULL) receives the loss before the step, h_grad (may be
 * NULL, HULL2D_MLP_PARAMS floats) the gradient in the parameter layout. */
hull2d_status hull2d_train_step(hull2d_ctx* ctx, const float* d_x, const float* d_t, int32_t B,
                                float lr, int32_t apply, float* h_loss, float* h_grad);

/* What the learned filter used in the last hull2d_compute with filter = 1:
 * dirs[32] (the 16 directions), cand[20] (input indices: the four Step-1
 * extremes, then the sample point extreme along each direction), y[32] (the
 * raw network outputs), *nv (corners of the discard polygon).  Any pointer may
 * be NULL.  INVALID_ARG if the last call did not use the learned filter. */
hull2d_status hull2d_debug_learned(hull2d_ctx* ctx, double* dirs, int32_t* cand, float* y,
                                   int32_t* nv);

/* The last hull2d_compute with method = 1: counts[14] = {m1, survivors in
 * regions 0-3, candidates in regions 0-3, kept points in regions 0-3, m2 (kept
 * points plus distinct corners)}, and kept[cap] the kept points' input
 * indices, region 0 first, each region in walking order.  Any pointer may be
 * NULL.  CAPACITY if cap is smaller than the kept points; INVALID_ARG if the
 * last call did not use the variant. */
hull2d_status hull2d_debug_chain(hull2d_ctx* ctx, int64_t* counts, int32_t* kept, int64_t cap);

/* ---- Checking entry points (exact predicates on the device) ------------ */

/* out[i] = sign of (b - a) x (c - a) for triple i, computed by the device
 * predicate; abc is device float64 [count][6] = (ax, ay, bx, by, cx, cy),
 * out is device int32 [count].  Synchronous. */
hull2d_status hull2d_debug_orient(hull2d_ctx* ctx, const double* d_abc, int64_t count,
                                  int32_t* d_out);

/* out[i] = the exact 32-bit angle key of point i about the pivot (x0, y0):
 * floor(2^31 * phi) with phi = dy/(|dx|+dy) for dx >= 0 and
 * 2 - dy/(|dx|+dy) for dx < 0 (dx = x - x0, dy = y - y0 >= 0).  Points must
 * satisfy y > y0, or y == y0 and x > x0.  d_xy device float64 [count][2],
 * d_out device uint32 [count].  Synchronous. */
hull2d_status hull2d_debug_angle_key(hull2d_ctx* ctx, const double* d_xy, int64_t count,
                                     double x0, double y0, uint32_t* d_out);

/* Stage results of the last hull2d_compute on this context, for checking
 * against a step-by-step model.  Any pointer may be NULL.  Host buffers:
 * extremes[4] (input indices of P_minx, P_miny, P_maxx, P_maxy);
 * sorted[cap] (input indices of the sorted round-1 survivors, Step 4; only
 * filled when every survivor was sorted, see counts[4]);
 * round2[cap] (input indices kept by round 2 in angular order, pivot first);
 * counts[6] = {n_sorted, l (position of P_l in [pivot, sorted...]),
 * n_round2, longest (input index of P_l), 1 if sorted was filled,
 * n_candidates}.
 * CAPACITY if cap is smaller than n_sorted or n_round2. */
hull2d_status hull2d_debug_stages(hull2d_ctx* ctx, int32_t* extremes, int32_t* sorted,
                                  int32_t* round2, int64_t cap, int64_t* counts);

/* The round-1 survivors of the last hull2d_compute on this context (Step 2,
 * Section 3.1; with filter = 1 the learned polygon's survivors): their input
 * indices in ascending order, copies of the pivot P_0 excluded.  idx: host,
 * cap entries; *n_out receives the count.  CAPACITY if cap is smaller (then
 * idx is untouched); INVALID_ARG if no compute call has run yet. */
hull2d_status hull2d_debug_round1(hull2d_ctx* ctx, int32_t* idx, int64_t cap, int64_t* n_out);

#ifdef __cplusplus
}
#endif
#endif
