// kernels.hpp - host launchers of the hull path's gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "common.hpp"
#include "steps.hpp"

namespace hx {

// Launch geometry shared by the launchers and the workspace sizing.
constexpr int kExtBlock = 256;
constexpr int kExtGridMax = 4096;   // partial-result slots of Step 1
constexpr int kF1Block = 256;
constexpr int kF1Ipt = 4;
constexpr int kF1Tile = kF1Block * kF1Ipt;       // points per round-1 tile
constexpr bool kF1Prefetch = true;               // round 1 loads tile t+1 during tile t
constexpr int kSortBlock = 256;
constexpr int kSortIpt = 16;
constexpr int kSortTile = kSortBlock * kSortIpt; // keys per radix tile
constexpr int kR2Block = 256;
constexpr int kR2Ipt = 8;
constexpr int kR2Tile = kR2Block * kR2Ipt;       // sorted points per round-2 tile
constexpr int kCpBlock = 256;
constexpr int kCpIpt = 16;
constexpr int kCpTile = kCpBlock * kCpIpt;       // flags per compaction tile
constexpr int kRunSmall = 16;                    // equal-key runs sorted by one thread
constexpr int kRunCap = 2048;                    // longest run one workgroup sorts in LDS
constexpr int kHistGridMax = 512;
constexpr int kMlpIn = 1024, kMlpHidden = 256, kMlpOut = 32, kMlpDirs = 16;  // learned filter
constexpr int kTailBlock = 1024;                 // the one-workgroup tail
constexpr int kTailCap = 12288;                  // candidates per region it sorts in LDS
constexpr uint32_t kTailSlots = 65536;           // candidates it reads (16-bit slots)
constexpr int kBatchBlock = 512;                 // threads per set in the batched kernel
constexpr int kScanPart = 6144;                  // kept points per workgroup of the device Step 8
constexpr int kScanMaxParts = 1024;              // its workgroups at most

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Step 1: partial extreme candidates per block, then the final reduction,
// the quadrilateral and the pivot.
// Per-block best of one direction (learned filter).
struct DirBest {
    double v;
    int32_t i;
    int32_t pad;
};

// lo: NULL, or (learned filter) the proposal whose candidates lo->cand[4..19]
// join the four extremes; the final block then writes their exact hull to
// lo->poly and the extremes to lo->cand[0..3].
struct LearnOut;
hipError_t launch_extremes(const double* xy, int64_t n, Cand* partial, int grid, Params* prm,
                           DevStatus* ds, LearnOut* lo, hipStream_t s);
int extremes_grid(int64_t n, int cu_count, int per_cu);
// The final reduction of Step 1 alone (over nblocks partial results).
hipError_t launch_extremes_final(const Cand* partial, int nblocks, Params* prm, DevStatus* ds,
                                 LearnOut* lo, hipStream_t s);
// Learned filter, one pass over the input (blocks = the Steps 2-3 blocks,
// at most kExtGridMax): Step 1's partial extremes of block b's input range,
// and the points of that range not strictly inside lo->spoly (which the
// final discard polygon contains), compacted in input order to pre_xy /
// pre_idx at the block's range, their count in pre_count[b].
hipError_t launch_pre(const double* xy, int64_t n, int blocks, const LearnOut* lo, Cand* partial,
                      double2* pre_xy, uint32_t* pre_idx, uint32_t* pre_count, hipStream_t s);

// Resident blocks per compute unit of the fixed-grid streaming kernels (from
// the runtime's occupancy calculator), so that one launch fills the chip
// exactly once: a block that cannot be resident would run in a second,
// mostly empty wave of blocks.
struct Occupancy {
    int extremes = 1, filter1 = 1, filter1_poly = 1;
};
// At least 1 when the query fails.
inline int resident_blocks(const void* kernel, int block) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, block, 0) != hipSuccess) {
        (void)hipGetLastError();
        b = 0;
    }
    return b > 0 ? b : 1;
}
void occupancy_filter(Occupancy& o);  // extremes, filter1
inline Occupancy query_occupancy() {
    Occupancy o;
    occupancy_filter(o);
    return o;
}

// Steps 2-3: strict-interior test against the quadrilateral, exact angle key,
// squared distance.  Block b compacts the survivors of its input range into
// the same range of comp_xy / comp_idx / keys (a segment of seg_count[b]
// points starting at b*filter1_chunk).
int filter1_blocks(int64_t n, int cu_count, int per_cu);
int64_t filter1_chunk(int64_t n, int blocks);
// poly: NULL for the quadrilateral, else the learned discard polygon.
hipError_t launch_filter1(const double* xy, int64_t n, int blocks, const Params* prm,
                          const Poly* poly, double2* comp_xy, uint32_t* comp_idx, uint32_t* keys,
                          uint32_t* seg_count, double* blk_d2, uint32_t* blk_best, DevStatus* ds,
                          hipStream_t s);

// Steps 2-3 with the learned polygon over launch_pre's output instead of the
// input (the same blocks and ranges).
hipError_t launch_filter1_pre(const double2* pre_xy, const uint32_t* pre_idx, const uint32_t* pre_count,
                              int64_t n, int blocks, const Params* prm, const Poly* poly,
                              double2* comp_xy, uint32_t* comp_idx, uint32_t* keys, uint32_t* seg_count,
                              double* blk_d2, uint32_t* blk_best, DevStatus* ds, hipStream_t s);

// Step 5 and the segment offsets (one block); also clears bmax (2 x
// kBuckets, the bucketed filter's sampled maxima) unless it is NULL.
hipError_t launch_longest(int blocks, const double* blk_d2, const uint32_t* blk_best,
                          const uint32_t* seg_count, uint32_t* seg_off, const double2* comp_xy,
                          const uint32_t* keys, Params* prm, DevStatus* ds, uint32_t* bmax,
                          hipStream_t s);

// Dense (key, slot) pairs of all survivors (for the full sort).
hipError_t launch_densify(int64_t n, int blocks, const uint32_t* seg_count, const uint32_t* seg_off,
                          const uint32_t* keys, uint32_t* dkeys, uint32_t* dslots, hipStream_t s);

// Steps 6-7, bucketed: coarse angle buckets (top bits of the angle key), the
// maximum direction key seen from P_l per bucket and region, an exclusive
// prefix over buckets, and the candidates that can still be running maxima.
// The candidates form a new (small) sorting problem with status ds2.
constexpr int kBmBlock = 512;
hipError_t launch_bucket_max(int64_t n, int segs, const uint32_t* seg_count, const double2* comp_xy,
                             const uint32_t* keys, const Params* prm, uint32_t* bmax, int parts,
                             hipStream_t s);
// The exact prefix maxima from `exact` (the bucket maxima over the
// candidates, 2 x kBuckets), the candidates they select (cand_kap: their
// kappa), then Steps 4 and 6-7 plus the stable removal, for a candidate set
// small enough for one workgroup per region (at most kTailSlots candidates,
// at most kTailCap selected per region); otherwise sets tail_state to
// kTailOverflow in the candidate status and writes nothing else that the
// other path needs.  ds: the round-1 status and the candidate status after
// it.  oslot [2][kTailCap] and ocount [2]: the kept slots per region.
// out_xy / out_idx: the kept points (right region, P_l, left region), device
// or mapped host memory; host_ds: host memory (device-visible) that receives
// both statuses, the candidate status with its kept count.  out_xy NULL:
// only the kept slots (the gather is launch_tail_out, or the device scan
// reads the slots itself).
hipError_t launch_tail(const double2* cand_xy, const uint32_t* cand_idx, const uint32_t* cand_key,
                       const uint32_t* cand_kap, const uint32_t* exact, const Params* prm,
                       DevStatus* ds, uint16_t* oslot, uint32_t* ocount, double2* out_xy,
                       int32_t* out_idx, DevStatus* host_ds, hipStream_t s);
// The kept points and statuses gathered for the host (the tail's output
// when the device scan below did not finish the hull).
hipError_t launch_tail_out(const double2* cand_xy, const uint32_t* cand_idx, DevStatus* ds,
                           const uint16_t* oslot, const uint32_t* ocount, double2* out_xy,
                           int32_t* out_idx, DevStatus* host_ds, hipStream_t s);

// Step 8 on the device (kernels_scan.hip): the hull of the kept points, in
// angular order about P_0, rotated to its lexicographically smallest vertex,
// as input indices in `out` (host-visible); host_ds receives the statuses
// (tail form: both problems, with n_kept, n_hull and scan_state of the
// candidate problem; list form: n_hull and scan_state of host_ds[1]).  The
// parts' chains go to part_xy / part_idx (at each part's first position,
// kScanPart points per part) and part_len [kScanMaxParts]; ticket is a
// counter that is zero between launches.
// Tail form: the kept slots of launch_tail (right region, P_l, left region).
hipError_t launch_scan_tail(const double2* cand_xy, const uint32_t* cand_idx, const uint16_t* oslot,
                            const uint32_t* ocount, const DevStatus* ds, double2* part_xy,
                            uint32_t* part_idx, uint32_t* part_len, uint32_t* ticket, int32_t* out,
                            DevStatus* host_ds, hipStream_t s);
// List form: m kept points in kept_xy / kept_idx (m <= kScanMaxParts * kScanPart).
hipError_t launch_scan_list(const double2* kept_xy, const int32_t* kept_idx, int64_t m, double x0,
                            double y0, int32_t p0_idx, const DevStatus* ds, double2* part_xy,
                            uint32_t* part_idx, uint32_t* part_len, uint32_t* ticket, int32_t* out,
                            DevStatus* host_ds, hipStream_t s);

// ---- the four-region variant (Section 5.1, Table 8) -------------------
constexpr int kChainBuckets = 65536;  // buckets along u per region
constexpr int kChainCap = 4096;       // candidates one workgroup sorts at a time
constexpr int kChainHostCap = 16384;  // kept points per region written to host memory directly

// Device counters of one call (cleared by the first kernel).
struct ChainStatus {
    uint32_t m1;           // round-1 survivors (regions 0-3 and the boundary)
    uint32_t n_region[4];  // survivors per region
    uint32_t n_cand;       // candidates of all regions
    uint32_t pad[10];
};

// Device tables of one call.
struct ChainTables {
    uint64_t* bmin;     // [4][kChainBuckets] minimum of v per bucket (order-preserving keys)
    double* prefix;     // [4][kChainBuckets] minimum over the earlier buckets
    uint32_t* count;    // [4][kChainBuckets] candidates per bucket
    uint32_t* offset;   // [4 * kChainBuckets + 1] where each bucket's candidates start
    uint32_t* cursor;   // [4][kChainBuckets] grouping cursors
    double* tile_min;   // [4 kChainBuckets / 1024] per-tile results of the table scans
    uint32_t* tile_sum;
    ChainStatus* st;
};
constexpr size_t kChainTableBytes = 4 * (size_t)kChainBuckets * (8 + 8 + 4 + 4 + 4) + 4 + 256 +
                                    4 * (size_t)kChainBuckets / 1024 * 12 + 256;

// What the last kernel leaves in host memory.
struct ChainHost {
    DevStatus ds0;          // the round-1 status (domain flags, Step-1 extremes)
    double cx[4], cy[4];    // the corners P_minx, P_miny, P_maxx, P_maxy
    int32_t ci[4];
    uint32_t m1;
    uint32_t n_region[4];
    uint32_t n_cand[4];     // candidates per region
    uint32_t n_kept[4];     // kept points per region
    uint32_t kept_at[4];    // where each region's kept list starts in out_xy / out_idx
    uint32_t on_host[4];    // 1: the list is also in the host buffers (kChainHostCap per region)
    uint32_t overflow[4];   // 1: a bucket held more candidates than one chunk (not computed)
};

// Steps 1-2 are done (prm, ds); the rest of the variant up to its kept
// lists.  cand_*: candidates (n entries at most); grp_*: the same grouped by
// bucket; out_*: kept lists (device, at the region's first candidate
// position); host, host_xy, host_idx: host-visible.
hipError_t launch_chain(const double* xy, int64_t n, const Params* prm, const DevStatus* ds, ChainTables T,
                        double2* cand_xy, uint32_t* cand_idx, uint32_t* cand_rb, double2* grp_xy,
                        uint32_t* grp_idx, double2* out_xy, int32_t* out_idx, ChainHost* host,
                        double2* host_xy, int32_t* host_idx, int grid, hipStream_t s);

// The batched form: one persistent launch, each workgroup computing whole
// hulls of the sets in `order` (device, S entries); per set s, its points are
// xy[offs[s], offs[s+1]) and its workspace the same range of every array.
// Output: hull[h_start[s] ..+ h_count[s]] (set-local indices, canonical),
// h_flags[s] (kFlagNonfinite / kFlagRange, or 4 = finish on the host);
// hull_cursor must be 0 at launch.
hipError_t launch_batch(const double2* xy, const int64_t* offs, const int32_t* order, int32_t S,
                        double2* sv_xy, uint32_t* sv_idx, uint32_t* sv_key, double2* cd_xy,
                        uint32_t* cd_idx, uint32_t* cd_key, uint32_t* ka, uint32_t* kb,
                        uint32_t* va, uint32_t* vb, uint8_t* flag, int32_t* hull,
                        uint32_t* hull_cursor, int32_t* h_count, int32_t* h_start,
                        uint32_t* h_flags, Counters* ctr, int grid, hipStream_t s);
int batch_blocks_per_cu();
// Clears the batched form's hull-buffer counter (meta[0]); a kernel rather
// than a memset so that the work can be captured in a graph.
hipError_t launch_batch_clear(uint32_t* meta, hipStream_t s);
constexpr uint32_t kBatchFallback = 4u;

// The tiled engine of the batched form: the passes over a set's points are
// split into tiles (kWideTile points unless the options say otherwise) and
// the tiles of all sets make one grid per pass; what spans a whole set
// (reductions, bucket prefixes, the sort and walk of each region, Step 8)
// takes one workgroup per set.
constexpr uint32_t kWideTile = 4096;
constexpr uint32_t kWideTileMin = 1024, kWideTileMax = 65536;
// The largest sets (by default at most kWideBigSets of at least kWideBigMin
// points) run the tiled engine's kernels on a second stream beside the
// others: their per-set kernels take the longest and would otherwise leave
// most compute units idle at the end of each per-set launch.
constexpr int32_t kWideBigSets = 128;
constexpr int64_t kWideBigMin = 65536;

// Per set, written by the host: the set's first point, its size, its tiles
// (t0 .. t0 + nt, `tile` points each, the last one shorter), its bucket
// counts (2^bf buckets per region for the bucket maxima, held in LDS; 2^bs
// per region for the sort buckets, whose ends take entries soff ..
// soff + 2^(bs+1) of bcnt).
constexpr int kWideFilterBits = 14;  // at most 16,384 filter buckets per region
constexpr int kWideSmallBits = 11;   // sets of at most 2^11 per region take the small Steps 6-7 workgroup
constexpr int kWideSortBits = 12;    // at most 4,096 sort buckets per region
struct WSetIn {
    int64_t o;
    uint32_t n, t0, nt, bf, bs, soff, tile;
};

// Per set, written by the device.
struct WSet {
    Params P;           // Step 1, then Step 5's fields
    uint32_t flags;     // domain flags, or kBatchFallback
    uint32_t m1;        // round-1 survivors
    uint32_t lslot;     // P_l's position among them
    uint32_t c[2];      // candidates of each region (sort regions: before P_l, P_l and after)
    uint32_t big[2];    // the largest bucket of each region
    uint32_t k[2];      // points each region keeps after the walk
    uint32_t klo[2];    // where each region's kept points start
    uint32_t pad;
};

// Step 5 within one tile: the farthest survivor, its index and position.
struct WFar {
    double d2;
    uint32_t idx, slot;
};

struct WideArgs {
    const double2* xy;
    const WSetIn* in;      // [S]
    WSet* ws;              // [S]
    const int32_t* order;  // [S] the sets of this launch, largest first
    int32_t S;             // sets in this launch
    int32_t S_large;       // its first S_large sets have more than 2^kWideSmallBits filter buckets per region
    int32_t items;         // points per thread per round in the passes over points: 2, 4 or 8
    uint32_t t_base, NT;   // this launch's tiles: t_base .. t_base + NT (global numbering)
    int32_t* tile_set;     // [NT]
    Cand* tile_ext;        // [NT][4]
    uint32_t* tile_flags;  // [NT]
    WFar* tile_far;        // [NT]
    uint32_t* tile_cnt;    // [NT] survivors of the tile (at its own first position)
    uint32_t* bcnt;        // the sort buckets' ends
    double2* sv_xy;        // [N] survivors; after the walk, the kept points
    uint32_t* sv_idx;
    uint32_t* sv_key;
    double2* cd_xy;        // [N] candidates, packed per set
    uint32_t* cd_idx;
    uint32_t* cd_key;
    uint32_t *ka, *kb, *va, *vb;  // [N] sort and Step-8 scratch
    uint2* gk;             // [N] candidates by sort bucket: (angle key, position in cd_*)
    uint8_t* flag;         // [N]
    int32_t* hull;         // output as for launch_batch
    uint32_t* hull_cursor;
    int32_t* h_count;
    int32_t* h_start;
    uint32_t* h_flags;
};
// The whole tiled engine on stream s (hull_cursor must be 0 at launch).
hipError_t launch_wide(const WideArgs& a, hipStream_t s);

// ---- learned-filter variant of Steps 1-2 and its network ----------------
constexpr int64_t kMlpParams = (int64_t)kMlpIn * kMlpHidden + kMlpHidden +
                               (int64_t)kMlpHidden * kMlpHidden + kMlpHidden +
                               (int64_t)kMlpHidden * kMlpOut + kMlpOut;

// Inference weights: bfloat16 bits, [out][in]; float32 biases.
struct MlpDev {
    const uint16_t* w1;
    const uint16_t* w2;
    const uint16_t* w3;
    const float* b1;
    const float* b2;
    const float* b3;
};

// What the proposal produced for one hull.
struct LearnOut {
    Poly poly;                  // the discard polygon
    Poly spoly;                 // the hull of the direction candidates alone (inside poly)
    double dirs[2 * kMlpDirs];  // directions used (network output, or the fallback)
    float y[kMlpOut];           // raw network outputs
    int32_t cand[kPolyMax];     // candidates: the four Step-1 extremes, then one per direction
    double cxy[2 * kMlpDirs];   // coordinates of the direction candidates
};

int learned_grid(int64_t n, int cu_count);
// sample histogram: part holds 4 doubles per block of `grid`; hist 1024 counts
hipError_t launch_histogram_sample(const double* xy, int64_t n, double* part, int grid, uint32_t* hist,
                                   hipStream_t s);
hipError_t launch_hist_to_x(const uint32_t* hist, int64_t n, float* x, hipStream_t s);
// rows inputs x [rows][1024] -> y [rows][32]; h1, h2 [rows][256] scratch.
hipError_t launch_mlp_infer(const float* x, int rows, const MlpDev& W, float* h1, float* h2, float* y,
                            hipStream_t s);
// The whole proposal in one workgroup: the sample histogram, the network and
// its 16 directions into lo->y and lo->dirs (the same arithmetic as
// launch_histogram_sample, launch_hist_to_x and launch_mlp_infer), then the
// sample point farthest along each direction into lo->cand[4 + j] (the
// polygon is built at the end of Step 1, launch_extremes).
hipError_t launch_front(const double* xy, int64_t n, const MlpDev& W, LearnOut* lo, hipStream_t s);
// training
hipError_t launch_gemm(int M, int N, int K, const float* A, int lda, int tA, const float* B, int ldb,
                       int tB, const float* bias, int relu, const float* mask, float* C, int ldc,
                       hipStream_t s);
hipError_t launch_mse(const float* y, const float* t, int count, float* d, float* loss, hipStream_t s);
hipError_t launch_colsum(const float* d, int M, int N, float* out, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_to_bf16(const float* w, int64_t count, uint16_t* wb, hipStream_t s);

hipError_t launch_bucket_scan(uint32_t* bmax, uint32_t* prefix, DevStatus* ds2, hipStream_t s);
hipError_t launch_prefilter(int64_t n, int segs, const uint32_t* seg_count, const double2* comp_xy,
                            const uint32_t* comp_idx, const uint32_t* keys, const Params* prm,
                            DevStatus* ds, const uint32_t* prefix, double2* cand_xy,
                            uint32_t* cand_idx, uint32_t* cand_key, uint32_t* cand_kap, uint32_t* exact,
                            DevStatus* ds2, hipStream_t s);

// Step 4: digit histograms, four stable radix passes, exact order inside
// equal-key runs.
hipError_t launch_histogram(const uint32_t* keys, const DevStatus* ds, uint32_t* hist, int grid,
                            hipStream_t s);
hipError_t launch_sort_pass(int64_t n, int pass, const uint32_t* keys_in, const uint32_t* vals_in,
                            uint32_t* keys_out, uint32_t* vals_out, const uint32_t* hist,
                            const DevStatus* ds, uint64_t* stat, Counters* ctr, uint32_t epoch,
                            int cu_count, hipStream_t s);
hipError_t launch_ties(int64_t n, const uint32_t* keys, uint32_t* slots, const double2* comp_xy,
                       const uint32_t* comp_idx, const Params* prm, DevStatus* ds,
                       uint32_t* long_list, hipStream_t s);
hipError_t launch_ties_long(const uint32_t* keys, uint32_t* slots, const double2* comp_xy,
                            const uint32_t* comp_idx, const Params* prm, DevStatus* ds,
                            const uint32_t* long_list, uint32_t* huge_list, int grid,
                            hipStream_t s);

// Exact order of one equal-key run longer than kRunCap at [start, start+L)
// of slots (tmp: scratch of the same size as slots); also finds P_l in it.
hipError_t launch_huge_run(uint32_t* slots, uint32_t* tmp, uint32_t start, uint32_t L,
                           const double2* comp_xy, const uint32_t* comp_idx, const Params* prm,
                           DevStatus* ds, hipStream_t s);

// Steps 6-7: second-round filter (one walk per region as a prefix scan, or
// the paper's per-thread subsets), then stable compaction of the kept points.
hipError_t launch_round2_scan(int64_t n, const uint32_t* slots, const double2* comp_xy,
                              const Params* prm, const DevStatus* ds, uint8_t* keep, uint64_t* stat,
                              Counters* ctr, uint32_t epoch, int cu_count, hipStream_t s);
hipError_t launch_round2_chunks(int64_t n, int64_t chunk, const uint32_t* slots,
                                const double2* comp_xy, const Params* prm, const DevStatus* ds,
                                uint8_t* keep, hipStream_t s);
hipError_t launch_compact(int64_t n, const uint8_t* keep, const uint32_t* slots,
                          const double2* comp_xy, const uint32_t* comp_idx, double2* out_xy,
                          int32_t* out_idx, DevStatus* ds, uint64_t* stat, Counters* ctr,
                          uint32_t epoch, int cu_count, hipStream_t s);

// Sets `words` 64-bit words at p to zero (a kernel, so that it may be captured).
hipError_t launch_clear_words(uint64_t* p, size_t words, hipStream_t s);

// Checking kernels.
hipError_t launch_debug_orient(const double* abc, int64_t count, int32_t* out, hipStream_t s);
hipError_t launch_debug_key(const double* xy, int64_t count, double x0, double y0, uint32_t* out,
                            hipStream_t s);

}  // namespace hx
