// common.hpp - shared device data structures of the hull path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hx {

// One extreme-point candidate of Step 1.
struct Cand {
    double x, y;
    int32_t i;
    int32_t pad;
};

// Per-call results that later kernels read (device memory, written once).
struct Params {
    Cand ext[4];        // P_minx, P_miny, P_maxx, P_maxy
    double qx[4], qy[4];  // distinct corners of the quadrilateral, counter-clockwise
    double ex[4], ey[4];  // edge vectors qx[j+1]-qx[j] (rounded)
    double qbound;      // float64 error bound valid for every edge test of Step 2
    double x0, y0;      // pivot P_0 = P_miny
    int32_t ncorner;    // distinct corners (discard nothing below 3)
    int32_t p0_idx;
    uint32_t flags;     // kFlagNonfinite | kFlagRange
    int32_t pad;
    // Step 5
    double lx, ly;      // P_l
    int32_t l_idx;      // input index of P_l (-1: no sorted points)
    uint32_t kl;        // angle key of P_l
    // direction keys (turn_key about P_l) of P_0 - P_l and P_l - P_0
    uint32_t turn_u, turn_v;
    int32_t pad2[2];
};

constexpr uint32_t kTailDone = 0u;
constexpr uint32_t kTailOverflow = 1u;
constexpr uint32_t kTailUnset = 0xFFFFFFFFu;  // host side: not yet written by the tail

// State of the device's Step 8 (k_scan), as the host copy of the candidate
// status reports it.
constexpr uint32_t kScanNone = 0u;      // not run (the tail gave up)
constexpr uint32_t kScanDone = 1u;      // the hull is in host memory
constexpr uint32_t kScanOverflow = 2u;  // the parts' chains did not fit: the host scans
constexpr uint32_t kScanUnset = 0xFFFFFFFFu;  // host side: not yet written

constexpr uint32_t kFlagNonfinite = 1u;
constexpr uint32_t kFlagRange = 2u;

// Status of one sorting problem (the round-1 survivors, or the round-2
// candidates of the bucketed filter); the host reads both back at the end of
// a call.
struct DevStatus {
    uint32_t flags;       // domain flags
    uint32_t huge_runs;   // equal-key runs too long for one workgroup
    uint32_t n_sorted;    // points of this problem (round 1: survivors other than copies of P_0)
    uint32_t n_p0;        // points equal to P_0 (P_0 included)
    uint32_t l_pos;       // position of P_l in this problem's sorted order
    uint32_t n_kept;      // round-2 survivors other than P_0
    uint32_t long_runs;   // equal-key runs handed to the workgroup sorter
    uint32_t l_slot;      // slot of P_l in this problem's arrays
    uint32_t n_right;     // points before P_l in angular order (bucketed filter)
    uint32_t tail_state;  // candidate problem: kTailDone, or kTailOverflow (too large for
                          // the one-workgroup tail; the multi-kernel path runs instead)
    uint32_t n_hull;      // host copy only: hull vertices found by the device scan (Step 8)
    uint32_t scan_state;  // host copy only: kScanNone, kScanDone or kScanOverflow
    int32_t ext[4];
    int32_t p0_idx, l_idx;
    double x0, y0;
};

// Ticket counters of the look-back kernels; they persist across calls, and
// each kernel resets its own counter when its last ticket has been taken.
struct Counters {
    uint32_t ticket[16 * 16];  // one 64-byte line per counter
};

enum TicketId {
    kTicketSort0 = 0,  // ..3
    kTicketRound2 = 4,
    kTicketCompact = 5,
    kTicketBatch = 7,
    kTicketScan = 8,
};

constexpr int kBucketBits = 12;                 // coarse angle buckets of the bucketed round 2
constexpr int kBuckets = 1 << kBucketBits;

// Look-back status word: [epoch:30 | flag:2 | value:32].  The epoch changes
// on every launch, so stale words from an earlier launch never look ready and
// the status arrays need no clearing.
constexpr uint32_t kStatAggregate = 1u;
constexpr uint32_t kStatInclusive = 2u;

__device__ inline uint64_t stat_pack(uint32_t epoch, uint32_t flag, uint32_t value) {
    return ((uint64_t)((epoch << 2) | flag) << 32) | value;
}
__device__ inline uint32_t stat_flag(uint64_t w, uint32_t epoch) {
    uint32_t hi = (uint32_t)(w >> 32);
    return (hi >> 2) == (epoch & 0x3FFFFFFFu) ? (hi & 3u) : 0u;
}
__device__ inline uint32_t stat_value(uint64_t w) { return (uint32_t)w; }

__device__ inline uint32_t take_ticket(uint32_t* c) {
    return __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void reset_ticket(uint32_t* c) {
    __hip_atomic_store(c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tile order for the look-back kernels.  Blocks at or beyond the tile count
// leave at once without touching the counter; the others take tiles in
// ticket order (a tile's predecessors are then held by running blocks), and
// each takes one ticket past the end before it leaves; the block that draws
// the last of those resets the counter for the next launch.  Returns the
// next tile, or `tiles` when the block is done.  All threads call it.
__device__ inline uint32_t next_tile(uint32_t* counter, uint32_t tiles, uint32_t* s_ticket) {
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = take_ticket(counter);
        const uint32_t players = min(gridDim.x, tiles);
        if (t == tiles + players - 1) reset_ticket(counter);
        *s_ticket = t;
    }
    __syncthreads();
    const uint32_t t = *s_ticket;
    return t < tiles ? t : tiles;
}

__device__ inline void stat_store(uint64_t* p, uint64_t w) {
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t stat_load(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Streaming accesses: data read or written once per pass, marked
// non-temporal so that it does not displace cached lines (on gfx950 a plain
// device copy reaches 4.5 TB/s, the same copy with non-temporal loads and
// stores 6.1 TB/s; the first-round passes gain from non-temporal loads of
// the input, while their outputs, read again soon after, are stored
// normally).
typedef double hx_double2_v __attribute__((ext_vector_type(2)));
__device__ inline double2 load_stream(const double2* p) {
    const hx_double2_v v = __builtin_nontemporal_load(reinterpret_cast<const hx_double2_v*>(p));
    return make_double2(v.x, v.y);
}
__device__ inline void store_stream(double2* p, double2 v) {
    hx_double2_v w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<hx_double2_v*>(p));
}
__device__ inline void store_stream(uint32_t* p, uint32_t v) { __builtin_nontemporal_store(v, p); }

// Wave64 helpers.
__device__ inline uint64_t lanemask_lt() {
    uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Lanes of the wave whose `valid` 8-bit digit equals this lane's: one ballot
// per bit, each folded in as "the lanes whose bit equals mine" with the
// lane's sign-extended bit (two 32-bit halves, no per-lane select).
__device__ inline uint64_t match_digit8(uint32_t dig, bool valid) {
    const uint64_t v = __ballot(valid);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int32_t f = (int32_t)(dig << (31 - b)) >> 31;  // all ones when bit b is set
        const uint64_t bb = __ballot(f < 0);
        lo &= ~((uint32_t)bb ^ (uint32_t)f);
        hi &= ~((uint32_t)(bb >> 32) ^ (uint32_t)f);
    }
    return ((uint64_t)hi << 32) | lo;
}

}  // namespace hx
