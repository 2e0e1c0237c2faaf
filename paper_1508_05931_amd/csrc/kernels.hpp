// kernels.hpp - host launchers of the hull path's gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace hx {

// Launch geometry shared by the launchers and the workspace sizing.
constexpr int kExtBlock = 256;
constexpr int kExtGridMax = 1024;
constexpr int kF1Block = 256;
constexpr int kF1Ipt = 8;
constexpr int kF1Tile = kF1Block * kF1Ipt;       // points per round-1 tile
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

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Step 1: partial extreme candidates per block, then the final reduction,
// the quadrilateral and the pivot.
hipError_t launch_extremes(const double* xy, int64_t n, Cand* partial, int grid, Params* prm,
                           DevStatus* ds, hipStream_t s);

// Steps 2-3: strict-interior test against the quadrilateral, exact angle key,
// squared distance, order-preserving compaction of the survivors.
hipError_t launch_filter1(const double* xy, int64_t n, const Params* prm, double2* comp_xy,
                          uint32_t* comp_idx, uint32_t* keys, uint64_t* stat, double* tile_d2,
                          uint32_t* tile_best, DevStatus* ds, Counters* ctr, uint32_t epoch,
                          int grid, hipStream_t s);

// Step 5: farthest point from the tile partials.
hipError_t launch_longest(int64_t n, const double* tile_d2, const uint32_t* tile_best,
                          const double2* comp_xy, Params* prm, DevStatus* ds, hipStream_t s);

// Step 4: digit histograms, four stable radix passes, exact order inside
// equal-key runs.
hipError_t launch_histogram(const uint32_t* keys, const DevStatus* ds, uint32_t* hist, int grid,
                            hipStream_t s);
hipError_t launch_sort_pass(int pass, const uint32_t* keys_in, const uint32_t* vals_in,
                            uint32_t* keys_out, uint32_t* vals_out, const uint32_t* hist,
                            const DevStatus* ds, uint64_t* stat, Counters* ctr, uint32_t epoch,
                            int grid, hipStream_t s);
hipError_t launch_ties(int64_t n, const uint32_t* keys, uint32_t* slots, const double2* comp_xy,
                       const uint32_t* comp_idx, const Params* prm, DevStatus* ds,
                       uint32_t* long_list, hipStream_t s);
hipError_t launch_ties_long(const uint32_t* keys, uint32_t* slots, const double2* comp_xy,
                            const uint32_t* comp_idx, const Params* prm, DevStatus* ds,
                            const uint32_t* long_list, uint32_t* huge_list, int grid,
                            hipStream_t s);

// Steps 6-7: second-round filter (one walk per region as a prefix scan, or
// the paper's per-thread subsets), then stable compaction of the kept points.
hipError_t launch_round2_scan(const uint32_t* slots, const double2* comp_xy, const Params* prm,
                              const DevStatus* ds, uint8_t* keep, uint64_t* stat,
                              Counters* ctr, uint32_t epoch, int grid, hipStream_t s);
hipError_t launch_round2_chunks(int64_t n, int64_t chunk, const uint32_t* slots,
                                const double2* comp_xy, const Params* prm, const DevStatus* ds,
                                uint8_t* keep, hipStream_t s);
hipError_t launch_compact(const uint8_t* keep, const uint32_t* slots, const double2* comp_xy,
                          const uint32_t* comp_idx, double2* out_xy, int32_t* out_idx,
                          DevStatus* ds, uint64_t* stat, Counters* ctr, uint32_t epoch, int grid,
                          hipStream_t s);

// Checking kernels.
hipError_t launch_debug_orient(const double* abc, int64_t count, int32_t* out, hipStream_t s);
hipError_t launch_debug_key(const double* xy, int64_t count, double x0, double y0, uint32_t* out,
                            hipStream_t s);

}  // namespace hx
