// records.hpp - a sorted point with the exact angular order of Section 2.1
// (the sort order of Step 4).
#pragma once

#include "common.hpp"
#include "exact.hpp"

namespace hx {

struct Rec {
    double x, y;
    uint32_t idx, slot;
};

__device__ inline Rec rec_load(uint32_t slot, const double2* __restrict__ comp,
                               const uint32_t* __restrict__ comp_idx) {
    double2 v = comp[slot];
    Rec r;
    r.x = v.x;
    r.y = v.y;
    r.idx = comp_idx[slot];
    r.slot = slot;
    return r;
}

// Strict total order of the sort: angle about the pivot (exact orientation),
// then distance along the ray, then input index.
__device__ inline bool rec_less(const Rec& a, const Rec& b, double x0, double y0) {
    return angle_less(a.x, a.y, a.idx, b.x, b.y, b.idx, x0, y0);
}

}  // namespace hx
