// kernels_filter.hip - Steps 1-3 and 5-7 of gScan on gfx950.
//
//   k_extremes / k_extremes_final  Step 1: four extreme points (Section 3.1)
//   k_filter1                      Step 2: discard points strictly inside the
//                                  quadrilateral (Section 3.1), fused with
//                                  Step 3 (exact angle key and squared
//                                  distance, Section 3.2) and an
//                                  order-preserving compaction
//   k_longest                      Step 5: farthest point from the pivot
//   k_round2_scan                  Steps 6-7: the Figure 2 filter, each region
//                                  as one walk, evaluated as a prefix scan
//   k_round2_chunks                Steps 6-7 with the paper's subsets, one
//                                  thread per subset (Section 3.4)
//   k_compact                      Step 7: stable removal of interior points
//
// Scan kernels chain tile prefixes by decoupled look-back (Merrill & Garland,
// "Single-pass Parallel Prefix Scan with Decoupled Look-back", 2016), with
// tiles taken in ticket order (see next_tile).
#include <float.h>

#include "exact.hpp"
#include "kernels.hpp"
#include "steps.hpp"

namespace hx {
namespace {

constexpr uint32_t kSlotP0 = 0xFFFFFFFFu;    // stands for the pivot P_0
constexpr uint32_t kSlotNone = 0xFFFFFFFEu;  // identity of the running maximum

// ---------------------------------------------------------------------------
// wave64 primitives
// ---------------------------------------------------------------------------
__device__ inline uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    const int lane = (int)__lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(v, off);
        if (lane >= off) v += o;
    }
    return v;
}

// Decoupled look-back for a sum, run by one whole wave.  Publishes the tile's
// aggregate, walks back over predecessors 64 at a time until an inclusive
// prefix is found, publishes its own inclusive prefix and returns the
// exclusive prefix (same value in every lane).
__device__ uint32_t lookback_sum(uint64_t* stat, uint32_t t, uint32_t agg, uint32_t epoch) {
    const uint32_t lane = __lane_id();
    if (t == 0) {
        if (lane == 0) stat_store(&stat[0], stat_pack(epoch, kStatInclusive, agg));
        return 0;
    }
    if (lane == 0) stat_store(&stat[t], stat_pack(epoch, kStatAggregate, agg));
    uint32_t excl = 0;
    int64_t top = (int64_t)t - 1;
    for (;;) {
        int64_t me = top - (int64_t)lane;
        uint32_t f = kStatInclusive, v = 0;
        if (me >= 0) {
            uint64_t w = stat_load(&stat[me]);
            f = stat_flag(w, epoch);
            v = stat_value(w);
        }
        uint64_t incl = __ballot(f == kStatInclusive);
        uint64_t notready = __ballot(f == 0u);
        uint32_t first = incl ? (uint32_t)(__ffsll((unsigned long long)incl) - 1) : 64u;
        uint64_t upto = first >= 63u ? ~0ull : ((2ull << first) - 1ull);
        if (notready & upto) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += wave_sum(lane <= first ? v : 0u);
        if (first < 64u) break;
        top -= 64;
    }
    if (lane == 0) stat_store(&stat[t], stat_pack(epoch, kStatInclusive, excl + agg));
    return excl;
}

// ---------------------------------------------------------------------------
// Step 1
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kExtBlock) void k_extremes(const double2* __restrict__ xy, int64_t n,
                                                        Cand* __restrict__ partial) {
    constexpr int NW = kExtBlock / 64;
    constexpr int U = 8;
    __shared__ Cand s_c[NW][4];
    __shared__ uint32_t s_flags;
    Cand c[4] = {sentinel(0), sentinel(1), sentinel(2), sentinel(3)};
    uint32_t bad = 0;
    if (threadIdx.x == 0) s_flags = 0;
    const int64_t stride = (int64_t)gridDim.x * kExtBlock;
    for (int64_t i = (int64_t)blockIdx.x * kExtBlock + threadIdx.x; i < n; i += stride * U) {
        double2 p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t j = i + u * stride;
            if (j < n) p[u] = load_stream(&xy[j]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t j = i + u * stride;
            if (j < n) {
                // only a point at or beyond one of the four current bests can
                // change one (exact: ties go through the full comparison)
                const bool need = (p[u].x <= c[0].x) | (p[u].y <= c[1].y) | (p[u].x >= c[2].x) |
                                  (p[u].y >= c[3].y);
                if (need) offer(c, p[u].x, p[u].y, (int32_t)j);
                bad |= domain_flags(p[u].x) | domain_flags(p[u].y);
            }
        }
    }
    reduce4_wave(c);
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    __syncthreads();
    if (bad) atomicOr(&s_flags, bad);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s_c[wave][k] = c[k];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        int k = (int)threadIdx.x;
        Cand b = s_c[0][k];
        for (int w = 1; w < NW; ++w) {
            Cand o = s_c[w][k];
            if (k == 0) take_better<0>(b, o);
            else if (k == 1) take_better<1>(b, o);
            else if (k == 2) take_better<2>(b, o);
            else take_better<3>(b, o);
        }
        b.pad = (int32_t)s_flags;
        partial[(int64_t)blockIdx.x * 4 + k] = b;
    }
}

// One block: final reduction of the partial candidates, the distinct
// counter-clockwise corners P_minx -> P_miny -> P_maxx -> P_maxy, the pivot,
// and the per-call reset of the status fields later kernels accumulate into.
// kLearned: then the discard polygon, the exact hull of the four extremes and
// the proposal's 16 candidates (lo->cand[4..19], coordinates lo->cxy) into
// lo->poly.
template <bool kLearned>
__global__ __launch_bounds__(1024) void k_extremes_final(const Cand* __restrict__ partial, int nblocks,
                                                        Params* __restrict__ prm,
                                                        DevStatus* __restrict__ ds,
                                                        LearnOut* __restrict__ lo) {
    constexpr int NW = 1024 / 64;
    __shared__ Cand s_c[NW][4];
    __shared__ uint32_t s_flags;
    if (threadIdx.x == 0) s_flags = 0;
    __syncthreads();
    Cand c[4] = {sentinel(0), sentinel(1), sentinel(2), sentinel(3)};
    uint32_t bad = 0;
    for (int b = (int)threadIdx.x; b < nblocks; b += 1024) {
        take_better<0>(c[0], partial[b * 4 + 0]);
        take_better<1>(c[1], partial[b * 4 + 1]);
        take_better<2>(c[2], partial[b * 4 + 2]);
        take_better<3>(c[3], partial[b * 4 + 3]);
        bad |= (uint32_t)partial[b * 4 + 0].pad;
    }
    reduce4_wave(c);
    if (bad) atomicOr(&s_flags, bad);
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s_c[wave][k] = c[k];
    }
    __syncthreads();
    // one criterion per wave (parallel chains), then the parameters and the
    // status built once in LDS and written out by every thread
    __shared__ Cand s_e[4];
    __shared__ Params s_p;
    __shared__ DevStatus s_s;
    if (lane == 0 && wave < 4) {
        Cand b = s_c[0][wave];
        for (int w = 1; w < NW; ++w) {
            const Cand o = s_c[w][wave];
            if (wave == 0) take_better<0>(b, o);
            else if (wave == 1) take_better<1>(b, o);
            else if (wave == 2) take_better<2>(b, o);
            else take_better<3>(b, o);
        }
        s_e[wave] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const Cand e[4] = {s_e[0], s_e[1], s_e[2], s_e[3]};
        make_params(s_p, e, s_flags);
        DevStatus S;
        S.flags = s_flags;
        S.huge_runs = 0;
        S.n_sorted = 0;
        S.n_p0 = 0;
        S.l_pos = 0;
        S.n_kept = 0;
        S.long_runs = 0;
        S.l_slot = kSlotNone;
        S.n_right = 0;
        S.tail_state = kTailDone;
        S.n_hull = 0;
        S.scan_state = kScanNone;
        for (int k = 0; k < 4; ++k) S.ext[k] = e[k].i;
        S.p0_idx = e[1].i;
        S.l_idx = -1;
        S.x0 = s_p.x0;
        S.y0 = s_p.y0;
        s_s = S;
    }
    __syncthreads();
    static_assert(sizeof(Params) % 4 == 0 && sizeof(DevStatus) % 4 == 0, "word copies");
    for (int i = (int)threadIdx.x; i < (int)(sizeof(Params) / 4); i += 1024)
        reinterpret_cast<uint32_t*>(prm)[i] = reinterpret_cast<const uint32_t*>(&s_p)[i];
    for (int i = (int)threadIdx.x; i < (int)(sizeof(DevStatus) / 4); i += 1024)
        reinterpret_cast<uint32_t*>(ds)[i] = reinterpret_cast<const uint32_t*>(&s_s)[i];
    if (kLearned) {
        static_assert(kPolyMax * kPolyMax <= 1024, "one thread per candidate pair");
        __shared__ double s_x[kPolyMax], s_y[kPolyMax];
        __shared__ int32_t s_use[kPolyMax];
        __shared__ Poly Q;
        const int t = (int)threadIdx.x;
        // the extremes' coordinates are here, the candidates' in lo; outside
        // the domain: no polygon (every point is refused anyway)
        if (t < kPolyMax) {
            const int32_t c = t < 4 ? s_e[t].i : lo->cand[t];
            const double x = t < 4 ? s_e[t].x : lo->cxy[2 * (t - 4)];
            const double y = t < 4 ? s_e[t].y : lo->cxy[2 * (t - 4) + 1];
            s_x[t] = x;
            s_y[t] = y;
            s_use[t] = s_flags == 0u && c != INT32_MAX && fabs(x) <= DBL_MAX && fabs(y) <= DBL_MAX;
        }
        __syncthreads();
        hull_of_points<kPolyMax>(s_x, s_y, s_use, Q);
        static_assert(sizeof(Poly) % 8 == 0, "double copies");
        for (int i = t; i < (int)(sizeof(Poly) / 8); i += 1024)
            reinterpret_cast<double*>(&lo->poly)[i] = reinterpret_cast<const double*>(&Q)[i];
        if (t < 4) lo->cand[t] = s_e[t].i;
    }
}

// ---------------------------------------------------------------------------
// Steps 2-3
//
// Block b owns the input range [b*chunk, (b+1)*chunk) and compacts its
// survivors, in input order, into the same range of the output arrays (a
// segment: survivors never outnumber inputs).  No block waits for another;
// the segment lengths are added up afterwards (k_longest), and later kernels
// read the survivors segment by segment.
// ---------------------------------------------------------------------------
// kPoly: the learned discard polygon (which contains the quadrilateral)
// replaces it.
// kPre: the input is the learned pre-filter's output (launch_pre): block b
// reads in_count[b] points at its range, their input indices in in_idx.
template <bool kPoly, bool kPre = false>
__global__ __launch_bounds__(kF1Block) void k_filter1(
    const double2* __restrict__ xy, int64_t n, int64_t chunk, const Params* __restrict__ prm,
    const Poly* __restrict__ poly,
    double2* __restrict__ comp_xy, uint32_t* __restrict__ comp_idx, uint32_t* __restrict__ keys,
    uint32_t* __restrict__ seg_count, double* __restrict__ blk_d2, uint32_t* __restrict__ blk_best,
    DevStatus* __restrict__ ds, const uint32_t* __restrict__ in_idx = nullptr,
    const uint32_t* __restrict__ in_count = nullptr) {
    constexpr int NW = kF1Block / 64;
    constexpr int G = kF1Ipt * NW;  // (item, wave) groups in position order
    __shared__ uint32_t s_off[G];
    __shared__ uint32_t s_total;
    __shared__ double s_bd2[NW];
    __shared__ uint32_t s_bidx[NW], s_bslot[NW], s_p0[NW];

    __shared__ Poly s_poly;
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    if (kPoly) {
        // one field per thread (the struct is a few hundred bytes)
        const double* src = reinterpret_cast<const double*>(poly);
        double* dst = reinterpret_cast<double*>(&s_poly);
        for (int i = (int)threadIdx.x; i < (int)(sizeof(Poly) / sizeof(double)); i += kF1Block)
            dst[i] = src[i];
        __syncthreads();
        // the polygon's corners are input points: in the Step-1 box, whose
        // bound the quadrilateral's test uses
        if (threadIdx.x == 0) s_poly.qb = prm->qbound;
        __syncthreads();
    }
    const int nc = prm->ncorner;
    const bool discard_all = prm->flags != 0u;
    const double x0 = prm->x0, y0 = prm->y0, qb = prm->qbound;
    double qx[4], qy[4], ex[4], ey[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        qx[j] = prm->qx[j];
        qy[j] = prm->qy[j];
        ex[j] = prm->ex[j];
        ey[j] = prm->ey[j];
    }
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = kPre ? beg + (int64_t)in_count[blockIdx.x] : min(n, beg + chunk);
    int64_t cursor = beg;  // next output position of this segment
    double bd2 = -1.0;     // this thread's farthest survivor so far
    uint32_t bidx = 0xFFFFFFFFu, bslot = 0xFFFFFFFFu;
    uint32_t p0c = 0;

    // the next tile's points are loaded while this tile is processed
    double2 nx[kF1Ipt];
    if (kF1Prefetch) {
#pragma unroll
        for (int k = 0; k < kF1Ipt; ++k) {
            const int64_t pos = beg + k * kF1Block + threadIdx.x;
            if (pos < end) nx[k] = load_stream(&xy[pos]);
        }
    }
    for (int64_t base = beg; base < end; base += kF1Tile) {
        double2 p[kF1Ipt];
        if (kF1Prefetch) {
#pragma unroll
            for (int k = 0; k < kF1Ipt; ++k) p[k] = nx[k];
            const int64_t nb = base + kF1Tile;
#pragma unroll
            for (int k = 0; k < kF1Ipt; ++k) {
                const int64_t pos = nb + k * kF1Block + threadIdx.x;
                if (pos < end) nx[k] = load_stream(&xy[pos]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < kF1Ipt; ++k) {
                const int64_t pos = base + k * kF1Block + threadIdx.x;
                if (pos < end) p[k] = load_stream(&xy[pos]);
            }
        }
        uint64_t mask[kF1Ipt];
        uint32_t key[kF1Ipt];
        // the points' input indices (their positions, unless pre-filtered)
        uint32_t pid[kPre ? kF1Ipt : 1];
        if constexpr (kPre) {
#pragma unroll
            for (int k = 0; k < kF1Ipt; ++k) {
                const int64_t pos = base + k * kF1Block + threadIdx.x;
                pid[k] = pos < end ? in_idx[pos] : 0u;
            }
        }
        double td2 = -1.0;
        uint32_t tidx = 0xFFFFFFFFu, tgrp = 0, trank = 0;
#pragma unroll
        for (int k = 0; k < kF1Ipt; ++k) {
            int64_t pos = base + k * kF1Block + threadIdx.x;
            bool surv = false;
            key[k] = 0;
            if (pos < end && !discard_all) {
                const double px = p[k].x, py = p[k].y;
                surv = kPoly ? !poly_inside(s_poly, px, py)
                             : !quad_inside(qx, qy, ex, ey, qb, nc, px, py);
                if (surv && px == x0 && py == y0) {
                    surv = false;
                    ++p0c;
                }
                if (surv) {
                    key[k] = angle_key(px, py, x0, y0);
                    const double d2 = dist2(px, py, x0, y0);
                    const uint32_t pi = kPre ? pid[kPre ? k : 0] : (uint32_t)pos;
                    const bool take = (d2 > td2) | ((d2 == td2) & (pi < tidx));
                    td2 = take ? d2 : td2;
                    tidx = take ? pi : tidx;
                    tgrp = take ? (uint32_t)(k * NW + wave) : tgrp;
                }
            }
            mask[k] = __ballot(surv);
            if (surv && tidx == (kPre ? pid[kPre ? k : 0] : (uint32_t)pos))
                trank = __popcll(mask[k] & lanemask_lt());
            if (lane == 0) s_off[k * NW + wave] = (uint32_t)__popcll(mask[k]);
        }
        __syncthreads();
        if (wave == 0) {
            uint32_t v = lane < G ? s_off[lane] : 0u;
            uint32_t inc = wave_incl_scan(v);
            if (lane < G) s_off[lane] = inc - v;
            if (lane == 63) s_total = inc;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kF1Ipt; ++k) {
            if ((mask[k] >> lane) & 1ull) {
                int64_t pos = base + k * kF1Block + threadIdx.x;
                int64_t o = cursor + s_off[k * NW + wave] + (uint32_t)__popcll(mask[k] & lanemask_lt());
                // plain stores: the survivors are read again soon (the
                // bucket maxima and the candidates), from the cache when
                // they are still there
                comp_xy[o] = p[k];
                comp_idx[o] = kPre ? pid[kPre ? k : 0] : (uint32_t)pos;
                keys[o] = key[k];
            }
        }
        // this tile's farthest survivor of this thread, with its output slot
        if (tidx != 0xFFFFFFFFu) {
            const uint32_t tslot = (uint32_t)(cursor + s_off[tgrp] + trank);
            const bool take = (td2 > bd2) | ((td2 == bd2) & (tidx < bidx));
            bd2 = take ? td2 : bd2;
            bidx = take ? tidx : bidx;
            bslot = take ? tslot : bslot;
        }
        cursor += s_total;
        __syncthreads();
    }
    // block results: segment length, farthest survivor, copies of the pivot
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        double od = __shfl_xor(bd2, m);
        uint32_t oi = __shfl_xor(bidx, m);
        uint32_t os = __shfl_xor(bslot, m);
        const bool take = (od > bd2) | ((od == bd2) & (oi < bidx));
        bd2 = take ? od : bd2;
        bidx = take ? oi : bidx;
        bslot = take ? os : bslot;
    }
    uint32_t p0w = wave_sum(p0c);
    if (lane == 0) {
        s_bd2[wave] = bd2;
        s_bidx[wave] = bidx;
        s_bslot[wave] = bslot;
        s_p0[wave] = p0w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double d = s_bd2[0];
        uint32_t bi = s_bidx[0], bs = s_bslot[0], pc = s_p0[0];
        for (int w = 1; w < NW; ++w) {
            const bool take = (s_bd2[w] > d) | ((s_bd2[w] == d) & (s_bidx[w] < bi));
            d = take ? s_bd2[w] : d;
            bi = take ? s_bidx[w] : bi;
            bs = take ? s_bslot[w] : bs;
            pc += s_p0[w];
        }
        blk_d2[blockIdx.x] = d;
        blk_best[2 * blockIdx.x] = bi;
        blk_best[2 * blockIdx.x + 1] = bs;
        seg_count[blockIdx.x] = (uint32_t)(cursor - beg);
        if (pc) atomicAdd(&ds->n_p0, pc);
    }
}

// Learned filter: Step 1's partial extremes and the pre-filter in one pass.
// Block b owns the input range [b*chunk, (b+1)*chunk) (as k_filter1 does)
// and compacts, in input order, the points not strictly inside the
// direction candidates' hull (lo->spoly) into the same range of pre_xy /
// pre_idx.  That hull lies inside the final discard polygon (the hull of
// the candidates and the four extremes), so only points the final test
// would discard are dropped here; the final test then reads the few points
// left instead of the input.  No common error bound is known yet (the
// bounding box comes from this pass), so each orientation test uses its own,
// and a point whose tests float64 cannot settle is kept (the final, exact
// test settles it).
// Points per thread and tile of k_pre: more loads in flight than Steps 2-3
// (the pass writes little).
constexpr int kPreIpt = 8;
constexpr int kPreTile = kF1Block * kPreIpt;

__global__ __launch_bounds__(kF1Block) void k_pre(const double2* __restrict__ xy, int64_t n, int64_t chunk,
                                                  const LearnOut* __restrict__ lo,
                                                  Cand* __restrict__ partial, double2* __restrict__ pre_xy,
                                                  uint32_t* __restrict__ pre_idx,
                                                  uint32_t* __restrict__ pre_count) {
    constexpr int NW = kF1Block / 64;
    constexpr int G = kPreIpt * NW;
    static_assert(G <= 64, "one wave scans the group counts");
    __shared__ uint32_t s_off[G];
    __shared__ uint32_t s_total;
    __shared__ Cand s_c[NW][4];
    __shared__ uint32_t s_flags;
    __shared__ PolyF s_poly;
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    if (threadIdx.x == 0) {
        make_polyf(lo->spoly, s_poly);
        s_flags = 0;
    }
    __syncthreads();
    Cand c[4] = {sentinel(0), sentinel(1), sentinel(2), sentinel(3)};
    uint32_t bad = 0;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = min(n, beg + chunk);
    int64_t cursor = beg;
    double2 nx[kPreIpt];
#pragma unroll
    for (int k = 0; k < kPreIpt; ++k) {
        const int64_t pos = beg + k * kF1Block + threadIdx.x;
        if (pos < end) nx[k] = load_stream(&xy[pos]);
    }
    for (int64_t base = beg; base < end; base += kPreTile) {
        double2 p[kPreIpt];
#pragma unroll
        for (int k = 0; k < kPreIpt; ++k) p[k] = nx[k];
#pragma unroll
        for (int k = 0; k < kPreIpt; ++k) {
            const int64_t pos = base + kPreTile + k * kF1Block + threadIdx.x;
            if (pos < end) nx[k] = load_stream(&xy[pos]);
        }
        uint64_t mask[kPreIpt];
#pragma unroll
        for (int k = 0; k < kPreIpt; ++k) {
            const int64_t pos = base + k * kF1Block + threadIdx.x;
            bool keep = false;
            if (pos < end) {
                const double px = p[k].x, py = p[k].y;
                const bool need = (px <= c[0].x) | (py <= c[1].y) | (px >= c[2].x) | (py >= c[3].y);
                if (need) offer(c, px, py, (int32_t)pos);
                bad |= domain_flags(px) | domain_flags(py);
                keep = !poly_surely_inside_f32(s_poly, px, py);
            }
            mask[k] = __ballot(keep);
            if (lane == 0) s_off[k * NW + wave] = (uint32_t)__popcll(mask[k]);
        }
        __syncthreads();
        if (wave == 0) {
            uint32_t v = lane < G ? s_off[lane] : 0u;
            uint32_t inc = wave_incl_scan(v);
            if (lane < G) s_off[lane] = inc - v;
            if (lane == 63) s_total = inc;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPreIpt; ++k) {
            if ((mask[k] >> lane) & 1ull) {
                const int64_t pos = base + k * kF1Block + threadIdx.x;
                const int64_t o = cursor + s_off[k * NW + wave] + (uint32_t)__popcll(mask[k] & lanemask_lt());
                pre_xy[o] = p[k];
                pre_idx[o] = (uint32_t)pos;
            }
        }
        cursor += s_total;
        __syncthreads();
    }
    reduce4_wave(c);
    if (bad) atomicOr(&s_flags, bad);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s_c[wave][k] = c[k];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = (int)threadIdx.x;
        Cand b = s_c[0][k];
        for (int w = 1; w < NW; ++w) {
            const Cand o = s_c[w][k];
            if (k == 0) take_better<0>(b, o);
            else if (k == 1) take_better<1>(b, o);
            else if (k == 2) take_better<2>(b, o);
            else take_better<3>(b, o);
        }
        b.pad = (int32_t)s_flags;
        partial[(int64_t)blockIdx.x * 4 + k] = b;
    }
    if (threadIdx.x == 0) pre_count[blockIdx.x] = (uint32_t)(cursor - beg);
}

// Step 5 and the segment totals: one block.  The farthest survivor (largest
// d2, then smallest index) over the block partials; the exclusive prefix of
// the segment lengths (seg_off) and their total n_sorted.
__global__ __launch_bounds__(1024) void k_longest(int nblk, const double* __restrict__ blk_d2,
                                                  const uint32_t* __restrict__ blk_best,
                                                  const uint32_t* __restrict__ seg_count,
                                                  uint32_t* __restrict__ seg_off,
                                                  const double2* __restrict__ comp_xy,
                                                  const uint32_t* __restrict__ keys,
                                                  Params* __restrict__ prm,
                                                  DevStatus* __restrict__ ds,
                                                  uint32_t* __restrict__ bmax) {
    __shared__ double s_d[16];
    __shared__ uint32_t s_i[16], s_s[16], s_c[16];
    // the bucketed filter's table of sampled bucket maxima starts empty
    if (bmax)
        for (int i = (int)threadIdx.x; i < 2 * kBuckets; i += 1024) bmax[i] = 0;
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    double d = -1.0;
    uint32_t bi = 0xFFFFFFFFu, bs = 0xFFFFFFFFu;
    for (int t = (int)threadIdx.x; t < nblk; t += 1024) {
        const double od = blk_d2[t];
        const uint32_t oi = blk_best[2 * t];
        const uint32_t os = blk_best[2 * t + 1];
        const bool tk = (od > d) | ((od == d) & (oi < bi));
        d = tk ? od : d;
        bi = tk ? oi : bi;
        bs = tk ? os : bs;
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        double od = __shfl_xor(d, m);
        uint32_t oi = __shfl_xor(bi, m);
        uint32_t os = __shfl_xor(bs, m);
        const bool tk = (od > d) | ((od == d) & (oi < bi));
        d = tk ? od : d;
        bi = tk ? oi : bi;
        bs = tk ? os : bs;
    }
    if (lane == 0) {
        s_d[wave] = d;
        s_i[wave] = bi;
        s_s[wave] = bs;
    }
    // exclusive scan of the segment lengths, 1024 at a time
    uint32_t carry = 0;
    for (int base = 0; base < nblk; base += 1024) {
        const int t = base + (int)threadIdx.x;
        const uint32_t v = t < nblk ? seg_count[t] : 0u;
        uint32_t inc = wave_incl_scan(v);
        __syncthreads();
        if (lane == 63) s_c[wave] = inc;
        __syncthreads();
        uint32_t pre = carry;
        uint32_t tot = 0;
        for (int w = 0; w < 16; ++w) {
            if (w < wave) pre += s_c[w];
            tot += s_c[w];
        }
        if (t < nblk) seg_off[t] = pre + inc - v;
        carry += tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 16; ++w) {
            const bool tk = (s_d[w] > d) | ((s_d[w] == d) & (s_i[w] < bi));
            d = tk ? s_d[w] : d;
            bi = tk ? s_i[w] : bi;
            bs = tk ? s_s[w] : bs;
        }
        ds->n_sorted = carry;
        if (bs != 0xFFFFFFFFu && carry > 0u) {
            double2 q = comp_xy[bs];
            prm->lx = q.x;
            prm->ly = q.y;
            prm->l_idx = (int32_t)bi;
            prm->kl = keys[bs];
            // reference directions of the second round, seen from P_l: toward
            // P_0 (right region) and away from it (left region, a half turn)
            uint32_t tu = turn_key(prm->x0, prm->y0, q.x, q.y);
            prm->turn_u = tu;
            prm->turn_v = tu + 0x80000000u;
            ds->l_slot = bs;
            ds->l_idx = (int32_t)bi;
        }
    }
}

// Dense (key, slot) pairs of the survivors, for the sort of every survivor:
// block b copies segment b to [seg_off[b], seg_off[b] + seg_count[b]).
__global__ __launch_bounds__(256) void k_densify(int64_t chunk, const uint32_t* __restrict__ seg_count,
                                                 const uint32_t* __restrict__ seg_off,
                                                 const uint32_t* __restrict__ keys,
                                                 uint32_t* __restrict__ dkeys,
                                                 uint32_t* __restrict__ dslots) {
    const uint32_t cnt = seg_count[blockIdx.x];
    const uint32_t o = seg_off[blockIdx.x];
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    for (uint32_t i = threadIdx.x; i < cnt; i += 256) {
        dkeys[o + i] = keys[beg + i];
        dslots[o + i] = (uint32_t)(beg + i);
    }
}

// ---------------------------------------------------------------------------
// Steps 6-7, one walk per region as a prefix scan.
//
// Right region (sorted before P_l, walked forward from P_temp = P_0): P_i is
// interior when it is strictly left of P_temp -> P_l, i.e. when
// orient(P_l, P_temp, P_i) < 0; otherwise P_temp <- P_i.  Seen from P_l, the
// directions to P_0 and to the right-region points lie in a half-open
// half-plane, so "B follows A" := orient(P_l, A, B) >= 0 is a total preorder
// there, and the walk's P_temp is always a maximum of everything walked so
// far.  Hence P_i is kept exactly when P_i follows the maximum of
// {P_0, P_1, ..., P_{i-1}}: a max-scan, associative, computed by tiles with
// a decoupled look-back of the running maximum.  The left region (walked
// backward from its last point, discarding points strictly right of
// P_temp -> P_l) is the mirror image with the sign flipped.  Copies of P_l
// (zero direction) only occur at the very end of the left walk and are
// always kept, which the formula reproduces.
// ---------------------------------------------------------------------------
struct Pt {
    double x, y;
    uint32_t s;
};

__device__ inline Pt pt_load(uint32_t slot, const double2* __restrict__ comp, double x0, double y0) {
    Pt p;
    p.s = slot;
    if (slot == kSlotP0) {
        p.x = x0;
        p.y = y0;
    } else if (slot == kSlotNone) {
        p.x = 0.0;
        p.y = 0.0;
    } else {
        double2 v = comp[slot];
        p.x = v.x;
        p.y = v.y;
    }
    return p;
}

// Later of a and b in the region's order (kSlotNone is the identity).
__device__ inline Pt pmax(const Pt& a, const Pt& b, double lx, double ly, int sgn) {
    const bool an = a.s == kSlotNone, bn = b.s == kSlotNone;
    const int o = orient(lx, ly, a.x, a.y, b.x, b.y);
    const bool take_b = an | ((!bn) & (sgn * o >= 0));
    Pt r;
    r.x = take_b ? b.x : a.x;
    r.y = take_b ? b.y : a.y;
    r.s = take_b ? b.s : a.s;
    return r;
}

__device__ inline Pt shfl_pt(const Pt& p, int src) {
    Pt r;
    r.x = __shfl(p.x, src);
    r.y = __shfl(p.y, src);
    r.s = __shfl(p.s, src);
    return r;
}

__device__ inline Pt shfl_up_pt(const Pt& p, int d) {
    Pt r;
    r.x = __shfl_up(p.x, d);
    r.y = __shfl_up(p.y, d);
    r.s = __shfl_up(p.s, d);
    return r;
}

__device__ inline Pt shfl_xor_pt(const Pt& p, int m) {
    Pt r;
    r.x = __shfl_xor(p.x, m);
    r.y = __shfl_xor(p.y, m);
    r.s = __shfl_xor(p.s, m);
    return r;
}

// Look-back of the running maximum; one wave.  `initial` is the value before
// tile 0 (P_0 for the right region, none for the left region).
__device__ Pt lookback_max(uint64_t* stat, uint32_t t, const Pt& agg, uint32_t initial,
                           const double2* __restrict__ comp, double x0, double y0, double lx,
                           double ly, int sgn, uint32_t epoch) {
    const uint32_t lane = __lane_id();
    Pt pre = pt_load(initial, comp, x0, y0);
    if (t == 0) {
        Pt inc = pmax(pre, agg, lx, ly, sgn);
        if (lane == 0) stat_store(&stat[0], stat_pack(epoch, kStatInclusive, inc.s));
        return pre;
    }
    if (lane == 0) stat_store(&stat[t], stat_pack(epoch, kStatAggregate, agg.s));
    Pt acc;
    acc.s = kSlotNone;
    acc.x = acc.y = 0.0;
    int64_t top = (int64_t)t - 1;
    for (;;) {
        int64_t me = top - (int64_t)lane;
        uint32_t f = kStatInclusive, v = initial;
        if (me >= 0) {
            uint64_t w = stat_load(&stat[me]);
            f = stat_flag(w, epoch);
            v = stat_value(w);
        }
        uint64_t incl = __ballot(f == kStatInclusive);
        uint64_t notready = __ballot(f == 0u);
        uint32_t first = incl ? (uint32_t)(__ffsll((unsigned long long)incl) - 1) : 64u;
        uint64_t upto = first >= 63u ? ~0ull : ((2ull << first) - 1ull);
        if (notready & upto) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        Pt mine = pt_load(lane <= first ? v : kSlotNone, comp, x0, y0);
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) mine = pmax(mine, shfl_xor_pt(mine, m), lx, ly, sgn);
        acc = pmax(mine, acc, lx, ly, sgn);
        if (first < 64u) break;
        top -= 64;
    }
    Pt inc = pmax(acc, agg, lx, ly, sgn);
    if (lane == 0) stat_store(&stat[t], stat_pack(epoch, kStatInclusive, inc.s));
    return acc;
}

__global__ __launch_bounds__(kR2Block) void k_round2_scan(
    const uint32_t* __restrict__ slots, const double2* __restrict__ comp,
    const Params* __restrict__ prm, const DevStatus* __restrict__ ds, uint8_t* __restrict__ keep,
    uint64_t* __restrict__ stat, Counters* __restrict__ ctr, uint32_t epoch) {
    constexpr int NW = kR2Block / 64;
    __shared__ uint32_t s_ticket;
    __shared__ Pt s_wave[NW];
    __shared__ Pt s_pre;

    const uint32_t ms = ds->n_sorted;
    const uint32_t lp = ds->l_pos;
    const uint32_t nR = ms > 0 ? lp : 0u;
    const uint32_t nL = ms > 0 ? ms - 1u - lp : 0u;
    const uint32_t ntR = (nR + kR2Tile - 1) / kR2Tile;
    const uint32_t ntL = (nL + kR2Tile - 1) / kR2Tile;
    const uint32_t ntiles = ntR + ntL;
    const double x0 = prm->x0, y0 = prm->y0, lx = prm->lx, ly = prm->ly;
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    if (blockIdx.x == 0 && threadIdx.x == 0 && ms > 0) keep[lp] = 1;
    if (blockIdx.x >= ntiles) return;

    uint32_t* counter = &ctr->ticket[16 * kTicketRound2];
    for (uint32_t t = next_tile(counter, ntiles, &s_ticket); t < ntiles;
         t = next_tile(counter, ntiles, &s_ticket)) {
        const bool right = t < ntR;
        const uint32_t rt = right ? t : t - ntR;
        const int sgn = right ? 1 : -1;
        const uint32_t cnt = min((uint32_t)kR2Tile, (right ? nR : nL) - rt * kR2Tile);
        uint64_t* st = right ? stat : stat + ntR;
        // this thread's items, consecutive in walk order
        Pt it[kR2Ipt];
        uint32_t pos[kR2Ipt];
        Pt m;
        m.s = kSlotNone;
        m.x = m.y = 0.0;
#pragma unroll
        for (int k = 0; k < kR2Ipt; ++k) {
            uint32_t w = threadIdx.x * kR2Ipt + k;
            uint32_t g = rt * kR2Tile + w;
            pos[k] = right ? g : ms - 1u - g;
            it[k].s = kSlotNone;
            it[k].x = it[k].y = 0.0;
            if (w < cnt) it[k] = pt_load(slots[pos[k]], comp, x0, y0);
        }
#pragma unroll
        for (int k = 0; k < kR2Ipt; ++k) m = pmax(m, it[k], lx, ly, sgn);
        // block exclusive scan of the thread maxima
        Pt inc = m;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            Pt o = shfl_up_pt(inc, d);
            if (lane >= d) inc = pmax(o, inc, lx, ly, sgn);
        }
        Pt ex = shfl_up_pt(inc, 1);
        if (lane == 0) {
            ex.s = kSlotNone;
            ex.x = ex.y = 0.0;
        }
        if (lane == 63) s_wave[wave] = inc;
        __syncthreads();
        Pt wpre;
        wpre.s = kSlotNone;
        wpre.x = wpre.y = 0.0;
        for (int w = 0; w < wave; ++w) wpre = pmax(wpre, s_wave[w], lx, ly, sgn);
        ex = pmax(wpre, ex, lx, ly, sgn);
        if (wave == 0) {
            Pt agg = s_wave[0];
            for (int w = 1; w < NW; ++w) agg = pmax(agg, s_wave[w], lx, ly, sgn);
            Pt pre = lookback_max(st, rt, agg, right ? kSlotP0 : kSlotNone, comp, x0, y0, lx,
                                  ly, sgn, epoch);
            if (lane == 0) s_pre = pre;
        }
        __syncthreads();
        Pt run = pmax(s_pre, ex, lx, ly, sgn);
#pragma unroll
        for (int k = 0; k < kR2Ipt; ++k) {
            uint32_t w = threadIdx.x * kR2Ipt + k;
            if (w < cnt) {
                bool kp = run.s == kSlotNone ||
                          sgn * orient(lx, ly, run.x, run.y, it[k].x, it[k].y) >= 0;
                keep[pos[k]] = kp ? 1 : 0;
                run = pmax(run, it[k], lx, ly, sgn);
            }
        }
        __syncthreads();
    }
}

// Steps 6-7 with the paper's subsets (Section 3.4): one thread walks one
// subset sequentially.  Every subset restarts P_temp at its first point in
// walking order (kept untested), except the right region's first subset,
// which starts from P_0 as Figure 2 does.
__global__ __launch_bounds__(256) void k_round2_chunks(int64_t chunk, const uint32_t* __restrict__ slots,
                                                       const double2* __restrict__ comp,
                                                       const Params* __restrict__ prm,
                                                       const DevStatus* __restrict__ ds,
                                                       uint8_t* __restrict__ keep) {
    const int64_t ms = ds->n_sorted;
    if (ms == 0) return;
    const int64_t lp = ds->l_pos;
    const int64_t mR = lp, mL = ms - 1 - lp;
    auto clen = [&](int64_t m) -> int64_t {
        if (m < 1) return 1;
        if (chunk == 0) return m;
        if (chunk < 0) return (m + 1023) / 1024;
        return chunk;
    };
    const int64_t cR = clen(mR), cL = clen(mL);
    const int64_t nchR = mR > 0 ? (mR + cR - 1) / cR : 0;
    const int64_t nchL = mL > 0 ? (mL + cL - 1) / cL : 0;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double x0 = prm->x0, y0 = prm->y0, lx = prm->lx, ly = prm->ly;
    if (c == 0) keep[lp] = 1;
    if (c < nchR) {
        int64_t s = c * cR, e = min(s + cR, mR);
        double tx = x0, ty = y0;
        int64_t i = s;
        if (c != 0) {
            double2 v = comp[slots[s]];
            tx = v.x;
            ty = v.y;
            keep[s] = 1;
            i = s + 1;
        }
        for (; i < e; ++i) {
            double2 v = comp[slots[i]];
            if (orient(tx, ty, lx, ly, v.x, v.y) > 0) {
                keep[i] = 0;
            } else {
                keep[i] = 1;
                tx = v.x;
                ty = v.y;
            }
        }
    } else if (c < nchR + nchL) {
        int64_t u = c - nchR;
        int64_t top = ms - 1 - u * cL;
        int64_t bot = max(lp + 1, top - cL + 1);
        double2 v = comp[slots[top]];
        double tx = v.x, ty = v.y;
        keep[top] = 1;
        for (int64_t i = top - 1; i >= bot; --i) {
            v = comp[slots[i]];
            if (orient(tx, ty, lx, ly, v.x, v.y) < 0) {
                keep[i] = 0;
            } else {
                keep[i] = 1;
                tx = v.x;
                ty = v.y;
            }
        }
    }
}

// Stable removal of the interior points (the kept ones stay in angular order).
__global__ __launch_bounds__(kCpBlock) void k_compact(
    const uint8_t* __restrict__ keep, const uint32_t* __restrict__ slots,
    const double2* __restrict__ comp, const uint32_t* __restrict__ comp_idx,
    double2* __restrict__ out_xy, int32_t* __restrict__ out_idx, DevStatus* __restrict__ ds,
    uint64_t* __restrict__ stat, Counters* __restrict__ ctr, uint32_t epoch) {
    constexpr int NW = kCpBlock / 64;
    static_assert(kCpIpt == 16, "one 16-byte vector of flags per thread");
    __shared__ uint32_t s_ticket;
    __shared__ uint32_t s_wave[NW];
    __shared__ uint32_t s_excl;
    const uint32_t ms = ds->n_sorted;
    const uint32_t ntiles = (ms + kCpTile - 1) / kCpTile;
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    if (blockIdx.x >= ntiles) return;
    uint32_t* counter = &ctr->ticket[16 * kTicketCompact];
    for (uint32_t t = next_tile(counter, ntiles, &s_ticket); t < ntiles;
         t = next_tile(counter, ntiles, &s_ticket)) {
        const uint32_t p0 = t * kCpTile + threadIdx.x * kCpIpt;
        uint4 v = *reinterpret_cast<const uint4*>(keep + p0);
        uint32_t wds[4] = {v.x, v.y, v.z, v.w};
        uint32_t bits = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            uint32_t b = (wds[k >> 2] >> (8 * (k & 3))) & 0xFFu;
            if (b && p0 + k < ms) bits |= 1u << k;
        }
        uint32_t c = __popc(bits);
        uint32_t inc = wave_incl_scan(c);
        if (lane == 63) s_wave[wave] = inc;
        __syncthreads();
        uint32_t wpre = 0, tot = 0;
        for (int w = 0; w < NW; ++w) {
            uint32_t x = s_wave[w];
            if (w < wave) wpre += x;
            tot += x;
        }
        if (wave == 0) {
            uint32_t excl = lookback_sum(stat, t, tot, epoch);
            if (lane == 0) {
                s_excl = excl;
                if (t == ntiles - 1) ds->n_kept = excl + tot;
            }
        }
        __syncthreads();
        uint32_t o = s_excl + wpre + inc - c;
        while (bits) {
            int k = __ffs(bits) - 1;
            bits &= bits - 1;
            uint32_t s = slots[p0 + k];
            out_xy[o] = comp[s];
            out_idx[o] = (int32_t)comp_idx[s];
            ++o;
        }
        __syncthreads();
    }
}

__global__ void k_clear_words(uint64_t* __restrict__ p, size_t words) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void k_debug_orient(const double* __restrict__ abc, int64_t count, int32_t* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const double* q = abc + 6 * i;
    out[i] = orient(q[0], q[1], q[2], q[3], q[4], q[5]);
}

__global__ void k_debug_key(const double* __restrict__ xy, int64_t count, double x0, double y0,
                            uint32_t* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    out[i] = angle_key(xy[2 * i], xy[2 * i + 1], x0, y0);
}

}  // namespace

hipError_t launch_extremes(const double* xy, int64_t n, Cand* partial, int grid, Params* prm,
                           DevStatus* ds, LearnOut* lo, hipStream_t s) {
    const double2* p = reinterpret_cast<const double2*>(xy);
    hipLaunchKernelGGL(k_extremes, dim3(grid), dim3(kExtBlock), 0, s, p, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (lo) {
        hipLaunchKernelGGL(k_extremes_final<true>, dim3(1), dim3(1024), 0, s, partial, grid, prm, ds, lo);
    } else {
        hipLaunchKernelGGL(k_extremes_final<false>, dim3(1), dim3(1024), 0, s, partial, grid, prm, ds, nullptr);
    }
    return hipGetLastError();
}

hipError_t launch_extremes_final(const Cand* partial, int nblocks, Params* prm, DevStatus* ds,
                                 LearnOut* lo, hipStream_t s) {
    if (lo)
        hipLaunchKernelGGL(k_extremes_final<true>, dim3(1), dim3(1024), 0, s, partial, nblocks, prm, ds, lo);
    else
        hipLaunchKernelGGL(k_extremes_final<false>, dim3(1), dim3(1024), 0, s, partial, nblocks, prm, ds,
                           nullptr);
    return hipGetLastError();
}
hipError_t launch_pre(const double* xy, int64_t n, int blocks, const LearnOut* lo, Cand* partial,
                      double2* pre_xy, uint32_t* pre_idx, uint32_t* pre_count, hipStream_t s) {
    if (blocks > kExtGridMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pre, dim3(blocks), dim3(kF1Block), 0, s, reinterpret_cast<const double2*>(xy), n,
                       filter1_chunk(n, blocks), lo, partial, pre_xy, pre_idx, pre_count);
    return hipGetLastError();
}
hipError_t launch_filter1_pre(const double2* pre_xy, const uint32_t* pre_idx, const uint32_t* pre_count,
                              int64_t n, int blocks, const Params* prm, const Poly* poly,
                              double2* comp_xy, uint32_t* comp_idx, uint32_t* keys, uint32_t* seg_count,
                              double* blk_d2, uint32_t* blk_best, DevStatus* ds, hipStream_t s) {
    hipLaunchKernelGGL((k_filter1<true, true>), dim3(blocks), dim3(kF1Block), 0, s, pre_xy, n,
                       filter1_chunk(n, blocks), prm, poly, comp_xy, comp_idx, keys, seg_count, blk_d2,
                       blk_best, ds, pre_idx, pre_count);
    return hipGetLastError();
}
int extremes_grid(int64_t n, int cu_count, int per_cu) {
    int64_t g = std::min<int64_t>((int64_t)cu_count * per_cu, ceil_div(n, kExtBlock * 8));
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, kExtGridMax));
}

int filter1_blocks(int64_t n, int cu_count, int per_cu) {
    int64_t g = std::min<int64_t>((int64_t)cu_count * per_cu, ceil_div(n, kF1Tile));
    return (int)std::max<int64_t>(g, 1);
}

void occupancy_filter(Occupancy& o) {
    // fewer, longer blocks than fit: three per compute unit measured
    // 88-91 us per 20M points against 94-98 us at the six that fit
    o.extremes = std::min(resident_blocks(reinterpret_cast<const void*>(k_extremes), kExtBlock), 3);
    o.filter1 = resident_blocks(reinterpret_cast<const void*>(k_filter1<false>), kF1Block);
    o.filter1_poly = resident_blocks(reinterpret_cast<const void*>(k_filter1<true>), kF1Block);
}

hipError_t launch_clear_words(uint64_t* p, size_t words, hipStream_t s) {
    if (words == 0) return hipSuccess;
    const int grid = (int)std::min<size_t>(1024, (words + 255) / 256);
    hipLaunchKernelGGL(k_clear_words, dim3(grid), dim3(256), 0, s, p, words);
    return hipGetLastError();
}

int64_t filter1_chunk(int64_t n, int blocks) {
    // whole tiles per block keep the loads aligned
    return ceil_div(ceil_div(n, blocks), kF1Tile) * kF1Tile;
}

hipError_t launch_filter1(const double* xy, int64_t n, int blocks, const Params* prm,
                          const Poly* poly, double2* comp_xy, uint32_t* comp_idx, uint32_t* keys,
                          uint32_t* seg_count, double* blk_d2, uint32_t* blk_best, DevStatus* ds,
                          hipStream_t s) {
    if (poly)
        hipLaunchKernelGGL(k_filter1<true>, dim3(blocks), dim3(kF1Block), 0, s,
                           reinterpret_cast<const double2*>(xy), n, filter1_chunk(n, blocks), prm,
                           poly, comp_xy, comp_idx, keys, seg_count, blk_d2, blk_best, ds);
    else
        hipLaunchKernelGGL(k_filter1<false>, dim3(blocks), dim3(kF1Block), 0, s,
                           reinterpret_cast<const double2*>(xy), n, filter1_chunk(n, blocks), prm,
                           poly, comp_xy, comp_idx, keys, seg_count, blk_d2, blk_best, ds);
    return hipGetLastError();
}

hipError_t launch_longest(int blocks, const double* blk_d2, const uint32_t* blk_best,
                          const uint32_t* seg_count, uint32_t* seg_off, const double2* comp_xy,
                          const uint32_t* keys, Params* prm, DevStatus* ds, uint32_t* bmax,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_longest, dim3(1), dim3(1024), 0, s, blocks, blk_d2, blk_best, seg_count,
                       seg_off, comp_xy, keys, prm, ds, bmax);
    return hipGetLastError();
}

hipError_t launch_densify(int64_t n, int blocks, const uint32_t* seg_count, const uint32_t* seg_off,
                          const uint32_t* keys, uint32_t* dkeys, uint32_t* dslots, hipStream_t s) {
    hipLaunchKernelGGL(k_densify, dim3(blocks), dim3(256), 0, s, filter1_chunk(n, blocks), seg_count,
                       seg_off, keys, dkeys, dslots);
    return hipGetLastError();
}

hipError_t launch_round2_scan(int64_t n, const uint32_t* slots, const double2* comp_xy,
                              const Params* prm, const DevStatus* ds, uint8_t* keep, uint64_t* stat,
                              Counters* ctr, uint32_t epoch, int cu_count, hipStream_t s) {
    const int grid = (int)std::min<int64_t>(ceil_div(n, kR2Tile) + 2, 4 * cu_count);
    hipLaunchKernelGGL(k_round2_scan, dim3(grid), dim3(kR2Block), 0, s, slots, comp_xy, prm, ds, keep,
                       stat, ctr, epoch);
    return hipGetLastError();
}

hipError_t launch_round2_chunks(int64_t n, int64_t chunk, const uint32_t* slots,
                                const double2* comp_xy, const Params* prm, const DevStatus* ds,
                                uint8_t* keep, hipStream_t s) {
    int64_t nch;
    if (chunk < 0) nch = 2 * 1024 + 2;
    else if (chunk == 0) nch = 2;
    else nch = ceil_div(n, chunk) + 2;
    int64_t grid = ceil_div(nch, 256);
    hipLaunchKernelGGL(k_round2_chunks, dim3((unsigned)grid), dim3(256), 0, s, chunk, slots,
                       comp_xy, prm, ds, keep);
    return hipGetLastError();
}

hipError_t launch_compact(int64_t n, const uint8_t* keep, const uint32_t* slots,
                          const double2* comp_xy, const uint32_t* comp_idx, double2* out_xy,
                          int32_t* out_idx, DevStatus* ds, uint64_t* stat, Counters* ctr,
                          uint32_t epoch, int cu_count, hipStream_t s) {
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kCpTile), 4 * cu_count));
    hipLaunchKernelGGL(k_compact, dim3(grid), dim3(kCpBlock), 0, s, keep, slots, comp_xy, comp_idx,
                       out_xy, out_idx, ds, stat, ctr, epoch);
    return hipGetLastError();
}

hipError_t launch_debug_orient(const double* abc, int64_t count, int32_t* out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_debug_orient, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s, abc,
                       count, out);
    return hipGetLastError();
}

hipError_t launch_debug_key(const double* xy, int64_t count, double x0, double y0, uint32_t* out,
                            hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_debug_key, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s, xy,
                       count, x0, y0, out);
    return hipGetLastError();
}

}  // namespace hx
