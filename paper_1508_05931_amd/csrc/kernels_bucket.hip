// kernels_bucket.hip - Steps 6-7 of gScan without sorting every survivor.
//
// Figure 2's walk keeps a point exactly when it follows the running maximum
// of everything walked before it in the region's order, "B follows A" being
// orient(P_l, A, B) >= 0 in the right region and <= 0 in the left one (see
// kernels_filter.hip).  Seen from P_l that order is the order of directions
// over a half-open half-plane, so an exact 32-bit direction key kappa (the
// full-turn key of p - P_l, measured from the region's reference direction)
// satisfies: kappa(A) < kappa(B) implies that B strictly follows A.
//
// Split the survivors into coarse angle buckets (top bits of the angle key
// about P_0; the walk visits buckets in key order in the right region and in
// reverse order in the left one).  A point whose kappa is below the largest
// kappa of an earlier bucket is strictly dominated by an earlier point, so the
// walk discards it.  Every point the walk keeps passes this test, and the
// walk's running maximum is always a kept point, so running Figure 2 over the
// passing points alone (the candidates, in exact angular order) keeps exactly
// the same points as running it over all of them.  The candidates are usually
// a few tenths of a percent of the survivors; they are then sorted and
// scanned by the same kernels as the full problem.
#include "exact.hpp"
#include "kernels.hpp"
#include "steps.hpp"

namespace hx {
namespace {

constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
constexpr int kPfBlock = 512;
constexpr int kPfItems = 4;    // points loaded per thread before any is used
constexpr int kPfCap = 4096;   // LDS slots buffered per block before a flush
constexpr int kBmItems = 4;
constexpr uint32_t kBmSample = 8;  // bucket maxima from 1/8 of each segment

__device__ inline Params load_params(const Params* __restrict__ prm) { return *prm; }

// Maxima of kappa per (region, bucket) over a sample: the first
// 1/kBmSample of each segment's survivors.  Each block builds its table in
// LDS, then folds its non-empty entries into bmax (cleared by k_longest)
// with device atomics.  Prefix maxima of a table built from any subset of
// the points are lower bounds of the exact ones, so the candidates they
// select include every point the exact table selects (the one-workgroup
// tail narrows them to exactly those).  Each block takes a contiguous range
// of segments; every thread loads kBmItems points before it uses any of
// them, so enough loads are in flight to cover the memory latency.
__global__ __launch_bounds__(kBmBlock) void k_bucket_max(int64_t chunk, int segs,
                                                        const uint32_t* __restrict__ seg_count,
                                                        const double2* __restrict__ comp_xy,
                                                        const uint32_t* __restrict__ keys,
                                                        const Params* __restrict__ prm,
                                                        uint32_t* __restrict__ bmax) {
    __shared__ uint32_t s_tab[2 * kBuckets];
    for (int i = (int)threadIdx.x; i < 2 * kBuckets; i += kBmBlock) s_tab[i] = 0;
    __syncthreads();
    const Params P = load_params(prm);
    const int spb = (segs + (int)gridDim.x - 1) / (int)gridDim.x;
    const int sg_end = min(segs, ((int)blockIdx.x + 1) * spb);
    for (int sg = (int)blockIdx.x * spb; sg < sg_end; ++sg) {
    // a sample: the first 1/kBmSample of the segment
    const uint32_t beg = (uint32_t)(sg * chunk);
    const uint32_t end = beg + (seg_count[sg] + kBmSample - 1) / kBmSample;
    for (uint32_t base = beg; base < end; base += kBmBlock * kBmItems) {
        double2 p[kBmItems];
        uint32_t k[kBmItems];
#pragma unroll
        for (int u = 0; u < kBmItems; ++u) {
            uint32_t s = base + u * kBmBlock + threadIdx.x;
            if (s < end) {
                p[u] = comp_xy[s];
                k[u] = keys[s];
            }
        }
#pragma unroll
        for (int u = 0; u < kBmItems; ++u) {
            uint32_t s = base + u * kBmBlock + threadIdx.x;
            if (s < end) {
                Cls c = classify(p[u].x, p[u].y, k[u], P);
                if (c.region != 2) atomicMax(&s_tab[c.region * kBuckets + c.bucket], c.kappa);
            }
        }
    }
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < 2 * kBuckets; i += kBmBlock)
        if (s_tab[i]) atomicMax(&bmax[i], s_tab[i]);
}

// Exclusive prefix maxima in walking order: ascending buckets for the right
// region (starting from kappa(P_0) = 0), descending for the left region
// (identity 0).  One block of 1024 threads, four buckets per thread.  Then
// clears the table for the bucket maxima over the candidates, and resets the
// status of the candidate problem.
__global__ __launch_bounds__(1024) void k_bucket_scan(uint32_t* __restrict__ bmax,
                                                      uint32_t* __restrict__ prefix,
                                                      DevStatus* __restrict__ ds2) {
    __shared__ uint32_t s_w[16];
    for (int region = 0; region < 2; ++region)
        bucket_prefix<1024>(bmax + region * kBuckets, prefix + region * kBuckets, region, s_w);
    // every read of bmax precedes the barriers inside bucket_prefix
    for (int i = (int)threadIdx.x; i < 2 * kBuckets; i += 1024) bmax[i] = 0;
    if (threadIdx.x == 0) {
        ds2->flags = 0;
        ds2->huge_runs = 0;
        ds2->n_sorted = 0;
        ds2->n_p0 = 0;
        ds2->l_pos = 0;
        ds2->n_kept = 0;
        ds2->long_runs = 0;
        ds2->l_slot = kNoSlot;
        ds2->n_right = 0;
        ds2->tail_state = kTailDone;
        ds2->n_hull = 0;
        ds2->scan_state = kScanNone;
    }
}

// Candidates: P_l and its copies, and every point whose kappa reaches the
// prefix maximum of its bucket, each with its kappa (all ones for P_l and
// its copies: seen from P_l they have no direction, so the exact test keeps
// each of them; they come last in the left region's walk, where a maximal
// key keeps them too).  Buffered per block in LDS, then appended with one atomic per
// flush (their order does not matter: they are sorted next).  Also the
// bucket maxima over the candidates (`exact`, cleared beforehand) and the
// size of the right region (the points before P_l in angular order).
__global__ __launch_bounds__(kPfBlock) void k_prefilter(
    int64_t chunk, const uint32_t* __restrict__ seg_count,
    const double2* __restrict__ comp_xy, const uint32_t* __restrict__ comp_idx,
    const uint32_t* __restrict__ keys, const Params* __restrict__ prm,
    DevStatus* __restrict__ ds, const uint32_t* __restrict__ prefix,
    double2* __restrict__ cand_xy, uint32_t* __restrict__ cand_idx, uint32_t* __restrict__ cand_key,
    uint32_t* __restrict__ cand_kap, uint32_t* __restrict__ exact, DevStatus* __restrict__ ds2) {
    __shared__ uint32_t s_buf[kPfCap], s_kap[kPfCap];
    __shared__ uint32_t s_n, s_base, s_right;
    if (threadIdx.x == 0) {
        s_n = 0;
        s_right = 0;
    }
    __syncthreads();
    const Params P = load_params(prm);
    const uint32_t lslot = ds->l_slot;
    const uint32_t beg = (uint32_t)(blockIdx.x * chunk);   // one segment per block
    const uint32_t end = beg + seg_count[blockIdx.x];
    auto flush = [&]() {
        __syncthreads();
        const uint32_t cnt = s_n;
        if (threadIdx.x == 0 && cnt) s_base = atomicAdd(&ds2->n_sorted, cnt);
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cnt; i += kPfBlock) {
            uint32_t s = s_buf[i];
            uint32_t o = s_base + i;
            cand_xy[o] = comp_xy[s];
            cand_idx[o] = comp_idx[s];
            cand_key[o] = keys[s];
            cand_kap[o] = s_kap[i];
            if (s == lslot) ds2->l_slot = o;
        }
        __syncthreads();
        if (threadIdx.x == 0) s_n = 0;
        __syncthreads();
    };
    uint32_t nr = 0;
    constexpr uint32_t kStep = kPfBlock * kPfItems;
    for (uint32_t base = beg; base < end; base += kStep) {
        double2 p[kPfItems];
        uint32_t k[kPfItems];
#pragma unroll
        for (int u = 0; u < kPfItems; ++u) {
            const uint32_t s = base + u * kPfBlock + threadIdx.x;
            if (s < end) {
                p[u] = comp_xy[s];
                k[u] = keys[s];
            }
        }
        // classify every item first (with the float32 direction key, within
        // kTurnSlack / 8 of the exact one), then fetch their prefix maxima
        // together (one memory latency per tile, not one per item).  A point
        // is kept unless its key plus kTurnSlack stays below the sampled
        // prefix maximum: then its exact key is below it, and below the
        // exact prefix maximum, so every exact candidate is kept.  Kept
        // points get their exact key.
        Cls c[kPfItems];
        uint32_t pre[kPfItems];
#pragma unroll
        for (int u = 0; u < kPfItems; ++u) {
            const uint32_t s = base + u * kPfBlock + threadIdx.x;
            c[u].region = 2;
            c[u].kappa = 0;
            c[u].bucket = 0;
            if (s < end) c[u] = classify_near(p[u].x, p[u].y, k[u], P.x0, P.y0, P.lx, P.ly, P.kl, P.turn_u, P.turn_v);
        }
#pragma unroll
        for (int u = 0; u < kPfItems; ++u)
            pre[u] = c[u].region < 2 ? prefix[c[u].region * kBuckets + c[u].bucket] : 0u;
#pragma unroll
        for (int u = 0; u < kPfItems; ++u) {
            const uint32_t s = base + u * kPfBlock + threadIdx.x;
            if (s < end) {
                const bool keep = (c[u].region == 2) || ((uint64_t)c[u].kappa + kTurnSlack >= pre[u]);
                nr += c[u].region == 0;
                if (keep) {
                    if (c[u].region < 2) c[u] = classify(p[u].x, p[u].y, k[u], P);
                    const uint32_t at = atomicAdd(&s_n, 1u);
                    s_buf[at] = s;
                    s_kap[at] = c[u].region == 2 ? 0xFFFFFFFFu : c[u].kappa;
                    if (c[u].region < 2 && c[u].kappa != 0u)
                        atomicMax(&exact[c[u].region * kBuckets + c[u].bucket], c[u].kappa);
                }
            }
        }
        __syncthreads();
        if (s_n > (uint32_t)(kPfCap - kStep)) flush();
    }
    flush();
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) nr += __shfl_xor(nr, m);
    if (__lane_id() == 0 && nr) atomicAdd(&s_right, nr);
    __syncthreads();
    if (threadIdx.x == 0 && s_right) atomicAdd(&ds->n_right, s_right);
}

}  // namespace

hipError_t launch_bucket_max(int64_t n, int segs, const uint32_t* seg_count, const double2* comp_xy,
                             const uint32_t* keys, const Params* prm, uint32_t* bmax, int parts,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_bucket_max, dim3(parts), dim3(kBmBlock), 0, s, filter1_chunk(n, segs), segs,
                       seg_count, comp_xy, keys, prm, bmax);
    return hipGetLastError();
}

hipError_t launch_bucket_scan(uint32_t* bmax, uint32_t* prefix, DevStatus* ds2, hipStream_t s) {
    hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(1024), 0, s, bmax, prefix, ds2);
    return hipGetLastError();
}

hipError_t launch_prefilter(int64_t n, int segs, const uint32_t* seg_count, const double2* comp_xy,
                            const uint32_t* comp_idx, const uint32_t* keys, const Params* prm,
                            DevStatus* ds, const uint32_t* prefix, double2* cand_xy,
                            uint32_t* cand_idx, uint32_t* cand_key, uint32_t* cand_kap, uint32_t* exact,
                            DevStatus* ds2, hipStream_t s) {
    hipLaunchKernelGGL(k_prefilter, dim3(segs), dim3(kPfBlock), 0, s, filter1_chunk(n, segs), seg_count,
                       comp_xy, comp_idx, keys, prm, ds, prefix, cand_xy, cand_idx, cand_key, cand_kap,
                       exact, ds2);
    return hipGetLastError();
}

}  // namespace hx
