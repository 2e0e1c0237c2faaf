// kernels_sort.hip - Step 4 of gScan on gfx950: sort of the round-1 survivors
// in ascending angle about the pivot (Sections 2.1 and 3.3).
//
// The survivors carry an exact 32-bit angle key (see exact.hpp): keys are a
// non-decreasing function of the exact angle, and different keys never
// invert two angles.  The sort is therefore
//   1. a stable least-significant-digit radix sort of (key, slot) pairs,
//      four passes of 8 bits, each pass one kernel in the single-pass style
//      of Adinets & Merrill ("Onesweep", 2022): an up-front histogram gives
//      the digit bases of every pass, tiles rank their keys in LDS with
//      wave-level match masks, and per-digit tile prefixes are chained by
//      decoupled look-back;
//   2. the exact order inside runs of equal keys (angle by the exact
//      orientation, then distance along the ray, then index), by one thread
//      for short runs and by one workgroup in LDS for longer ones.
#include "exact.hpp"
#include "kernels.hpp"
#include "records.hpp"

namespace hx {
namespace {

constexpr int kRadix = 256;

__device__ inline uint32_t wave_incl_scan_u32(uint32_t v) {
    const int lane = (int)__lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(v, off);
        if (lane >= off) v += o;
    }
    return v;
}

// Digit histograms of all four passes.  Per-wave LDS histograms (fewer
// collisions on skewed digits), merged per block, added to global memory.
__global__ __launch_bounds__(256) void k_histogram(const uint32_t* __restrict__ keys,
                                                  const DevStatus* __restrict__ ds,
                                                  uint32_t* __restrict__ hist) {
    constexpr int NW = 256 / 64;
    __shared__ uint32_t s_h[NW][4][kRadix];
    const int wave = (int)(threadIdx.x >> 6);
    for (int i = (int)threadIdx.x; i < NW * 4 * kRadix; i += 256) (&s_h[0][0][0])[i] = 0;
    __syncthreads();
    const uint32_t ms = ds->n_sorted;
    const uint32_t stride = gridDim.x * 256u;
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < ms; i += stride) {
        uint32_t k = keys[i];
        atomicAdd(&s_h[wave][0][k & 0xFFu], 1u);
        atomicAdd(&s_h[wave][1][(k >> 8) & 0xFFu], 1u);
        atomicAdd(&s_h[wave][2][(k >> 16) & 0xFFu], 1u);
        atomicAdd(&s_h[wave][3][k >> 24], 1u);
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < 4 * kRadix; i += 256) {
        uint32_t v = 0;
        for (int w = 0; w < NW; ++w) v += (&s_h[w][0][0])[i];
        if (v) atomicAdd(&hist[i], v);
    }
}

// One stable radix pass over bits [8*pass, 8*pass+8).
// Tile layout: wave w owns positions [w*64*IPT, (w+1)*64*IPT) of the tile,
// item k of lane l at w*64*IPT + k*64 + l (coalesced loads, and ranking
// item-major keeps the pass stable).
__global__ __launch_bounds__(kSortBlock) void k_sort_pass(
    int pass, const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
    const uint32_t* __restrict__ hist, const DevStatus* __restrict__ ds,
    uint64_t* __restrict__ stat, Counters* __restrict__ ctr, uint32_t epoch) {
    constexpr int NW = kSortBlock / 64;
    constexpr int IPT = kSortIpt;
    static_assert(kSortBlock == kRadix, "one thread per digit");
    __shared__ uint32_t s_ticket;
    __shared__ uint32_t s_wc[NW][kRadix];     // per-wave digit counters, then wave prefixes
    __shared__ uint32_t s_tl[kRadix];         // tile-local digit offsets
    __shared__ int64_t s_adj[kRadix];         // global destination minus tile-local position
    __shared__ uint32_t s_base[kRadix];       // global digit base of this pass
    __shared__ uint32_t s_wsum[NW];
    __shared__ uint32_t s_keys[kSortTile];
    __shared__ uint32_t s_vals[kSortTile];

    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    const int d = (int)threadIdx.x;  // the digit this thread looks back for
    const uint32_t ms = ds->n_sorted;
    const uint32_t ntiles = (ms + kSortTile - 1) / kSortTile;
    const int shift = 8 * pass;
    if (blockIdx.x >= ntiles) return;

    // exclusive scan of this pass's global histogram: digit bases
    {
        uint32_t h = hist[pass * kRadix + d];
        uint32_t inc = wave_incl_scan_u32(h);
        if (lane == 63) s_wsum[wave] = inc;
        __syncthreads();
        uint32_t pre = 0;
        for (int w = 0; w < wave; ++w) pre += s_wsum[w];
        s_base[d] = pre + inc - h;
        __syncthreads();
    }

    uint32_t* counter = &ctr->ticket[16 * (kTicketSort0 + pass)];
    for (uint32_t t = next_tile(counter, ntiles, &s_ticket); t < ntiles;
         t = next_tile(counter, ntiles, &s_ticket)) {
        for (int w = 0; w < NW; ++w) s_wc[w][d] = 0;
        __syncthreads();
        const uint32_t base = t * kSortTile;
        uint32_t key[IPT], val[IPT], rank[IPT];
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            uint32_t p = base + wave * 64 * IPT + k * 64 + lane;
            key[k] = 0xFFFFFFFFu;
            val[k] = 0;
            if (p < ms) {
                key[k] = keys_in[p];
                val[k] = vals_in ? vals_in[p] : p;
            }
        }
        // wave-level multi-split: rank of each key among equal digits
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            uint32_t p = base + wave * 64 * IPT + k * 64 + lane;
            const bool valid = p < ms;
            uint32_t dig = (key[k] >> shift) & 0xFFu;
            const uint64_t m = match_digit8(dig, valid);
            uint32_t prior = 0;
            if (valid) prior = s_wc[wave][dig];
            uint32_t below = (uint32_t)__popcll(m & lanemask_lt());
            bool leader = valid && below == 0u;
            // all lanes have read their counter before the leaders update it
            __builtin_amdgcn_wave_barrier();
            if (leader) s_wc[wave][dig] = prior + (uint32_t)__popcll(m);
            __builtin_amdgcn_wave_barrier();
            rank[k] = prior + below;
        }
        __syncthreads();
        // thread d: wave prefixes and tile total of digit d
        uint32_t tot = 0;
        for (int w = 0; w < NW; ++w) {
            uint32_t c = s_wc[w][d];
            s_wc[w][d] = tot;
            tot += c;
        }
        // tile-local exclusive offsets over digits
        {
            uint32_t inc = wave_incl_scan_u32(tot);
            if (lane == 63) s_wsum[wave] = inc;
            __syncthreads();
            uint32_t pre = 0;
            for (int w = 0; w < wave; ++w) pre += s_wsum[w];
            s_tl[d] = pre + inc - tot;
        }
        // decoupled look-back of digit d over the previous tiles
        uint32_t excl = 0;
        uint64_t* sd = stat + (size_t)t * kRadix + d;
        if (t == 0) {
            stat_store(sd, stat_pack(epoch, kStatInclusive, tot));
        } else {
            stat_store(sd, stat_pack(epoch, kStatAggregate, tot));
            int64_t j = (int64_t)t - 1;
            while (j >= 0) {
                uint64_t w = stat_load(stat + (size_t)j * kRadix + d);
                uint32_t f = stat_flag(w, epoch);
                if (f == 0u) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += stat_value(w);
                if (f == kStatInclusive) break;
                --j;
            }
            stat_store(sd, stat_pack(epoch, kStatInclusive, excl + tot));
        }
        __syncthreads();
        s_adj[d] = (int64_t)s_base[d] + excl - s_tl[d];
        // scatter into LDS in digit order
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            uint32_t p = base + wave * 64 * IPT + k * 64 + lane;
            if (p < ms) {
                uint32_t dig = (key[k] >> shift) & 0xFFu;
                uint32_t lp = s_tl[dig] + s_wc[wave][dig] + rank[k];
                s_keys[lp] = key[k];
                s_vals[lp] = val[k];
            }
        }
        __syncthreads();
        const uint32_t cnt = min((uint32_t)kSortTile, ms - base);
        for (uint32_t i = threadIdx.x; i < cnt; i += kSortBlock) {
            uint32_t k = s_keys[i];
            uint32_t dig = (k >> shift) & 0xFFu;
            int64_t dst = s_adj[dig] + i;
            keys_out[dst] = k;
            vals_out[dst] = s_vals[i];
        }
        __syncthreads();
    }
}

// Equal-key runs: a run of at most kRunSmall keys is put in exact order by
// the thread at its start (insertion sort); longer runs are listed for
// k_ties_long.  Also records where P_l ends up.
__global__ __launch_bounds__(256) void k_ties(const uint32_t* __restrict__ keys,
                                              uint32_t* __restrict__ slots,
                                              const double2* __restrict__ comp,
                                              const uint32_t* __restrict__ comp_idx,
                                              const Params* __restrict__ prm,
                                              DevStatus* __restrict__ ds,
                                              uint32_t* __restrict__ long_list) {
    const uint32_t ms = ds->n_sorted;
    const uint32_t lslot = ds->l_slot;
    const double x0 = prm->x0, y0 = prm->y0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ms; i += stride) {
        const uint32_t k = keys[i];
        const bool same_prev = i > 0 && keys[i - 1] == k;
        const bool same_next = i + 1 < ms && keys[i + 1] == k;
        if (!same_prev && !same_next) {
            if (slots[i] == lslot) ds->l_pos = i;
            continue;
        }
        if (same_prev) continue;  // handled by the run's first thread
        uint32_t L = 2;
        while (i + L < ms && L <= (uint32_t)kRunSmall && keys[i + L] == k) ++L;
        if (L > (uint32_t)kRunSmall) {
            uint32_t at = atomicAdd(&ds->long_runs, 1u);
            long_list[at] = i;
            continue;
        }
        Rec r[kRunSmall];
        for (uint32_t a = 0; a < L; ++a) r[a] = rec_load(slots[i + a], comp, comp_idx);
        for (uint32_t a = 1; a < L; ++a) {
            Rec v = r[a];
            uint32_t b = a;
            while (b > 0 && rec_less(v, r[b - 1], x0, y0)) {
                r[b] = r[b - 1];
                --b;
            }
            r[b] = v;
        }
        for (uint32_t a = 0; a < L; ++a) {
            slots[i + a] = r[a].slot;
            if (r[a].slot == lslot) ds->l_pos = i + a;
        }
    }
}

// Bitonic sort of one run of at most kRunCap slots in LDS by the exact
// comparator (an index permutation is sorted; padding sorts last).  All
// threads of the block take part.
__device__ void sort_run_lds(uint32_t* __restrict__ run, uint32_t L, const double2* __restrict__ comp,
                             const uint32_t* __restrict__ comp_idx, double x0, double y0,
                             uint32_t lslot, uint32_t pos0, DevStatus* __restrict__ ds,
                             Rec* s_r, uint16_t* s_p) {
    uint32_t P = 1;
    while (P < L) P <<= 1;
    for (uint32_t a = threadIdx.x; a < L; a += blockDim.x) s_r[a] = rec_load(run[a], comp, comp_idx);
    for (uint32_t a = threadIdx.x; a < P; a += blockDim.x) s_p[a] = (uint16_t)a;
    __syncthreads();
    for (uint32_t kk = 2; kk <= P; kk <<= 1) {
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
            for (uint32_t a = threadIdx.x; a < P; a += blockDim.x) {
                uint32_t b = a ^ j;
                if (b > a) {
                    uint32_t ia = s_p[a], ib = s_p[b];
                    bool b_first;
                    if (ia >= L) b_first = ib < L;
                    else if (ib >= L) b_first = false;
                    else b_first = rec_less(s_r[ib], s_r[ia], x0, y0);
                    bool asc = (a & kk) == 0;
                    if (asc ? b_first : !b_first && ia != ib) {
                        s_p[a] = (uint16_t)ib;
                        s_p[b] = (uint16_t)ia;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t a = threadIdx.x; a < L; a += blockDim.x) {
        uint32_t sl = s_r[s_p[a]].slot;
        run[a] = sl;
        if (sl == lslot) ds->l_pos = pos0 + a;
    }
    __syncthreads();
}

// Longer equal-key runs: one workgroup per run.  Runs beyond kRunCap are
// listed for the merge fallback.
__global__ __launch_bounds__(256) void k_ties_long(const uint32_t* __restrict__ keys,
                                                   uint32_t* __restrict__ slots,
                                                   const double2* __restrict__ comp,
                                                   const uint32_t* __restrict__ comp_idx,
                                                   const Params* __restrict__ prm,
                                                   DevStatus* __restrict__ ds,
                                                   const uint32_t* __restrict__ long_list,
                                                   uint32_t* __restrict__ huge_list) {
    __shared__ Rec s_r[kRunCap];
    __shared__ uint16_t s_p[kRunCap];
    __shared__ uint32_t s_len;
    const uint32_t nl = ds->long_runs;
    const uint32_t ms = ds->n_sorted;
    const uint32_t lslot = ds->l_slot;
    const double x0 = prm->x0, y0 = prm->y0;
    for (uint32_t r = blockIdx.x; r < nl; r += gridDim.x) {
        const uint32_t s = long_list[r];
        if (threadIdx.x == 0) {
            // first position after the run (binary search on the sorted keys)
            const uint32_t k = keys[s];
            uint32_t lo = s + 1, hi = ms;
            while (lo < hi) {
                uint32_t mid = lo + (hi - lo) / 2;
                if (keys[mid] == k) lo = mid + 1;
                else hi = mid;
            }
            s_len = lo - s;
        }
        __syncthreads();
        const uint32_t L = s_len;
        if (L > (uint32_t)kRunCap) {
            if (threadIdx.x == 0) {
                uint32_t at = atomicAdd(&ds->huge_runs, 1u);
                huge_list[2 * at] = s;
                huge_list[2 * at + 1] = L;
            }
            __syncthreads();
            continue;
        }
        sort_run_lds(slots + s, L, comp, comp_idx, x0, y0, lslot, s, ds, s_r, s_p);
    }
}

// Merge fallback for a run longer than kRunCap (many points on one ray from
// the pivot, or many copies of one point): every kRunCap-chunk is sorted in
// LDS, then sorted blocks of width w are merged pairwise, one output element
// per thread, by a binary search of its merge-path diagonal.
__global__ __launch_bounds__(256) void k_chunk_sort(uint32_t* __restrict__ run, uint32_t L,
                                                    const double2* __restrict__ comp,
                                                    const uint32_t* __restrict__ comp_idx,
                                                    const Params* __restrict__ prm,
                                                    DevStatus* __restrict__ ds) {
    __shared__ Rec s_r[kRunCap];
    __shared__ uint16_t s_p[kRunCap];
    const uint32_t c0 = blockIdx.x * (uint32_t)kRunCap;
    const uint32_t len = min((uint32_t)kRunCap, L - c0);
    sort_run_lds(run + c0, len, comp, comp_idx, prm->x0, prm->y0, 0xFFFFFFFFu, 0u, ds, s_r, s_p);
}

__global__ __launch_bounds__(256) void k_merge_pass(const uint32_t* __restrict__ in,
                                                    uint32_t* __restrict__ out, uint32_t L,
                                                    uint32_t w, const double2* __restrict__ comp,
                                                    const uint32_t* __restrict__ comp_idx,
                                                    const Params* __restrict__ prm,
                                                    DevStatus* __restrict__ ds, uint32_t pos0) {
    const uint32_t p = blockIdx.x * 256u + threadIdx.x;
    if (p >= L) return;
    const double x0 = prm->x0, y0 = prm->y0;
    const uint32_t pair = p / (2 * w);
    const uint32_t a0 = pair * 2 * w;
    const uint32_t na = min(w, L - a0);
    const uint32_t b0 = a0 + na;
    const uint32_t nb = min(w, L - b0 < L ? L - b0 : 0u);
    const uint32_t d = p - a0;
    // smallest i in [max(0, d-nb), min(d, na)] with A[i] after B[d-i-1]
    uint32_t lo = d > nb ? d - nb : 0u, hi = min(d, na);
    while (lo < hi) {
        uint32_t i = lo + (hi - lo) / 2;
        Rec ra = rec_load(in[a0 + i], comp, comp_idx);
        Rec rb = rec_load(in[b0 + d - i - 1], comp, comp_idx);
        if (rec_less(rb, ra, x0, y0)) hi = i;
        else lo = i + 1;
    }
    const uint32_t i = lo, j = d - lo;
    uint32_t v;
    if (i >= na) v = in[b0 + j];
    else if (j >= nb) v = in[a0 + i];
    else {
        Rec ra = rec_load(in[a0 + i], comp, comp_idx);
        Rec rb = rec_load(in[b0 + j], comp, comp_idx);
        v = rec_less(rb, ra, x0, y0) ? rb.slot : ra.slot;
    }
    out[p] = v;
    if (v == ds->l_slot) ds->l_pos = pos0 + p;
}

}  // namespace

hipError_t launch_histogram(const uint32_t* keys, const DevStatus* ds, uint32_t* hist, int grid,
                            hipStream_t s) {
    hipError_t e = hipMemsetAsync(hist, 0, 4 * kRadix * sizeof(uint32_t), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_histogram, dim3(grid), dim3(256), 0, s, keys, ds, hist);
    return hipGetLastError();
}

hipError_t launch_sort_pass(int64_t n, int pass, const uint32_t* keys_in, const uint32_t* vals_in,
                            uint32_t* keys_out, uint32_t* vals_out, const uint32_t* hist,
                            const DevStatus* ds, uint64_t* stat, Counters* ctr, uint32_t epoch,
                            int cu_count, hipStream_t s) {
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kSortTile), 4 * cu_count));
    hipLaunchKernelGGL(k_sort_pass, dim3(grid), dim3(kSortBlock), 0, s, pass, keys_in, vals_in, keys_out,
                       vals_out, hist, ds, stat, ctr, epoch);
    return hipGetLastError();
}

hipError_t launch_ties(int64_t n, const uint32_t* keys, uint32_t* slots, const double2* comp_xy,
                       const uint32_t* comp_idx, const Params* prm, DevStatus* ds,
                       uint32_t* long_list, hipStream_t s) {
    int64_t grid = ceil_div(n, 256);
    if (grid > 4096) grid = 4096;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_ties, dim3((unsigned)grid), dim3(256), 0, s, keys, slots, comp_xy,
                       comp_idx, prm, ds, long_list);
    return hipGetLastError();
}

hipError_t launch_huge_run(uint32_t* slots, uint32_t* tmp, uint32_t start, uint32_t L,
                           const double2* comp_xy, const uint32_t* comp_idx, const Params* prm,
                           DevStatus* ds, hipStream_t s) {
    uint32_t* run = slots + start;
    uint32_t* other = tmp + start;
    const uint32_t chunks = (L + kRunCap - 1) / kRunCap;
    hipLaunchKernelGGL(k_chunk_sort, dim3(chunks), dim3(256), 0, s, run, L, comp_xy, comp_idx, prm, ds);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t* a = run;
    uint32_t* b = other;
    for (uint32_t w = kRunCap; w < L; w *= 2) {
        hipLaunchKernelGGL(k_merge_pass, dim3((L + 255) / 256), dim3(256), 0, s, a, b, L, w, comp_xy,
                           comp_idx, prm, ds, start);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint32_t* t = a;
        a = b;
        b = t;
    }
    if (a != run) return hipMemcpyAsync(run, a, (size_t)L * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    return hipSuccess;
}

hipError_t launch_ties_long(const uint32_t* keys, uint32_t* slots, const double2* comp_xy,
                            const uint32_t* comp_idx, const Params* prm, DevStatus* ds,
                            const uint32_t* long_list, uint32_t* huge_list, int grid,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_ties_long, dim3(grid), dim3(256), 0, s, keys, slots, comp_xy, comp_idx,
                       prm, ds, long_list, huge_list);
    return hipGetLastError();
}

}  // namespace hx
