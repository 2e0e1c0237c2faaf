// kernels_tail.hip - the end of the bucketed path in one workgroup.
//
// After the bucketed filter the second round only has a small candidate set
// left (a few ten thousand points at most on uniform inputs of 20M points).
// For such a set the multi-kernel sort, the look-back scan of Steps 6-7 and
// the compaction are dominated by launch gaps and look-back latency, so two
// independent workgroups of 1024 threads do it, one region each, with the
// region's keys and slots in LDS and every global access issued in batches:
//
//   0. the exact prefix maxima of the region's buckets in walking order,
//      from the bucket maxima over the candidates (the candidates were
//      selected with bucket maxima over a sample of the survivors, so they
//      are a superset of those the exact table selects);
//   1. collect the region's candidates that reach the prefix maximum of
//      their bucket: the right region is every candidate before P_l in the
//      exact angular order of Step 4, the left region is P_l and every
//      candidate after it;
//   2. Step 4 on them: a stable LSD radix sort of (angle key, slot), four
//      passes of 8 bits with wave-level match masks, then the exact order
//      inside runs of equal keys (one thread per short run, the whole
//      workgroup per long run);
//   3. Steps 6-7 as a max-scan (the same formulation as k_round2_scan: a
//      point is kept when it follows, seen from P_l, the maximum of all points
//      walked before it; the right region is walked forward from P_0, the left
//      one backward from its last point, P_l itself is always kept);
//   4. the stable removal: the kept points' slots in angular order per
//      region; k_tail_out (many blocks) then gathers the points and writes
//      the right region, P_l and the left region in order.
//
// More than kTailSlots candidates, a region with more than kTailCap selected
// points, more than kTailLongMax long runs or a run longer than kRunCap sets
// tail_state = kTailOverflow and the host runs the multi-kernel path on all
// candidates instead; the result is the same (points that are not running
// maxima never change the walk).
#include "exact.hpp"
#include "kernels.hpp"
#include "records.hpp"
#include "steps.hpp"

namespace hx {
namespace {

constexpr int kTB = kTailBlock;
constexpr int kTW = kTB / 64;
constexpr int kTI = kTailCap / kTB;     // items per thread
constexpr int kTailLongMax = 64;        // equal-key runs longer than kRunSmall per region
constexpr int kRadixT = 256;
static_assert(kTailCap % kTB == 0, "whole items per thread");
static_assert(kTailCap <= 65536, "slots and counters are 16-bit");
static_assert((size_t)kRunCap * sizeof(Rec) <= (size_t)kTailCap * sizeof(uint32_t),
              "a long run's records fit in the spare key buffer");

struct alignas(16) TailLds {
    uint32_t key[2][kTailCap];     // angle keys, ping-pong
    uint16_t ix[2][kTailCap];      // candidate slots, ping-pong
    uint16_t wc[kTW][kRadixT];     // per-wave digit counters, then wave prefixes
    uint32_t dbase[kRadixT];       // digit totals, then digit bases
    uint32_t wsum[kTW];
    uint32_t longs[kTailLongMax];
    uint32_t wk[kTW], ws[kTW];     // wave aggregates of the round-2 scan
    uint32_t count, nlong, total, runlen;
};

// A walked item: its direction key seen from P_l in the region's walking
// order (larger follows) and its candidate slot (kSlotP0: P_0, whose key is
// 0; kSlotNone: the identity, nothing walked yet).
struct KPt {
    uint32_t k, s;
};
constexpr uint32_t kSlotNone = 0xFFFFFFFFu;
constexpr uint32_t kSlotP0 = 0xFFFFFFFEu;

__device__ inline KPt kpt_none() {
    KPt p;
    p.k = 0;
    p.s = kSlotNone;
    return p;
}

// Whether b follows a in the walk (sgn +1: right region, -1: left region),
// i.e. b becomes the running maximum.  A larger key follows strictly (the
// key is a monotone quantisation of the exact direction); equal keys fall
// back to the exact orientation seen from P_l, collinear counting as
// following.
__device__ inline bool kpt_follows(const KPt& a, const KPt& b, const double2* __restrict__ cand_xy,
                                   double x0, double y0, double lx, double ly, int sgn) {
    if (b.s == kSlotNone) return false;
    if (a.s == kSlotNone) return true;
    if (a.k != b.k) return b.k > a.k;
    if (a.s == b.s) return true;
    const double2 pa = a.s == kSlotP0 ? make_double2(x0, y0) : cand_xy[a.s];
    const double2 pb = b.s == kSlotP0 ? make_double2(x0, y0) : cand_xy[b.s];
    return sgn * orient(lx, ly, pa.x, pa.y, pb.x, pb.y) >= 0;
}

__device__ inline KPt shfl_up_kpt(const KPt& p, int d) {
    KPt r;
    r.k = __shfl_up(p.k, d);
    r.s = __shfl_up(p.s, d);
    return r;
}

__device__ inline uint32_t wsum_incl(uint32_t v) {
    const int lane = (int)__lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(v, off);
        if (lane >= off) v += o;
    }
    return v;
}

// Exclusive block sum (all threads call it; `total` gets the block total).
__device__ inline uint32_t block_excl_sum(uint32_t v, TailLds& S, uint32_t& total) {
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    const uint32_t inc = wsum_incl(v);
    if (lane == 63) S.wsum[wave] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kTW; ++w) {
        const uint32_t x = S.wsum[w];
        pre += w < wave ? x : 0u;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return pre + inc - v;
}

// One workgroup's part (every return is uniform over the workgroup).
__device__ __forceinline__ void tail_body(const double2* __restrict__ cand_xy,
                                          const uint32_t* __restrict__ cand_idx,
                                          const uint32_t* __restrict__ cand_key,
                                          const uint32_t* __restrict__ cand_kap,
                                          const uint32_t* __restrict__ exact,
                                          const Params* __restrict__ prm,
                                          DevStatus* __restrict__ ds2, uint16_t* __restrict__ oslot,
                                          uint32_t* __restrict__ ocount, TailLds& S) {
    const int tid = (int)threadIdx.x;
    const int lane = (int)__lane_id(), wave = tid >> 6;
    const int region = (int)blockIdx.x;  // 0: right region, 1: left region
    const int sgn = region == 0 ? 1 : -1;
    const uint32_t nc = ds2->n_sorted;
    const double x0 = prm->x0, y0 = prm->y0, lx = prm->lx, ly = prm->ly;
    const uint32_t kl = prm->kl;
    const uint32_t lslot = ds2->l_slot;
    auto give_up = [&]() {
        if (tid == 0) ds2->tail_state = kTailOverflow;
    };
    if (nc == 0) {
        if (tid == 0) ocount[region] = 0;
        return;
    }
    if (nc > kTailSlots || lslot >= nc) {
        give_up();
        return;
    }
    const Rec rl = rec_load(lslot, cand_xy, cand_idx);

    // Whether candidate i (angle key `key`) lies in this workgroup's region
    // (right: before P_l in the exact angular order; left: P_l and after),
    // and whether it is a copy of P_l (always kept).
    auto in_region = [&](uint32_t i, uint32_t key, bool& copy) -> bool {
        bool before;
        copy = false;
        if (key != kl) {
            before = key < kl;
        } else if (i == lslot) {
            before = false;
            copy = true;
        } else {
            const Rec r = rec_load(i, cand_xy, cand_idx);
            before = rec_less(r, rl, x0, y0);
            copy = (r.x == rl.x) & (r.y == rl.y);
        }
        return before == (region == 0);
    };

    // ---- 0. the exact prefix maxima of this region: the candidates hold
    //         every running maximum of the walk (they were selected with
    //         lower bounds of the prefix maxima), and every prefix maximum is
    //         attained at a running maximum, so the bucket maxima over the
    //         candidates (`exact`, built while they were selected) give the
    //         exact prefix maxima.  The table lives in the second key buffer
    //         until the sort needs it.
    uint32_t* tab = S.key[1];
    bucket_prefix<kTB>(exact + region * kBuckets, tab, region, S.wsum);
    if (tid == 0) {
        S.count = 0;
        S.nlong = 0;
    }
    __syncthreads();

    // ---- 1. collect this region's candidates that reach the prefix maximum
    //         of their bucket (keys loaded kTI at a time, the next batch
    //         while the current one is placed; one LDS atomic per wave and
    //         batch)
    constexpr uint32_t kStep = (uint32_t)(kTB * kTI);
    uint32_t kv[kTI], kp[kTI];
#pragma unroll
    for (int k = 0; k < kTI; ++k) {
        const uint32_t i = (uint32_t)(k * kTB + tid);
        kv[k] = i < nc ? cand_key[i] : 0u;
        kp[k] = i < nc ? cand_kap[i] : 0u;
    }
    for (uint32_t base = 0; base < nc; base += kStep) {
        uint32_t nkv[kTI], nkp[kTI];
#pragma unroll
        for (int k = 0; k < kTI; ++k) {
            const uint32_t i = base + kStep + (uint32_t)(k * kTB + tid);
            nkv[k] = i < nc ? cand_key[i] : 0u;
            nkp[k] = i < nc ? cand_kap[i] : 0u;
        }
        uint64_t mk[kTI];
        uint32_t tot = 0;
#pragma unroll
        for (int k = 0; k < kTI; ++k) {
            const uint32_t i = base + (uint32_t)(k * kTB + tid);
            bool copy = false;
            const bool mine = i < nc && in_region(i, kv[k], copy) &&
                              (copy || kp[k] >= tab[kv[k] >> (32 - kBucketBits)]);
            mk[k] = __ballot(mine);
            tot += (uint32_t)__popcll(mk[k]);
        }
        if (tot) {
            uint32_t at = 0;
            if (lane == 0) at = atomicAdd(&S.count, tot);
            at = __shfl(at, 0);
            const uint64_t lt = lanemask_lt();
#pragma unroll
            for (int k = 0; k < kTI; ++k) {
                const uint32_t i = base + (uint32_t)(k * kTB + tid);
                const uint32_t q = at + (uint32_t)__popcll(mk[k] & lt);
                if (((mk[k] >> lane) & 1ull) && q < (uint32_t)kTailCap) {
                    S.key[0][q] = kv[k];
                    S.ix[0][q] = (uint16_t)i;
                }
                at += (uint32_t)__popcll(mk[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < kTI; ++k) {
            kv[k] = nkv[k];
            kp[k] = nkp[k];
        }
    }
    __syncthreads();
    const uint32_t cnt = S.count;
    if (cnt > (uint32_t)kTailCap) {
        give_up();
        return;
    }
    // items per thread for this region (the unrolled loops below stop at ipt)
    const int ipt = (int)max(1u, (cnt + kTB - 1) / kTB);

    // ---- 2a. stable LSD radix sort in LDS.  Wave w owns positions
    //          [w*64*ipt, (w+1)*64*ipt), item k of lane l at
    //          w*64*ipt + k*64 + l, ranked item-major (stable).
    int cur = 0;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        for (int j = tid; j < kTW * kRadixT; j += kTB) (&S.wc[0][0])[j] = 0;
        __syncthreads();
        uint32_t key[kTI], rank[kTI];
        uint16_t slot[kTI];
#pragma unroll
        for (int k = 0; k < kTI; ++k) {
            const uint32_t p = (uint32_t)(wave * 64 * ipt + k * 64 + lane);
            const bool valid = k < ipt && p < cnt;
            key[k] = valid ? S.key[cur][p] : 0u;
            slot[k] = valid ? S.ix[cur][p] : (uint16_t)0;
        }
#pragma unroll
        for (int k = 0; k < kTI; ++k) {
            if (k < ipt) {  // uniform: the ballots below need every lane
                const uint32_t p = (uint32_t)(wave * 64 * ipt + k * 64 + lane);
                const bool valid = p < cnt;
                const uint32_t dig = (key[k] >> shift) & 0xFFu;
                const uint64_t m = match_digit8(dig, valid);
                uint32_t prior = 0;
                if (valid) prior = S.wc[wave][dig];
                const uint32_t below = (uint32_t)__popcll(m & lanemask_lt());
                // every lane has read its counter before the leaders move it
                __builtin_amdgcn_wave_barrier();
                if (valid && below == 0u) S.wc[wave][dig] = (uint16_t)(prior + (uint32_t)__popcll(m));
                __builtin_amdgcn_wave_barrier();
                rank[k] = prior + below;
            }
        }
        __syncthreads();
        // digit d: wave prefixes and total
        if (tid < kRadixT) {
            uint32_t tot = 0;
#pragma unroll
            for (int w = 0; w < kTW; ++w) {
                const uint32_t c = S.wc[w][tid];
                S.wc[w][tid] = (uint16_t)tot;
                tot += c;
            }
            S.dbase[tid] = tot;
        }
        __syncthreads();
        // a pass where every key has the digit of position 0 keeps the order
        // (every thread reads the same values; cnt == 0 skips every pass)
        const bool same = S.dbase[(S.key[cur][0] >> shift) & 0xFFu] == cnt;
        __syncthreads();
        if (same) continue;
        if (tid < kRadixT) {
            const uint32_t v = S.dbase[tid];
            const uint32_t inc = wsum_incl(v);
            if (lane == 63) S.wsum[wave] = inc;
            S.dbase[tid] = inc - v;  // wave-local exclusive prefix for now
        }
        __syncthreads();
        if (tid < kRadixT) {
            uint32_t pre = 0;
            for (int w = 0; w < wave; ++w) pre += S.wsum[w];
            S.dbase[tid] += pre;
        }
        __syncthreads();
        const int nxt = cur ^ 1;
#pragma unroll
        for (int k = 0; k < kTI; ++k) {
            const uint32_t p = (uint32_t)(wave * 64 * ipt + k * 64 + lane);
            if (k < ipt && p < cnt) {
                const uint32_t dig = (key[k] >> shift) & 0xFFu;
                const uint32_t q = S.dbase[dig] + S.wc[wave][dig] + rank[k];
                S.key[nxt][q] = key[k];
                S.ix[nxt][q] = slot[k];
            }
        }
        cur = nxt;
        __syncthreads();
    }

    // ---- 2b. exact order inside runs of equal keys
    uint32_t* kk = S.key[cur];
    uint16_t* xx = S.ix[cur];
    for (uint32_t p = (uint32_t)tid; p < cnt; p += kTB) {
        const uint32_t k = kk[p];
        if (p > 0 && kk[p - 1] == k) continue;
        if (!(p + 1 < cnt && kk[p + 1] == k)) continue;
        uint32_t L = 2;
        while (p + L < cnt && L <= (uint32_t)kRunSmall && kk[p + L] == k) ++L;
        if (L > (uint32_t)kRunSmall) {
            const uint32_t at = atomicAdd(&S.nlong, 1u);
            if (at < (uint32_t)kTailLongMax) S.longs[at] = p;
            continue;
        }
        Rec r[kRunSmall];
        for (uint32_t a = 0; a < L; ++a) r[a] = rec_load(xx[p + a], cand_xy, cand_idx);
        for (uint32_t a = 1; a < L; ++a) {
            const Rec v = r[a];
            uint32_t b = a;
            while (b > 0 && rec_less(v, r[b - 1], x0, y0)) {
                r[b] = r[b - 1];
                --b;
            }
            r[b] = v;
        }
        for (uint32_t a = 0; a < L; ++a) xx[p + a] = (uint16_t)r[a].slot;
    }
    __syncthreads();
    const uint32_t nl = S.nlong;
    if (nl > (uint32_t)kTailLongMax) {
        give_up();
        return;
    }
    Rec* s_r = reinterpret_cast<Rec*>(S.key[cur ^ 1]);
    uint16_t* s_p = S.ix[cur ^ 1];
    for (uint32_t j = 0; j < nl; ++j) {
        const uint32_t s = S.longs[j];
        if (tid == 0) {
            uint32_t e = s + 1;
            while (e < cnt && kk[e] == kk[s]) ++e;
            S.runlen = e - s;
        }
        __syncthreads();
        const uint32_t L = S.runlen;
        if (L > (uint32_t)kRunCap) {
            give_up();
            return;
        }
        uint32_t P = 1;
        while (P < L) P <<= 1;
        for (uint32_t a = (uint32_t)tid; a < L; a += kTB) s_r[a] = rec_load(xx[s + a], cand_xy, cand_idx);
        for (uint32_t a = (uint32_t)tid; a < P; a += kTB) s_p[a] = (uint16_t)a;
        __syncthreads();
        for (uint32_t kb = 2; kb <= P; kb <<= 1) {
            for (uint32_t jj = kb >> 1; jj > 0; jj >>= 1) {
                for (uint32_t a = (uint32_t)tid; a < P; a += kTB) {
                    const uint32_t b = a ^ jj;
                    if (b > a) {
                        const uint32_t ia = s_p[a], ib = s_p[b];
                        bool b_first;
                        if (ia >= L) b_first = ib < L;
                        else if (ib >= L) b_first = false;
                        else b_first = rec_less(s_r[ib], s_r[ia], x0, y0);
                        const bool asc = (a & kb) == 0;
                        if (asc ? b_first : (!b_first && ia != ib)) {
                            s_p[a] = (uint16_t)ib;
                            s_p[b] = (uint16_t)ia;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (uint32_t a = (uint32_t)tid; a < L; a += kTB) xx[s + a] = (uint16_t)s_r[s_p[a]].slot;
        __syncthreads();
    }

    // ---- 3. Steps 6-7.  Walk index w = tid*ipt + k.  Right region: position
    //         w, after P_0.  Left region: position cnt-1-w; P_l (position 0)
    //         is not walked and always kept.  Each item is its (kappa, slot):
    //         larger kappa follows, so the scan is integer work except on
    //         equal keys.
    const uint32_t nwalk = region == 0 ? cnt : cnt - 1;
    auto walk_pos = [&](uint32_t w) -> uint32_t { return region == 0 ? w : cnt - 1 - w; };
    auto follows = [&](const KPt& a, const KPt& b) -> bool {
        return kpt_follows(a, b, cand_xy, x0, y0, lx, ly, sgn);
    };
    KPt it[kTI];
#pragma unroll
    for (int k = 0; k < kTI; ++k) {
        const uint32_t w = (uint32_t)(tid * ipt + k);
        it[k].s = (k < ipt && w < nwalk) ? (uint32_t)xx[walk_pos(w)] : kSlotNone;
    }
#pragma unroll
    for (int k = 0; k < kTI; ++k) it[k].k = it[k].s != kSlotNone ? cand_kap[it[k].s] : 0u;
    KPt agg = kpt_none();
#pragma unroll
    for (int k = 0; k < kTI; ++k)
        if (follows(agg, it[k])) agg = it[k];
    KPt inc = agg;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const KPt o = shfl_up_kpt(inc, d);
        if (lane >= d && !follows(o, inc)) inc = o;
    }
    KPt ex = shfl_up_kpt(inc, 1);
    if (lane == 0) ex = kpt_none();
    if (lane == 63) {
        S.wk[wave] = inc.k;
        S.ws[wave] = inc.s;
    }
    __syncthreads();
    KPt run = kpt_none();
    if (region == 0) run.s = kSlotP0;  // kappa(P_0) = 0
    for (int w = 0; w < wave; ++w) {
        KPt o;
        o.k = S.wk[w];
        o.s = S.ws[w];
        if (follows(run, o)) run = o;
    }
    if (follows(run, ex)) run = ex;
    uint32_t kmask = 0;
#pragma unroll
    for (int k = 0; k < kTI; ++k) {
        if (it[k].s != kSlotNone && follows(run, it[k])) {
            kmask |= 1u << k;
            run = it[k];
        }
    }
    // ---- 4. the kept points' slots in angular order: right region in walk
    //         order, left region in reverse (its positions fall as the walk
    //         index rises); k_tail_out gathers and writes them.
    uint32_t tot;
    const uint32_t c = (uint32_t)__popc(kmask);
    const uint32_t excl = block_excl_sum(c, S, tot);
    uint16_t* out = oslot + (size_t)region * kTailCap;
    uint32_t j = excl;
#pragma unroll
    for (int k = 0; k < kTI; ++k) {
        if ((kmask >> k) & 1u) {
            out[region == 0 ? j : tot - 1u - j] = (uint16_t)it[k].s;
            ++j;
        }
    }
    if (tid == 0) ocount[region] = tot;
}

// One workgroup per region.
__global__ __launch_bounds__(kTB) void k_tail(const double2* __restrict__ cand_xy,
                                              const uint32_t* __restrict__ cand_idx,
                                              const uint32_t* __restrict__ cand_key,
                                              const uint32_t* __restrict__ cand_kap,
                                              const uint32_t* __restrict__ exact,
                                              const Params* __restrict__ prm,
                                              DevStatus* __restrict__ ds2,
                                              uint16_t* __restrict__ oslot,
                                              uint32_t* __restrict__ ocount) {
    __shared__ TailLds S;
    tail_body(cand_xy, cand_idx, cand_key, cand_kap, exact, prm, ds2, oslot, ocount, S);
}

// The stable removal's output: the right region's kept points, P_l, the
// left region's, gathered by slot and written to (host) memory by many
// blocks; block 0 also sets the kept count and copies both problem statuses
// (round 1 and candidates) to host memory, so the host needs no copy of its
// own.  Nothing is written but the statuses when the tail gave up.
constexpr int kOutBlock = 256;
constexpr int kOutGrid = 32;

__global__ __launch_bounds__(kOutBlock) void k_tail_out(const double2* __restrict__ cand_xy,
                                                        const uint32_t* __restrict__ cand_idx,
                                                        DevStatus* __restrict__ ds,
                                                        const uint16_t* __restrict__ oslot,
                                                        const uint32_t* __restrict__ ocount,
                                                        double2* __restrict__ out_xy,
                                                        int32_t* __restrict__ out_idx,
                                                        DevStatus* __restrict__ host_ds) {
    const DevStatus* ds2 = ds + 1;
    const bool done = ds2->tail_state == kTailDone;
    const uint32_t nc = ds2->n_sorted;
    const uint32_t nr = done && nc > 0 ? ocount[0] : 0u;
    const uint32_t nl = done && nc > 0 ? ocount[1] : 0u;
    const uint32_t total = done && nc > 0 ? nr + 1u + nl : 0u;
    const uint32_t lslot = ds2->l_slot;
    for (uint32_t q = blockIdx.x * kOutBlock + threadIdx.x; q < total; q += kOutGrid * kOutBlock) {
        const uint32_t sl = q < nr ? (uint32_t)oslot[q]
                          : q == nr ? lslot
                                    : (uint32_t)oslot[kTailCap + (q - nr - 1u)];
        out_xy[q] = cand_xy[sl];
        out_idx[q] = (int32_t)cand_idx[sl];
    }
    if (blockIdx.x == 0 && threadIdx.x < 2 * sizeof(DevStatus) / sizeof(uint32_t)) {
        const int w = (int)threadIdx.x;
        uint32_t v = reinterpret_cast<const uint32_t*>(ds)[w];
        // n_kept of the candidate problem
        if (w == (int)((sizeof(DevStatus) + offsetof(DevStatus, n_kept)) / sizeof(uint32_t)) && done)
            v = total;
        reinterpret_cast<uint32_t*>(host_ds)[w] = v;
    }
}

}  // namespace

hipError_t launch_tail(const double2* cand_xy, const uint32_t* cand_idx, const uint32_t* cand_key,
                       const uint32_t* cand_kap, const uint32_t* exact, const Params* prm,
                       DevStatus* ds, uint16_t* oslot, uint32_t* ocount, double2* out_xy,
                       int32_t* out_idx, DevStatus* host_ds, hipStream_t s) {
    hipLaunchKernelGGL(k_tail, dim3(2), dim3(kTB), 0, s, cand_xy, cand_idx, cand_key, cand_kap, exact,
                       prm, ds + 1, oslot, ocount);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !out_xy) return e;
    return launch_tail_out(cand_xy, cand_idx, ds, oslot, ocount, out_xy, out_idx, host_ds, s);
}

hipError_t launch_tail_out(const double2* cand_xy, const uint32_t* cand_idx, DevStatus* ds,
                           const uint16_t* oslot, const uint32_t* ocount, double2* out_xy,
                           int32_t* out_idx, DevStatus* host_ds, hipStream_t s) {
    hipLaunchKernelGGL(k_tail_out, dim3(kOutGrid), dim3(kOutBlock), 0, s, cand_xy, cand_idx, ds, oslot,
                       ocount, out_xy, out_idx, host_ds);
    return hipGetLastError();
}

}  // namespace hx
