// kernels_chain.hip - the four-region variant of Section 5.1 (Table 8's
// comparison method, CudaChain's design built on Akl and Toussaint's
// heuristic), sharing Steps 1-2 with gScan.
//
// After the quadrilateral of Steps 1-2, a survivor strictly outside edge k of
// the cycle P_minx -> P_miny -> P_maxx -> P_maxy -> P_minx (the first such
// edge) belongs to region k.  In region k the coordinates rotated by -90
// degrees k times, (u, v) = (x, y), (y, -x), (-x, -y), (-y, x), put the
// region in the lower-left position: its hull chain runs from corner k to
// corner k+1 with u rising and v falling.  Each region is ordered by
// (u, v, index) and walked, keeping a point only when its v is strictly below
// every v before it (the second round by coordinate comparisons); the final
// hull is one stack scan per region over corner k, the kept points and
// corner k+1 (the paper's second stage, on the host).
//
// Sorting every region survivor is not needed to find the kept points.
// Region k's u range [u(corner k), u(corner k+1)] is cut into kChainBuckets
// buckets by a monotone float64 map of u, so a point of an earlier bucket
// always precedes a point of a later one.  A kept point has v below every v
// of every earlier bucket, so v < (minimum of v over the earlier buckets) is
// necessary: only those candidates are sorted and walked.  Walking only the
// candidates keeps the same points: the smallest v before any point is first
// reached at a point kept by the full walk, which passes the bucket test.
//
// Kernels: two passes over the input (the first takes each bucket's minimum
// of v with device atomics, issued only where a point lowers the value it
// reads; the second appends the candidates), a prefix of the bucket minima,
// a grouping of the candidates by bucket, and one workgroup per region that
// sorts the candidates exactly in LDS, chunk by chunk along the buckets, and
// walks them with the running minimum carried from chunk to chunk.
#include <hip/hip_runtime.h>

#include "exact.hpp"
#include "kernels.hpp"

namespace hx {
namespace {

constexpr int kCB = kChainBuckets;
constexpr int kPassBlock = 256;
constexpr int kPassU = 4;
constexpr int kSample = 8;  // pass 0 reads one block of points in kSample
constexpr int kCandBuf = 2048;  // pass 1: candidates buffered per block
constexpr int kTailT = 1024;
constexpr uint64_t kKeyEmpty = ~0ull;

// Order-preserving map of a float64 to 64 bits (-0 taken as +0).
__device__ inline uint64_t key_of(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v + 0.0);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ inline double value_of(uint64_t k) {
    const uint64_t b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    return __longlong_as_double((long long)b);
}

__device__ inline void rot_uv(int r, double x, double y, double& u, double& v) {
    u = r == 0 ? x : r == 1 ? y : r == 2 ? -x : -y;
    v = r == 0 ? y : r == 1 ? -x : r == 2 ? -y : x;
}

// Per-call constants of the region test and the bucket map (kept in LDS:
// they are indexed by the point's region).
struct Regions {
    double cx[4], cy[4];     // P_minx, P_miny, P_maxx, P_maxy (with repeats)
    double lo[4], scale[4];  // bucket = floor((u - lo) * scale), clamped
    double qx[4], qy[4], ex[4], ey[4];  // the distinct corners' quadrilateral
    double qb;               // float64 edge-test bound (every point in the Step-1 box)
    int nc;                  // distinct corners
    int none;                // domain error: every point is refused
};

// Thread 0 fills R; the caller synchronises.
__device__ inline void load_regions(const Params* __restrict__ prm, Regions& R) {
    if (threadIdx.x != 0) return;
    for (int k = 0; k < 4; ++k) {
        R.cx[k] = prm->ext[k].x;
        R.cy[k] = prm->ext[k].y;
        R.qx[k] = prm->qx[k];
        R.qy[k] = prm->qy[k];
        R.ex[k] = prm->ex[k];
        R.ey[k] = prm->ey[k];
    }
    for (int k = 0; k < 4; ++k) {
        double ul, vl, uh, vh;
        rot_uv(k, R.cx[k], R.cy[k], ul, vl);
        rot_uv(k, R.cx[(k + 1) & 3], R.cy[(k + 1) & 3], uh, vh);
        R.lo[k] = ul;
        R.scale[k] = uh > ul ? (double)kCB / (uh - ul) : 0.0;
    }
    R.qb = prm->qbound;
    R.nc = prm->ncorner;
    R.none = prm->flags != 0u ? 1 : 0;
}

// -1: strictly inside the quadrilateral (discarded by round 1); 0..3: the
// first edge k of the corner cycle with p strictly right of it (outside);
// 4: on the quadrilateral's boundary.
__device__ inline int region_of(const Regions& R, double x, double y) {
    int o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int k1 = (k + 1) & 3;
        const double l = (R.cx[k1] - R.cx[k]) * (y - R.cy[k]);
        const double r = (R.cy[k1] - R.cy[k]) * (x - R.cx[k]);
        const double det = l - r;
        o[k] = det > R.qb ? 1 : (-det > R.qb ? -1 : orient(R.cx[k], R.cy[k], R.cx[k1], R.cy[k1], x, y));
    }
    const bool inside = R.nc == 4 ? (o[0] > 0 && o[1] > 0 && o[2] > 0 && o[3] > 0)
                                  : quad_inside(R.qx, R.qy, R.ex, R.ey, R.qb, R.nc, x, y);
    if (inside) return -1;
    return o[0] < 0 ? 0 : o[1] < 0 ? 1 : o[2] < 0 ? 2 : o[3] < 0 ? 3 : 4;
}

__device__ inline int bucket_of(const Regions& R, int r, double u) {
    const double t = (u - R.lo[r]) * R.scale[r];
    return t >= (double)(kCB - 1) ? kCB - 1 : t > 0.0 ? (int)t : 0;
}

__device__ inline uint32_t wave_total(uint32_t v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

__global__ void k_chain_clear(ChainTables T) {
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 4 * kCB; i += stride) {
        T.bmin[i] = kKeyEmpty;
        T.count[i] = 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x < sizeof(ChainStatus) / sizeof(uint32_t))
        reinterpret_cast<uint32_t*>(T.st)[threadIdx.x] = 0u;
}

// Pass 0, over a sample (every kSample-th block of kPassBlock points): each
// bucket's minimum of v over the sample.  Those are upper bounds of the
// true minima, so the candidate test of pass 1 (v below the minimum over
// the earlier buckets) keeps a superset of the exact candidates; walking
// that superset keeps the same points (the smallest v before any point is
// first reached at a point kept by the full walk, which passes the test
// whatever the table).  Pass 1, over every point: survivors per region, and
// the candidates, appended with their region and bucket and counted per
// bucket.
template <int kPass>
__global__ __launch_bounds__(kPassBlock) void k_chain_pass(const double2* __restrict__ xy, int64_t n,
                                                           const Params* __restrict__ prm, ChainTables T,
                                                           double2* __restrict__ cand_xy,
                                                           uint32_t* __restrict__ cand_idx,
                                                           uint32_t* __restrict__ cand_rb) {
    __shared__ Regions R;
    load_regions(prm, R);
    __shared__ uint32_t s_cnt[kPassBlock / 64][5];
    // pass 1: this block's candidates (input index, region and bucket),
    // appended to the global list with one atomic per flush
    __shared__ uint32_t s_bi[kCandBuf], s_brb[kCandBuf];
    __shared__ uint32_t s_bn, s_at;
    if (threadIdx.x == 0) s_bn = 0;
    __syncthreads();
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    uint32_t cnt[5] = {0u, 0u, 0u, 0u, 0u};
    auto flush = [&]() {
        __syncthreads();
        const uint32_t nb = s_bn;
        if (threadIdx.x == 0 && nb) s_at = atomicAdd(&T.st->n_cand, nb);
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < nb; j += kPassBlock) {
            const uint32_t i = s_bi[j];
            cand_xy[s_at + j] = xy[i];
            cand_idx[s_at + j] = i;
            cand_rb[s_at + j] = s_brb[j];
        }
        __syncthreads();
        if (threadIdx.x == 0) s_bn = 0;
        __syncthreads();
    };
    // pass 0 takes blocks 0, kSample, 2 kSample, ... of kPassBlock points
    const int64_t step = kPass == 0 ? (int64_t)kSample * kPassBlock : kPassBlock;
    const int64_t stride = (int64_t)gridDim.x * step;
    // kPassU points per thread and turn, their loads issued together
    for (int64_t base = (int64_t)blockIdx.x * step; base < n; base += stride * kPassU) {
        if (kPass == 1) {
            // every thread reads the same fill level (nobody appends between
            // the two barriers), so all of them flush or none
            __syncthreads();
            const bool full = s_bn + kPassBlock * kPassU > (uint32_t)kCandBuf;
            __syncthreads();
            if (full) flush();
        }
        double2 pu[kPassU];
#pragma unroll
        for (int q = 0; q < kPassU; ++q) {
            const int64_t i = base + q * stride + threadIdx.x;
            pu[q] = i < n && !R.none ? load_stream(&xy[i]) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int q = 0; q < kPassU; ++q) {
            const int64_t i = base + q * stride + threadIdx.x;
            const double2 p = pu[q];
            int r = -1;
            double u = 0.0, v = 0.0;
            if (i < n && !R.none) r = region_of(R, p.x, p.y);
            if (kPass == 0) {
                if (r >= 0 && r < 4) {
                    rot_uv(r, p.x, p.y, u, v);
                    const int b = bucket_of(R, r, u);
                    const uint64_t key = key_of(v);
                    uint64_t* cell = &T.bmin[r * kCB + b];
                    // a plain read: the value only falls, so a stale one
                    // costs at most an atomic that changes nothing
                    if (key < *cell)
                        __hip_atomic_fetch_min(cell, key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            } else {
                cnt[0] += r == 0;
                cnt[1] += r == 1;
                cnt[2] += r == 2;
                cnt[3] += r == 3;
                cnt[4] += r == 4;
                bool cand = false;
                int b = 0;
                if (r >= 0 && r < 4) {
                    rot_uv(r, p.x, p.y, u, v);
                    b = bucket_of(R, r, u);
                    cand = v < T.prefix[r * kCB + b];
                }
                const uint64_t mask = __ballot(cand);
                if (mask) {
                    uint32_t at = 0;
                    const int leader = __ffsll((unsigned long long)mask) - 1;
                    if (lane == leader) at = atomicAdd(&s_bn, (uint32_t)__popcll(mask));
                    at = __shfl(at, leader);
                    if (cand) {
                        const uint32_t o = at + (uint32_t)__popcll(mask & lanemask_lt());
                        s_bi[o] = (uint32_t)i;
                        s_brb[o] = ((uint32_t)r << 16) | (uint32_t)b;
                    }
                }
            }
        }
    }
    if (kPass == 1) {
        flush();
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const uint32_t t = wave_total(cnt[k]);
            if (lane == 0) s_cnt[wave][k] = t;
        }
        __syncthreads();
        if (threadIdx.x < 5) {
            uint32_t t = 0;
            for (int w = 0; w < kPassBlock / 64; ++w) t += s_cnt[w][threadIdx.x];
            if (t) {
                if (threadIdx.x < 4) atomicAdd(&T.st->n_region[threadIdx.x], t);
                atomicAdd(&T.st->m1, t);
            }
        }
    }
}

// The two table scans, by tiles of kScanTile entries (kTiles in all, a
// region's tiles consecutive).  kPhase 0: exclusive prefix minima of the
// bucket minima within each region (T.prefix); kPhase 1: the candidates'
// grouping offsets, exclusive sums of the per-bucket counts over (region,
// bucket) (T.offset, T.cursor, and the total at T.offset[4 kChainBuckets]).
// k_chain_tiles: each tile's minimum or sum; k_chain_scan: one block per
// tile, its carry from the earlier tiles' results, then the tile's scan.
constexpr int kScanTile = 1024;
constexpr int kTiles = 4 * kCB / kScanTile;
constexpr int kTilesPerRegion = kCB / kScanTile;
static_assert(kTiles <= 1024, "one thread per tile in the carry");

__device__ inline double bucket_min(const ChainTables& T, int e) {
    const uint64_t k = T.bmin[e];
    return k == kKeyEmpty ? __builtin_inf() : value_of(k);
}

template <int kPhase>
__global__ __launch_bounds__(kScanTile) void k_chain_tiles(ChainTables T) {
    __shared__ double s_m[kScanTile / 64];
    __shared__ uint32_t s_s[kScanTile / 64];
    const int tid = (int)threadIdx.x, lane = (int)__lane_id(), wave = tid >> 6;
    const int e = (int)blockIdx.x * kScanTile + tid;
    if (kPhase == 0) {
        double m = bucket_min(T, e);
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) m = fmin(m, __shfl_xor(m, d));
        if (lane == 0) s_m[wave] = m;
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < kScanTile / 64; ++w) m = fmin(m, s_m[w]);
            T.tile_min[blockIdx.x] = m;
        }
    } else {
        uint32_t c = wave_total(T.count[e]);
        if (lane == 0) s_s[wave] = c;
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < kScanTile / 64; ++w) c += s_s[w];
            T.tile_sum[blockIdx.x] = c;
        }
    }
}

template <int kPhase>
__global__ __launch_bounds__(kScanTile) void k_chain_scan(ChainTables T) {
    __shared__ double s_m[kScanTile / 64];
    __shared__ uint32_t s_s[kScanTile / 64];
    __shared__ double s_carry_m;
    __shared__ uint32_t s_carry_s;
    const int tid = (int)threadIdx.x, lane = (int)__lane_id(), wave = tid >> 6;
    const int tile = (int)blockIdx.x;
    const int e = tile * kScanTile + tid;
    // the carry: wave 0 folds the earlier tiles (of the region, for minima)
    if (wave == 0) {
        const int first = kPhase == 0 ? (tile / kTilesPerRegion) * kTilesPerRegion : 0;
        double m = __builtin_inf();
        uint32_t c = 0;
        for (int t = first + lane; t < tile; t += 64) {
            if (kPhase == 0) m = fmin(m, T.tile_min[t]);
            else c += T.tile_sum[t];
        }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) {
            m = fmin(m, __shfl_xor(m, d));
            c += __shfl_xor(c, d);
        }
        if (lane == 0) {
            s_carry_m = m;
            s_carry_s = c;
        }
    }
    if (kPhase == 0) {
        const double v = bucket_min(T, e);
        double inc = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double o = __shfl_up(inc, d);
            if (lane >= d) inc = fmin(inc, o);
        }
        if (lane == 63) s_m[wave] = inc;
        __syncthreads();
        double ex = __shfl_up(inc, 1);
        if (lane == 0) ex = __builtin_inf();
        for (int w = 0; w < wave; ++w) ex = fmin(ex, s_m[w]);
        T.prefix[e] = fmin(ex, s_carry_m);
    } else {
        const uint32_t v = T.count[e];
        uint32_t inc = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(inc, d);
            if (lane >= d) inc += o;
        }
        if (lane == 63) s_s[wave] = inc;
        __syncthreads();
        uint32_t ex = inc - v;
        for (int w = 0; w < wave; ++w) ex += s_s[w];
        ex += s_carry_s;
        T.offset[e] = ex;
        T.cursor[e] = ex;
        if (e == 4 * kCB - 1) T.offset[4 * kCB] = ex + v;
    }
}

// The bucket minima folded over the candidates too (into the sampled
// table): the smallest v of the earlier buckets is attained at a candidate,
// so the prefix of this table is the exact one.
__global__ __launch_bounds__(256) void k_chain_cand_min(ChainTables T, const double2* __restrict__ cand_xy,
                                                        const uint32_t* __restrict__ cand_rb) {
    const uint32_t nc = T.st->n_cand;
    for (uint32_t j = blockIdx.x * 256 + threadIdx.x; j < nc; j += gridDim.x * 256) {
        const uint32_t rb = cand_rb[j];
        const int r = (int)(rb >> 16);
        double u, v;
        rot_uv(r, cand_xy[j].x, cand_xy[j].y, u, v);
        const uint64_t key = key_of(v);
        uint64_t* cell = &T.bmin[r * kCB + (int)(rb & 0xFFFFu)];
        if (key < *cell) __hip_atomic_fetch_min(cell, key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The exact candidates (v below the exact minimum over the earlier buckets):
// marked (bit 31 of cand_rb) and counted per bucket.
__global__ __launch_bounds__(256) void k_chain_count(ChainTables T, const double2* __restrict__ cand_xy,
                                                     uint32_t* __restrict__ cand_rb) {
    const uint32_t nc = T.st->n_cand;
    for (uint32_t j = blockIdx.x * 256 + threadIdx.x; j < nc; j += gridDim.x * 256) {
        const uint32_t rb = cand_rb[j];
        const int r = (int)(rb >> 16);
        const int cell = r * kCB + (int)(rb & 0xFFFFu);
        double u, v;
        rot_uv(r, cand_xy[j].x, cand_xy[j].y, u, v);
        if (v < T.prefix[cell]) {
            cand_rb[j] = rb | 0x80000000u;
            atomicAdd(&T.count[cell], 1u);
        }
    }
}

// Candidates grouped by (region, bucket); the order inside a bucket is
// whatever the atomics give (the tail sorts exactly).
__global__ __launch_bounds__(256) void k_chain_group(ChainTables T, const double2* __restrict__ cand_xy,
                                                     const uint32_t* __restrict__ cand_idx,
                                                     const uint32_t* __restrict__ cand_rb,
                                                     double2* __restrict__ grp_xy,
                                                     uint32_t* __restrict__ grp_idx) {
    const uint32_t nc = T.st->n_cand;
    for (uint32_t j = blockIdx.x * 256 + threadIdx.x; j < nc; j += gridDim.x * 256) {
        const uint32_t rb = cand_rb[j];
        if (!(rb & 0x80000000u)) continue;  // not an exact candidate
        const uint32_t cell = ((rb >> 16) & 0x7FFFu) * kCB + (rb & 0xFFFFu);
        const uint32_t o = atomicAdd(&T.cursor[cell], 1u);
        grp_xy[o] = cand_xy[j];
        grp_idx[o] = cand_idx[j];
    }
}

struct TailLds {
    double x[kChainCap], y[kChainCap];
    uint32_t idx[kChainCap];
    uint16_t perm[kChainCap];
    double wmin[kTailT / 64];
    uint32_t wsum[kTailT / 64];
    uint32_t misc[4];
};

// (u, v, index) order of two loaded candidates of region r.
__device__ inline bool before(const TailLds& S, int r, int a, int b) {
    double ua, va, ub, vb;
    rot_uv(r, S.x[a], S.y[a], ua, va);
    rot_uv(r, S.x[b], S.y[b], ub, vb);
    if (ua != ub) return ua < ub;
    if (va != vb) return va < vb;
    return S.idx[a] < S.idx[b];
}

// Block-wide exclusive sum of c; *tot receives the total.  All threads.
__device__ inline uint32_t block_excl(TailLds& S, uint32_t c, uint32_t* tot) {
    const int tid = (int)threadIdx.x, lane = (int)__lane_id(), wave = tid >> 6;
    uint32_t ci = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(ci, d);
        if (lane >= d) ci += o;
    }
    __syncthreads();
    if (lane == 63) S.wsum[wave] = ci;
    __syncthreads();
    uint32_t ex = ci - c, t = 0;
    for (int w = 0; w < kTailT / 64; ++w) {
        if (w < wave) ex += S.wsum[w];
        t += S.wsum[w];
    }
    *tot = t;
    return ex;
}

// Sorts S.perm[0, P) (P a power of two, at most kChainCap) by the region's
// order; entries whose slot is not valid (valid(slot) false) sort last.
template <class Valid>
__device__ void sort_slots(TailLds& S, int r, int P, const Valid& valid) {
    const int tid = (int)threadIdx.x;
    for (int kk = 2; kk <= P; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int a = tid; a < P; a += kTailT) {
                const int bb = a ^ j;
                if (bb > a) {
                    const int ia = S.perm[a], ib = S.perm[bb];
                    const bool va = valid(ia), vb = valid(ib);
                    bool b_first;
                    if (!va) b_first = vb;
                    else if (!vb) b_first = false;
                    else b_first = before(S, r, ib, ia);
                    const bool asc = (a & kk) == 0;
                    if (asc ? b_first : (!b_first && ia != ib)) {
                        S.perm[a] = (uint16_t)ib;
                        S.perm[bb] = (uint16_t)ia;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// The walk over the first cn sorted slots (S.perm): a point is kept when its
// v is below every v before it (exclusive prefix minimum, and the carry from
// earlier chunks); kept points appended to out at rbeg + *kept.
__device__ void walk(TailLds& S, int r, int cn, double& carry, uint32_t& kept, uint32_t rbeg,
                     double2* __restrict__ out_xy, int32_t* __restrict__ out_idx) {
    constexpr int E = kChainCap / kTailT;
    const int tid = (int)threadIdx.x, lane = (int)__lane_id(), wave = tid >> 6;
    double vv[E];
    double m = __builtin_inf();
    for (int e = 0; e < E; ++e) {
        const int a = tid * E + e;
        double u = 0.0, v = __builtin_inf();
        if (a < cn) rot_uv(r, S.x[S.perm[a]], S.y[S.perm[a]], u, v);
        vv[e] = v;
        m = fmin(m, v);
    }
    double inc = m;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double o = __shfl_up(inc, d);
        if (lane >= d) inc = fmin(inc, o);
    }
    if (lane == 63) S.wmin[wave] = inc;
    __syncthreads();
    double ex = __shfl_up(inc, 1);
    if (lane == 0) ex = __builtin_inf();
    double cm = __builtin_inf();
    for (int w = 0; w < kTailT / 64; ++w) {
        if (w < wave) ex = fmin(ex, S.wmin[w]);
        cm = fmin(cm, S.wmin[w]);
    }
    ex = fmin(ex, carry);
    uint32_t flags = 0, c = 0;
    for (int e = 0; e < E; ++e) {
        if (vv[e] < ex) {
            flags |= 1u << e;
            ++c;
        }
        ex = fmin(ex, vv[e]);
    }
    uint32_t tot;
    uint32_t o = kept + block_excl(S, c, &tot);
    for (int e = 0; e < E; ++e) {
        if ((flags >> e) & 1u) {
            const int a = S.perm[tid * E + e];
            out_xy[rbeg + o] = make_double2(S.x[a], S.y[a]);
            out_idx[rbeg + o] = (int32_t)S.idx[a];
            ++o;
        }
    }
    kept += tot;
    carry = fmin(carry, cm);
    __syncthreads();
}

// One workgroup per region: the grouped candidates in chunks of whole
// buckets (at most kChainCap each), each sorted in LDS and walked with the
// running minimum of v carried over; the kept points go to out (device) at
// the region's first candidate position, and, when they fit, to host memory.
// A bucket holding more candidates than one chunk (many repeats of a point,
// say) is taken in rounds: each round keeps the kChainCap / 2 smallest
// candidates after the last one walked, merging slices of the bucket into
// the sorted half, and walks them.
__global__ __launch_bounds__(kTailT) void k_chain_tail(ChainTables T, const Params* __restrict__ prm,
                                                       const DevStatus* __restrict__ ds,
                                                       const double2* __restrict__ grp_xy,
                                                       const uint32_t* __restrict__ grp_idx,
                                                       double2* __restrict__ out_xy,
                                                       int32_t* __restrict__ out_idx,
                                                       ChainHost* __restrict__ host,
                                                       double2* __restrict__ host_xy,
                                                       int32_t* __restrict__ host_idx) {
    __shared__ TailLds S;
    constexpr int H = kChainCap / 2;
    const int r = (int)blockIdx.x;
    const int tid = (int)threadIdx.x;
    const uint32_t* off = T.offset + r * kCB;
    const uint32_t rbeg = off[0];
    const uint32_t rend = T.offset[(r + 1) * kCB];
    double carry = __builtin_inf();
    uint32_t kept = 0;
    int b0 = 0;
    while (b0 < kCB && off[b0] < rend) {
        // the longest run of whole buckets from b0 that fits one chunk
        int lo = b0, hi = kCB;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            const uint32_t end = mid == kCB ? rend : off[mid];
            if (end - off[b0] <= (uint32_t)kChainCap) lo = mid;
            else hi = mid - 1;
        }
        if (lo > b0) {
            const uint32_t cb = off[b0], ce = lo == kCB ? rend : off[lo];
            const int cn = (int)(ce - cb);
            b0 = lo;
            if (cn == 0) continue;
            int P = 1;
            while (P < cn) P <<= 1;
            for (int a = tid; a < cn; a += kTailT) {
                const double2 p = grp_xy[cb + (uint32_t)a];
                S.x[a] = p.x;
                S.y[a] = p.y;
                S.idx[a] = grp_idx[cb + (uint32_t)a];
            }
            for (int a = tid; a < P; a += kTailT) S.perm[a] = (uint16_t)a;
            __syncthreads();
            sort_slots(S, r, P, [&](int a) { return a < cn; });
            walk(S, r, cn, carry, kept, rbeg, out_xy, out_idx);
            continue;
        }
        // bucket b0 alone holds more than one chunk
        const uint32_t cb = off[b0], ce = b0 + 1 == kCB ? rend : off[b0 + 1];
        b0 += 1;
        const uint32_t nb = ce - cb;
        uint32_t done = 0;
        double lu = 0.0, lv = 0.0;
        uint32_t li = 0;
        bool have_last = false;
        while (done < nb) {
            int best = 0;  // sorted candidates in slots [0, best)
            // slices of one candidate per thread
            static_assert(kTailT <= H, "a slice fits the free half");
            for (uint32_t sb = cb; sb < ce; sb += kTailT) {
                // this slice's candidates after the last walked one, to [H, H + cin)
                const uint32_t q = sb + (uint32_t)tid;
                bool take = false;
                double2 p = make_double2(0.0, 0.0);
                uint32_t pi = 0;
                if (q < ce) {
                    p = grp_xy[q];
                    pi = grp_idx[q];
                    take = true;
                    if (have_last) {
                        double u, v;
                        rot_uv(r, p.x, p.y, u, v);
                        take = u != lu ? u > lu : v != lv ? v > lv : pi > li;
                    }
                }
                uint32_t cin;
                const uint32_t at = block_excl(S, take ? 1u : 0u, &cin);
                if (take) {
                    S.x[H + at] = p.x;
                    S.y[H + at] = p.y;
                    S.idx[H + at] = pi;
                }
                for (int a = tid; a < kChainCap; a += kTailT) S.perm[a] = (uint16_t)a;
                __syncthreads();
                const int nbst = best, nin = (int)cin;
                sort_slots(S, r, kChainCap,
                           [&](int a) { return a < H ? a < nbst : a - H < nin; });
                // the smallest H (or fewer) become the new sorted half
                const int keep = min(H, nbst + nin);
                static_assert(H == 2 * kTailT, "two kept slots per thread");
                const int a0 = tid, a1 = tid + kTailT;
                double x0 = 0.0, y0 = 0.0, x1 = 0.0, y1 = 0.0;
                uint32_t i0 = 0, i1 = 0;
                if (a0 < keep) {
                    const int sl = S.perm[a0];
                    x0 = S.x[sl];
                    y0 = S.y[sl];
                    i0 = S.idx[sl];
                }
                if (a1 < keep) {
                    const int sl = S.perm[a1];
                    x1 = S.x[sl];
                    y1 = S.y[sl];
                    i1 = S.idx[sl];
                }
                __syncthreads();
                if (a0 < keep) {
                    S.x[a0] = x0;
                    S.y[a0] = y0;
                    S.idx[a0] = i0;
                }
                if (a1 < keep) {
                    S.x[a1] = x1;
                    S.y[a1] = y1;
                    S.idx[a1] = i1;
                }
                __syncthreads();
                best = keep;
            }
            if (best == 0) break;  // every candidate has been walked
            for (int a = tid; a < best; a += kTailT) S.perm[a] = (uint16_t)a;
            __syncthreads();
            walk(S, r, best, carry, kept, rbeg, out_xy, out_idx);
            rot_uv(r, S.x[best - 1], S.y[best - 1], lu, lv);
            li = S.idx[best - 1];
            have_last = true;
            done += (uint32_t)best;
            __syncthreads();
        }
    }
    // to host memory: the kept list when it fits, the counts, and (block 0)
    // the statuses and the corners
    const bool to_host = kept <= (uint32_t)kChainHostCap;
    if (to_host) {
        for (uint32_t k = (uint32_t)tid; k < kept; k += kTailT) {
            host_xy[(uint32_t)r * kChainHostCap + k] = out_xy[rbeg + k];
            host_idx[(uint32_t)r * kChainHostCap + k] = out_idx[rbeg + k];
        }
    }
    if (tid == 0) {
        host->n_kept[r] = kept;
        host->kept_at[r] = rbeg;
        host->on_host[r] = to_host ? 1u : 0u;
        host->overflow[r] = 0u;
        host->n_cand[r] = rend - rbeg;
    }
    if (r == 0) {
        if (tid < (int)(sizeof(DevStatus) / sizeof(uint32_t)))
            reinterpret_cast<uint32_t*>(&host->ds0)[tid] = reinterpret_cast<const uint32_t*>(ds)[tid];
        if (tid < 4) {
            host->cx[tid] = prm->ext[tid].x;
            host->cy[tid] = prm->ext[tid].y;
            host->ci[tid] = prm->ext[tid].i;
            host->n_region[tid] = T.st->n_region[tid];
        }
        if (tid == 0) host->m1 = T.st->m1;
    }
}

}  // namespace

hipError_t launch_chain(const double* xy, int64_t n, const Params* prm, const DevStatus* ds, ChainTables T,
                        double2* cand_xy, uint32_t* cand_idx, uint32_t* cand_rb, double2* grp_xy,
                        uint32_t* grp_idx, double2* out_xy, int32_t* out_idx, ChainHost* host,
                        double2* host_xy, int32_t* host_idx, int grid, hipStream_t s) {
    const double2* p = reinterpret_cast<const double2*>(xy);
    hipLaunchKernelGGL(k_chain_clear, dim3(256), dim3(1024), 0, s, T);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_chain_pass<0>, dim3(grid), dim3(kPassBlock), 0, s, p, n, prm, T, cand_xy,
                       cand_idx, cand_rb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_chain_tiles<0>, dim3(kTiles), dim3(kScanTile), 0, s, T);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_chain_scan<0>, dim3(kTiles), dim3(kScanTile), 0, s, T);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_chain_pass<1>, dim3(grid), dim3(kPassBlock), 0, s, p, n, prm, T, cand_xy,
                       cand_idx, cand_rb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_chain_cand_min, dim3(256), dim3(256), 0, s, T, cand_xy, cand_rb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_chain_tiles<0>, dim3(kTiles), dim3(kScanTile), 0, s, T);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_chain_scan<0>, dim3(kTiles), dim3(kScanTile), 0, s, T);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_chain_count, dim3(256), dim3(256), 0, s, T, cand_xy, cand_rb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_chain_tiles<1>, dim3(kTiles), dim3(kScanTile), 0, s, T);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_chain_scan<1>, dim3(kTiles), dim3(kScanTile), 0, s, T);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_chain_group, dim3(256), dim3(256), 0, s, T, cand_xy, cand_idx, cand_rb, grp_xy,
                       grp_idx);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_chain_tail, dim3(4), dim3(kTailT), 0, s, T, prm, ds, grp_xy, grp_idx, out_xy,
                       out_idx, host, host_xy, host_idx);
    return hipGetLastError();
}

}  // namespace hx
