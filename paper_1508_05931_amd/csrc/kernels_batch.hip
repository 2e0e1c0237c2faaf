// kernels_batch.hip - many hulls in one launch (the batched form of the
// hull path).
//
// A persistent kernel: every workgroup takes sets in ticket order (the host
// orders them largest first) and computes one set's hull from start to end:
//
//   Step 1      four extreme points, quadrilateral, pivot P_0 (Section 3.1)
//   Steps 2-3   strict-interior discard, exact angle key, squared distance;
//               survivors appended to the set's workspace
//   Step 5      farthest survivor P_l
//   Steps 6-7   the bucketed second round: per-bucket maxima of the direction
//               key seen from P_l, their prefix maxima, the candidates; then
//               per region a stable radix sort of the candidates (Step 4 on
//               them) with the exact order of equal keys, the walk of Figure 2
//               as a max-scan, and the stable removal
//   Step 8      the Graham scan of the kept points (pivot first): chunks are
//               reduced in parallel to the hull of P_0 and the chunk, which
//               keeps every vertex of the whole hull (in HBM while more than
//               2048 points are left, then in LDS), until one thread
//               finishes the last few; the hull is rotated to its
//               lexicographic minimum and written as set-local indices
//
// Everything a set needs lives in its own slice [offset, offset + n) of the
// workspace arrays, so sets never interfere.  A set whose equal-key runs are
// too long for the workgroup sorter is flagged and finished by the host with
// the single-hull path.
#include "exact.hpp"
#include "kernels.hpp"
#include "records.hpp"
#include "steps.hpp"

namespace hx {
namespace {

constexpr int kBB = kBatchBlock;        // threads per workgroup
constexpr int kBW = kBB / 64;           // waves
constexpr int kBI = 4;                  // items per thread per tile
constexpr int kBT = kBB * kBI;          // items per tile
constexpr int kBLongMax = 64;           // equal-key runs longer than kRunSmall per region
constexpr uint32_t kGLds = 2048;        // Step 8: below this size the points move to LDS
constexpr uint32_t kGOne = 64;          // Step 8: one thread finishes below this size
constexpr uint32_t kNone = 0xFFFFFFFFu;

struct alignas(16) BatchLds {
    union {
        uint32_t tab[2][kBuckets];      // bucket maxima, then exclusive prefix maxima
        struct {
            uint32_t hist[4][256];      // digit counts of the four passes
            uint32_t base[256];         // running destination of each digit
            uint32_t tot[256];          // digit counts of the current tile
            uint16_t wc[kBW][256];      // per-wave digit counters, then wave prefixes
        } rs;
        struct {
            Rec r[kRunCap];
            uint16_t p[kRunCap];
        } run;
        struct {
            double x[kGLds], y[kGLds];  // kept points still in play
            uint32_t pos[kGLds];        // their kept-list positions
            uint16_t a[kGLds], b[kGLds], c[kGLds];
        } gs;
    } u;
    Cand ext[kBW][4];
    double wx[kBW], wy[kBW];
    uint32_t wv[kBW];
    uint32_t wsum[kBW];
    double bd2[kBW];
    uint32_t bidx[kBW], bslot[kBW];
    uint32_t longs[kBLongMax];
    Params P;
    uint32_t flags, cnt, nlong, runlen, lcand, ticket, h, start, hpos;
};

struct BatchArgs {
    const double2* xy;
    const int64_t* offs;
    const int32_t* order;
    int32_t S;
    double2* sv_xy;
    uint32_t* sv_idx;
    uint32_t* sv_key;
    double2* cd_xy;
    uint32_t* cd_idx;
    uint32_t* cd_key;
    uint32_t* ka;
    uint32_t* kb;
    uint32_t* va;
    uint32_t* vb;
    uint8_t* flag;
    int32_t* hull;
    uint32_t* hull_cursor;
    int32_t* h_count;
    int32_t* h_start;
    uint32_t* h_flags;
    Counters* ctr;
};

constexpr uint32_t kSetFallback = kBatchFallback;  // finished by the host (single-hull path)

// ---------------------------------------------------------------------------
// block helpers
// ---------------------------------------------------------------------------
__device__ inline uint32_t bw_incl(uint32_t v) {
    const int lane = (int)__lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(v, off);
        if (lane >= off) v += o;
    }
    return v;
}

// Exclusive block sum; `total` gets the block total.  All threads call it.
__device__ inline uint32_t bexcl(uint32_t v, BatchLds& S, uint32_t& total) {
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    const uint32_t inc = bw_incl(v);
    if (lane == 63) S.wsum[wave] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBW; ++w) {
        const uint32_t x = S.wsum[w];
        pre += w < wave ? x : 0u;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return pre + inc - v;
}

// Append `mine` items to an LDS counter, one atomic per wave; returns this
// lane's position (valid where mine is true).
__device__ inline uint32_t wave_append(bool mine, uint32_t* counter) {
    const int lane = (int)__lane_id();
    const uint64_t m = __ballot(mine);
    if (m == 0) return 0;
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t at = 0;
    if (lane == leader) at = atomicAdd(counter, (uint32_t)__popcll(m));
    return __shfl(at, leader) + (uint32_t)__popcll(m & lanemask_lt());
}

struct BPt {
    double x, y;
    bool v;
};

__device__ inline BPt bpt_none() {
    BPt p;
    p.x = 0.0;
    p.y = 0.0;
    p.v = false;
    return p;
}

// Later of a and b in the walk's order seen from P_l (straight-line selects).
__device__ inline BPt bmax(const BPt& a, const BPt& b, double lx, double ly, int sgn) {
    const int o = orient(lx, ly, a.x, a.y, b.x, b.y);
    const bool take_b = (!a.v) | (b.v & (sgn * o >= 0));
    BPt r;
    r.x = take_b ? b.x : a.x;
    r.y = take_b ? b.y : a.y;
    r.v = take_b ? b.v : a.v;
    return r;
}

__device__ inline BPt shfl_up_bpt(const BPt& p, int d) {
    BPt r;
    r.x = __shfl_up(p.x, d);
    r.y = __shfl_up(p.y, d);
    r.v = __shfl_up((int)p.v, d) != 0;
    return r;
}

// ---------------------------------------------------------------------------
// Step 4 on one region: stable LSD radix sort of (key, slot), the workgroup
// walking the tiles in order.  Returns 0 when the result is in (k0, v0), 1
// when it is in (k1, v1).
// ---------------------------------------------------------------------------
__device__ int wg_radix(BatchLds& S, uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                        uint32_t cnt) {
    const int tid = (int)threadIdx.x, lane = (int)__lane_id(), wave = tid >> 6;
    for (int j = tid; j < 4 * 256; j += kBB) (&S.u.rs.hist[0][0])[j] = 0;
    __syncthreads();
    for (uint32_t i = (uint32_t)tid; i < cnt; i += kBB) {
        const uint32_t k = k0[i];
        atomicAdd(&S.u.rs.hist[0][k & 0xFFu], 1u);
        atomicAdd(&S.u.rs.hist[1][(k >> 8) & 0xFFu], 1u);
        atomicAdd(&S.u.rs.hist[2][(k >> 16) & 0xFFu], 1u);
        atomicAdd(&S.u.rs.hist[3][k >> 24], 1u);
    }
    __syncthreads();
    int cur = 0;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        uint32_t* ks = cur ? k1 : k0;
        uint32_t* vs = cur ? v1 : v0;
        uint32_t* kd = cur ? k0 : k1;
        uint32_t* vd = cur ? v0 : v1;
        // every key with the digit of position 0: the pass keeps the order
        if (cnt == 0 || S.u.rs.hist[pass][(ks[0] >> shift) & 0xFFu] == cnt) continue;
        if (tid < 256) {
            const uint32_t v = S.u.rs.hist[pass][tid];
            const uint32_t inc = bw_incl(v);
            if (lane == 63) S.wsum[wave] = inc;
            S.u.rs.base[tid] = inc - v;
        }
        __syncthreads();
        if (tid < 256) {
            uint32_t pre = 0;
            for (int w = 0; w < wave; ++w) pre += S.wsum[w];
            S.u.rs.base[tid] += pre;
        }
        __syncthreads();
        for (uint32_t t0 = 0; t0 < cnt; t0 += kBT) {
            for (int j = tid; j < kBW * 256; j += kBB) (&S.u.rs.wc[0][0])[j] = 0;
            __syncthreads();
            uint32_t key[kBI], val[kBI], rank[kBI];
#pragma unroll
            for (int k = 0; k < kBI; ++k) {
                const uint32_t p = t0 + (uint32_t)(wave * 64 * kBI + k * 64 + lane);
                key[k] = 0;
                val[k] = 0;
                if (p < cnt) {
                    key[k] = ks[p];
                    val[k] = vs[p];
                }
            }
#pragma unroll
            for (int k = 0; k < kBI; ++k) {
                const uint32_t p = t0 + (uint32_t)(wave * 64 * kBI + k * 64 + lane);
                const bool valid = p < cnt;
                const uint32_t dig = (key[k] >> shift) & 0xFFu;
                const uint64_t m = match_digit8(dig, valid);
                uint32_t prior = 0;
                if (valid) prior = S.u.rs.wc[wave][dig];
                const uint32_t below = (uint32_t)__popcll(m & lanemask_lt());
                __builtin_amdgcn_wave_barrier();
                if (valid && below == 0u) S.u.rs.wc[wave][dig] = (uint16_t)(prior + (uint32_t)__popcll(m));
                __builtin_amdgcn_wave_barrier();
                rank[k] = prior + below;
            }
            __syncthreads();
            if (tid < 256) {
                uint32_t tot = 0;
                for (int w = 0; w < kBW; ++w) {
                    const uint32_t c = S.u.rs.wc[w][tid];
                    S.u.rs.wc[w][tid] = (uint16_t)tot;
                    tot += c;
                }
                S.u.rs.tot[tid] = tot;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kBI; ++k) {
                const uint32_t p = t0 + (uint32_t)(wave * 64 * kBI + k * 64 + lane);
                if (p < cnt) {
                    const uint32_t dig = (key[k] >> shift) & 0xFFu;
                    const uint32_t q = S.u.rs.base[dig] + S.u.rs.wc[wave][dig] + rank[k];
                    kd[q] = key[k];
                    vd[q] = val[k];
                }
            }
            __syncthreads();
            if (tid < 256) S.u.rs.base[tid] += S.u.rs.tot[tid];
            __syncthreads();
        }
        cur ^= 1;
    }
    return cur;
}

// Exact order inside runs of equal keys (sorted keys K, slots V into the
// candidate arrays).  Returns false when a run is too long for the
// workgroup (the set goes to the host).
__device__ bool wg_ties(BatchLds& S, const uint32_t* K, uint32_t* V, uint32_t cnt, const double2* cxy,
                        const uint32_t* cidx, double x0, double y0) {
    const int tid = (int)threadIdx.x;
    if (tid == 0) S.nlong = 0;
    __syncthreads();
    for (uint32_t p = (uint32_t)tid; p < cnt; p += kBB) {
        const uint32_t k = K[p];
        if (p > 0 && K[p - 1] == k) continue;
        if (!(p + 1 < cnt && K[p + 1] == k)) continue;
        uint32_t L = 2;
        while (p + L < cnt && L <= (uint32_t)kRunSmall && K[p + L] == k) ++L;
        if (L > (uint32_t)kRunSmall) {
            const uint32_t at = atomicAdd(&S.nlong, 1u);
            if (at < (uint32_t)kBLongMax) S.longs[at] = p;
            continue;
        }
        Rec r[kRunSmall];
        for (uint32_t a = 0; a < L; ++a) r[a] = rec_load(V[p + a], cxy, cidx);
        for (uint32_t a = 1; a < L; ++a) {
            const Rec v = r[a];
            uint32_t b = a;
            while (b > 0 && rec_less(v, r[b - 1], x0, y0)) {
                r[b] = r[b - 1];
                --b;
            }
            r[b] = v;
        }
        for (uint32_t a = 0; a < L; ++a) V[p + a] = r[a].slot;
    }
    __syncthreads();
    const uint32_t nl = S.nlong;
    if (nl > (uint32_t)kBLongMax) return false;
    for (uint32_t j = 0; j < nl; ++j) {
        const uint32_t s = S.longs[j];
        if (tid == 0) {
            uint32_t e = s + 1;
            while (e < cnt && K[e] == K[s]) ++e;
            S.runlen = e - s;
        }
        __syncthreads();
        const uint32_t L = S.runlen;
        if (L > (uint32_t)kRunCap) return false;
        uint32_t P = 1;
        while (P < L) P <<= 1;
        for (uint32_t a = (uint32_t)tid; a < L; a += kBB) S.u.run.r[a] = rec_load(V[s + a], cxy, cidx);
        for (uint32_t a = (uint32_t)tid; a < P; a += kBB) S.u.run.p[a] = (uint16_t)a;
        __syncthreads();
        for (uint32_t kb = 2; kb <= P; kb <<= 1) {
            for (uint32_t jj = kb >> 1; jj > 0; jj >>= 1) {
                for (uint32_t a = (uint32_t)tid; a < P; a += kBB) {
                    const uint32_t b = a ^ jj;
                    if (b > a) {
                        const uint32_t ia = S.u.run.p[a], ib = S.u.run.p[b];
                        bool b_first;
                        if (ia >= L) b_first = ib < L;
                        else if (ib >= L) b_first = false;
                        else b_first = rec_less(S.u.run.r[ib], S.u.run.r[ia], x0, y0);
                        const bool asc = (a & kb) == 0;
                        if (asc ? b_first : (!b_first && ia != ib)) {
                            S.u.run.p[a] = (uint16_t)ib;
                            S.u.run.p[b] = (uint16_t)ia;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (uint32_t a = (uint32_t)tid; a < L; a += kBB) V[s + a] = S.u.run.r[S.u.run.p[a]].slot;
        __syncthreads();
    }
    return true;
}

// Steps 6-7 on one sorted region (slots V into the candidate arrays): the
// walk as a max-scan over tiles in walking order, the running maximum carried
// from tile to tile; keep flags by position.  Right region: positions
// 0..cnt-1 after P_0.  Left region: positions cnt-1 down to 1, P_l (position
// 0) always kept.
__device__ void wg_walk(BatchLds& S, const uint32_t* V, uint32_t cnt, int region,
                        const double2* cxy, uint8_t* flag, double x0, double y0, double lx,
                        double ly) {
    const int tid = (int)threadIdx.x, lane = (int)__lane_id(), wave = tid >> 6;
    const int sgn = region == 0 ? 1 : -1;
    const uint32_t nwalk = region == 0 ? cnt : (cnt > 0 ? cnt - 1 : 0);
    BPt carry = bpt_none();
    if (region == 0) {
        carry.x = x0;
        carry.y = y0;
        carry.v = true;
    }
    for (uint32_t t0 = 0; t0 < nwalk; t0 += kBT) {
        BPt it[kBI];
        BPt agg = bpt_none();
#pragma unroll
        for (int k = 0; k < kBI; ++k) {
            const uint32_t w = t0 + (uint32_t)(tid * kBI + k);
            it[k] = bpt_none();
            if (w < nwalk) {
                const double2 v = cxy[V[region == 0 ? w : cnt - 1 - w]];
                it[k].x = v.x;
                it[k].y = v.y;
                it[k].v = true;
            }
        }
#pragma unroll
        for (int k = 0; k < kBI; ++k) agg = bmax(agg, it[k], lx, ly, sgn);
        BPt inc = agg;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const BPt o = shfl_up_bpt(inc, d);
            if (lane >= d) inc = bmax(o, inc, lx, ly, sgn);
        }
        BPt ex = shfl_up_bpt(inc, 1);
        if (lane == 0) ex = bpt_none();
        if (lane == 63) {
            S.wx[wave] = inc.x;
            S.wy[wave] = inc.y;
            S.wv[wave] = inc.v ? 1u : 0u;
        }
        __syncthreads();
        BPt run = carry, all = carry;
        for (int w = 0; w < kBW; ++w) {
            BPt o;
            o.x = S.wx[w];
            o.y = S.wy[w];
            o.v = S.wv[w] != 0u;
            if (w < wave) run = bmax(run, o, lx, ly, sgn);
            all = bmax(all, o, lx, ly, sgn);
        }
        run = bmax(run, ex, lx, ly, sgn);
#pragma unroll
        for (int k = 0; k < kBI; ++k) {
            const uint32_t w = t0 + (uint32_t)(tid * kBI + k);
            if (w < nwalk) {
                const bool kp = (!run.v) ||
                                sgn * orient(lx, ly, run.x, run.y, it[k].x, it[k].y) >= 0;
                flag[region == 0 ? w : cnt - 1 - w] = kp ? 1 : 0;
                run = bmax(run, it[k], lx, ly, sgn);
            }
        }
        carry = all;
        __syncthreads();
    }
    if (region == 1 && tid == 0 && cnt > 0) flag[0] = 1;
    __syncthreads();
}

// Stable removal: kept candidates of one region in position order appended to
// (oxy, oidx) from `at`; returns the new end.
__device__ uint32_t wg_compact(BatchLds& S, const uint32_t* V, const uint8_t* flag, uint32_t cnt,
                               const double2* cxy, const uint32_t* cidx, double2* oxy,
                               uint32_t* oidx, uint32_t at) {
    const int tid = (int)threadIdx.x;
    for (uint32_t t0 = 0; t0 < cnt; t0 += kBT) {
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < kBI; ++k) {
            const uint32_t p = t0 + (uint32_t)(tid * kBI + k);
            c += (p < cnt && flag[p]) ? 1u : 0u;
        }
        uint32_t tot;
        uint32_t o = at + bexcl(c, S, tot);
#pragma unroll
        for (int k = 0; k < kBI; ++k) {
            const uint32_t p = t0 + (uint32_t)(tid * kBI + k);
            if (p < cnt && flag[p]) {
                const uint32_t sl = V[p];
                oxy[o] = cxy[sl];
                oidx[o] = cidx[sl];
                ++o;
            }
        }
        at += tot;
    }
    return at;
}

// Step 8 on a chunk: Graham scan of P_0 followed by K[A[beg..end)) (pop while
// the last two stack points and the new one do not turn left, skip a point
// equal to the top).  The stack, without P_0, goes to st[0..); returns its
// size.  The result is the hull of P_0 and the chunk, so a point it drops is
// no vertex of the whole hull either.
__device__ uint32_t graham_run(const double2* K, const uint32_t* A, uint32_t beg, uint32_t end,
                               uint32_t* st, double x0, double y0) {
    uint32_t top = 0;              // stack entries above P_0
    double tx = x0, ty = y0;       // top of the stack (P_0 when top == 0)
    double sx = x0, sy = y0;       // the entry below it (valid when top >= 1)
    for (uint32_t i = beg; i < end; ++i) {
        const uint32_t pos = A ? A[i] : i;
        const double2 p = K[pos];
        if (p.x == tx && p.y == ty) continue;
        while (top >= 1) {
            if (orient(sx, sy, tx, ty, p.x, p.y) > 0) break;
            --top;
            tx = sx;
            ty = sy;
            if (top >= 2) {
                const double2 q = K[st[top - 2]];
                sx = q.x;
                sy = q.y;
            } else {
                sx = x0;
                sy = y0;
            }
        }
        st[top++] = pos;
        sx = tx;
        sy = ty;
        tx = p.x;
        ty = p.y;
    }
    return top;
}

// graham_run on points staged in LDS (positions are u16 indices into x, y).
__device__ uint32_t graham_lds(const double* __restrict__ gx, const double* __restrict__ gy,
                               const uint16_t* A, uint32_t beg, uint32_t end, uint16_t* st, double x0,
                               double y0) {
    uint32_t top = 0;
    double tx = x0, ty = y0, sx = x0, sy = y0;
    for (uint32_t i = beg; i < end; ++i) {
        const uint32_t pos = A ? A[i] : i;
        const double px = gx[pos], py = gy[pos];
        if (px == tx && py == ty) continue;
        while (top >= 1) {
            if (orient(sx, sy, tx, ty, px, py) > 0) break;
            --top;
            tx = sx;
            ty = sy;
            if (top >= 2) {
                sx = gx[st[top - 2]];
                sy = gy[st[top - 2]];
            } else {
                sx = x0;
                sy = y0;
            }
        }
        st[top++] = (uint16_t)pos;
        sx = tx;
        sy = ty;
        tx = px;
        ty = py;
    }
    return top;
}

// ---------------------------------------------------------------------------
// One set, start to end.
// ---------------------------------------------------------------------------
__device__ void batch_set(const BatchArgs& A, BatchLds& S, int32_t s) {
    const int tid = (int)threadIdx.x, lane = (int)__lane_id(), wave = tid >> 6;
    const int64_t o = A.offs[s];
    const uint32_t n = (uint32_t)(A.offs[s + 1] - o);
    if (n == 0) {
        if (tid == 0) {
            A.h_count[s] = 0;
            A.h_start[s] = 0;
            A.h_flags[s] = 0;
        }
        return;
    }
    const double2* xy = A.xy + o;
    double2* sv_xy = A.sv_xy + o;
    uint32_t* sv_idx = A.sv_idx + o;
    uint32_t* sv_key = A.sv_key + o;
    double2* cd_xy = A.cd_xy + o;
    uint32_t* cd_idx = A.cd_idx + o;
    uint32_t* cd_key = A.cd_key + o;
    uint32_t* ka = A.ka + o;
    uint32_t* kb = A.kb + o;
    uint32_t* va = A.va + o;
    uint32_t* vb = A.vb + o;
    uint8_t* flag = A.flag + o;

    // ---- Step 1
    if (tid == 0) S.flags = 0;
    Cand c[4] = {sentinel(0), sentinel(1), sentinel(2), sentinel(3)};
    uint32_t bad = 0;
    double2 nx[kBI];  // the next tile, loaded while this one is processed
#pragma unroll
    for (int k = 0; k < kBI; ++k) {
        const uint32_t i = (uint32_t)(k * kBB + tid);
        if (i < n) nx[k] = load_stream(&xy[i]);
    }
    for (uint32_t b0 = 0; b0 < n; b0 += kBT) {
        double2 p[kBI];
#pragma unroll
        for (int k = 0; k < kBI; ++k) {
            p[k] = nx[k];
            const uint32_t i = b0 + kBT + (uint32_t)(k * kBB + tid);
            if (i < n) nx[k] = load_stream(&xy[i]);
        }
#pragma unroll
        for (int k = 0; k < kBI; ++k) {
            const uint32_t i = b0 + (uint32_t)(k * kBB + tid);
            if (i < n) {
                const bool need = (p[k].x <= c[0].x) | (p[k].y <= c[1].y) | (p[k].x >= c[2].x) |
                                  (p[k].y >= c[3].y);
                if (need) offer(c, p[k].x, p[k].y, (int32_t)i);
                bad |= domain_flags(p[k].x) | domain_flags(p[k].y);
            }
        }
    }
    reduce4_wave(c);
    __syncthreads();
    if (bad) atomicOr(&S.flags, bad);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) S.ext[wave][k] = c[k];
    }
    __syncthreads();
    if (tid == 0) {
        Cand e[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] = S.ext[0][k];
        for (int w = 1; w < kBW; ++w) {
            take_better<0>(e[0], S.ext[w][0]);
            take_better<1>(e[1], S.ext[w][1]);
            take_better<2>(e[2], S.ext[w][2]);
            take_better<3>(e[3], S.ext[w][3]);
        }
        make_params(S.P, e, S.flags);
    }
    __syncthreads();
    if (S.flags != 0u) {
        if (tid == 0) {
            A.h_count[s] = 0;
            A.h_start[s] = 0;
            A.h_flags[s] = S.flags;
        }
        __syncthreads();
        return;
    }
    const double x0 = S.P.x0, y0 = S.P.y0;
    const int32_t p0_idx = S.P.p0_idx;

    // ---- Steps 2-3 and 5
    {
        double qx[4], qy[4], ex[4], ey[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            qx[j] = S.P.qx[j];
            qy[j] = S.P.qy[j];
            ex[j] = S.P.ex[j];
            ey[j] = S.P.ey[j];
        }
        const double qb = S.P.qbound;
        const int nc = S.P.ncorner;
        if (tid == 0) S.cnt = 0;
        __syncthreads();
        double bd2 = -1.0;
        uint32_t bidx = kNone, bslot = kNone;
        for (uint32_t b0 = 0; b0 < n; b0 += kBT) {
            double2 p[kBI];
#pragma unroll
            for (int k = 0; k < kBI; ++k) {
                const uint32_t i = b0 + (uint32_t)(k * kBB + tid);
                if (i < n) p[k] = load_stream(&xy[i]);
            }
#pragma unroll
            for (int k = 0; k < kBI; ++k) {
                const uint32_t i = b0 + (uint32_t)(k * kBB + tid);
                bool surv = false;
                if (i < n) {
                    surv = !quad_inside(qx, qy, ex, ey, qb, nc, p[k].x, p[k].y) &&
                           !(p[k].x == x0 && p[k].y == y0);
                }
                const uint32_t at = wave_append(surv, &S.cnt);
                if (surv) {
                    const uint32_t key = angle_key(p[k].x, p[k].y, x0, y0);
                    sv_xy[at] = p[k];
                    sv_idx[at] = i;
                    sv_key[at] = key;
                    const double d2 = dist2(p[k].x, p[k].y, x0, y0);
                    const bool tk = (d2 > bd2) | ((d2 == bd2) & (i < bidx));
                    bd2 = tk ? d2 : bd2;
                    bidx = tk ? i : bidx;
                    bslot = tk ? at : bslot;
                }
            }
        }
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) {
            const double od = __shfl_xor(bd2, m);
            const uint32_t oi = __shfl_xor(bidx, m);
            const uint32_t os = __shfl_xor(bslot, m);
            const bool tk = (od > bd2) | ((od == bd2) & (oi < bidx));
            bd2 = tk ? od : bd2;
            bidx = tk ? oi : bidx;
            bslot = tk ? os : bslot;
        }
        if (lane == 0) {
            S.bd2[wave] = bd2;
            S.bidx[wave] = bidx;
            S.bslot[wave] = bslot;
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < kBW; ++w) {
                const bool tk = (S.bd2[w] > bd2) | ((S.bd2[w] == bd2) & (S.bidx[w] < bidx));
                bd2 = tk ? S.bd2[w] : bd2;
                bidx = tk ? S.bidx[w] : bidx;
                bslot = tk ? S.bslot[w] : bslot;
            }
            if (S.cnt > 0) {
                const double2 q = sv_xy[bslot];
                S.P.lx = q.x;
                S.P.ly = q.y;
                S.P.l_idx = (int32_t)bidx;
                S.P.kl = sv_key[bslot];
                const uint32_t tu = turn_key(x0, y0, q.x, q.y);
                S.P.turn_u = tu;
                S.P.turn_v = tu + 0x80000000u;
            }
            S.bslot[0] = bslot;
        }
        __syncthreads();
    }
    const uint32_t m1 = S.cnt;
    const uint32_t lslot = S.bslot[0];
    uint32_t m = 0;  // kept points after the second round (P_0 not counted)

    if (m1 > 0) {
        const Params P = S.P;
        // ---- Steps 6-7: bucket maxima, prefix maxima, candidates
        for (int j = tid; j < 2 * kBuckets; j += kBB) (&S.u.tab[0][0])[j] = 0;
        __syncthreads();
        for (uint32_t i = (uint32_t)tid; i < m1; i += kBB) {
            const double2 p = sv_xy[i];
            const Cls cl = classify(p.x, p.y, sv_key[i], P);
            if (cl.region < 2) atomicMax(&S.u.tab[cl.region][cl.bucket], cl.kappa);
        }
        __syncthreads();
        {
            // exclusive prefix maxima in walking order: right region ascending
            // from kappa(P_0) = 0, left region descending (identity 0)
            constexpr int PER = 2 * kBuckets / kBB;  // per thread, over both regions
            static_assert(kBuckets % (kBB / 2) == 0, "whole buckets per thread");
            const int region = tid < kBB / 2 ? 0 : 1;
            const int r = tid - region * (kBB / 2);  // thread rank within its region
            const int rw = r >> 6;
            uint32_t v[PER];
            uint32_t tmax = 0;
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int w = r * PER + k;
                const int b = region == 0 ? w : kBuckets - 1 - w;
                v[k] = S.u.tab[region][b];
                tmax = max(tmax, v[k]);
            }
            uint32_t inc = tmax;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t q = __shfl_up(inc, d);
                if (lane >= d) inc = max(inc, q);
            }
            uint32_t ex = __shfl_up(inc, 1);
            if (lane == 0) ex = 0;
            if (lane == 63) S.wsum[wave] = inc;
            __syncthreads();
            for (int w = 0; w < rw; ++w) ex = max(ex, S.wsum[region * (kBW / 2) + w]);
            uint32_t run = ex;
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int w = r * PER + k;
                const int b = region == 0 ? w : kBuckets - 1 - w;
                S.u.tab[region][b] = run;
                run = max(run, v[k]);
            }
        }
        __syncthreads();
        if (tid == 0) {
            S.cnt = 0;
            S.lcand = kNone;
        }
        __syncthreads();
        for (uint32_t b0 = 0; b0 < m1; b0 += kBB) {
            const uint32_t i = b0 + (uint32_t)tid;
            bool keep = false;
            double2 p;
            uint32_t key = 0;
            if (i < m1) {
                p = sv_xy[i];
                key = sv_key[i];
                const Cls cl = classify(p.x, p.y, key, P);
                keep = cl.region == 2 || cl.kappa >= S.u.tab[cl.region & 1][cl.bucket];
            }
            const uint32_t at = wave_append(keep, &S.cnt);
            if (keep) {
                cd_xy[at] = p;
                cd_idx[at] = sv_idx[i];
                cd_key[at] = key;
                if (i == lslot) S.lcand = at;
            }
        }
        __syncthreads();
        const uint32_t nc = S.cnt;
        const uint32_t lcand = S.lcand;
        const Rec rl = rec_load(lcand, cd_xy, cd_idx);

        // ---- per region: collect, sort, exact ties, walk, stable removal
        for (int region = 0; region < 2; ++region) {
            if (tid == 0) S.cnt = 0;
            __syncthreads();
            for (uint32_t b0 = 0; b0 < nc; b0 += kBB) {
                const uint32_t i = b0 + (uint32_t)tid;
                bool mine = false;
                uint32_t key = 0;
                if (i < nc) {
                    key = cd_key[i];
                    bool before;
                    if (key != P.kl) {
                        before = key < P.kl;
                    } else if (i == lcand) {
                        before = false;
                    } else {
                        const Rec r = rec_load(i, cd_xy, cd_idx);
                        before = rec_less(r, rl, x0, y0);
                    }
                    mine = before == (region == 0);
                }
                const uint32_t at = wave_append(mine, &S.cnt);
                if (mine) {
                    ka[at] = key;
                    va[at] = i;
                }
            }
            __syncthreads();
            const uint32_t cnt = S.cnt;
            const int cur = wg_radix(S, ka, va, kb, vb, cnt);
            const uint32_t* K = cur ? kb : ka;
            uint32_t* V = cur ? vb : va;
            const bool ok = wg_ties(S, K, V, cnt, cd_xy, cd_idx, x0, y0);
            if (!ok) {
                if (tid == 0) {
                    A.h_count[s] = 0;
                    A.h_start[s] = 0;
                    A.h_flags[s] = kSetFallback;
                }
                __syncthreads();
                return;
            }
            wg_walk(S, V, cnt, region, cd_xy, flag, x0, y0, P.lx, P.ly);
            m = wg_compact(S, V, flag, cnt, cd_xy, cd_idx, sv_xy, sv_idx, m);
            __syncthreads();
        }
    }

    // ---- Step 8: reduce chunks in parallel (in HBM while many points are
    //      left, then in LDS), then one thread
    uint32_t* cur_a = nullptr;  // positions into the kept list (null: all of them)
    uint32_t len = m;
    uint32_t* bufs[3] = {ka, kb, va};
    int nb = 0;
    bool stuck = false;
    while (len > kGLds && !stuck) {
        const uint32_t ch = max(16u, (len + kBB - 1) / kBB);
        uint32_t* st = bufs[nb % 3] == cur_a ? bufs[(nb + 1) % 3] : bufs[nb % 3];
        uint32_t* dst = nullptr;
        for (int q = 0; q < 3; ++q)
            if (bufs[q] != cur_a && bufs[q] != st) dst = bufs[q];
        const uint32_t beg = min(len, (uint32_t)tid * ch), end = min(len, beg + ch);
        const uint32_t h = graham_run(sv_xy, cur_a, beg, end, st + beg, x0, y0);
        uint32_t tot;
        const uint32_t at = bexcl(h, S, tot);
        for (uint32_t j = 0; j < h; ++j) dst[at + j] = st[beg + j];
        __syncthreads();
        stuck = (uint64_t)tot * 10u > (uint64_t)len * 9u;
        cur_a = dst;
        len = tot;
        ++nb;
    }
    const bool in_lds = len <= kGLds;
    uint32_t* fin = ka;       // final stack (HBM path)
    uint16_t* fin16 = nullptr;  // final stack (LDS path)
    if (in_lds) {
        for (uint32_t i = (uint32_t)tid; i < len; i += kBB) {
            const uint32_t pos = cur_a ? cur_a[i] : i;
            const double2 q = sv_xy[pos];
            S.u.gs.x[i] = q.x;
            S.u.gs.y[i] = q.y;
            S.u.gs.pos[i] = pos;
        }
        __syncthreads();
        uint16_t* cur = nullptr;
        uint16_t* b16[3] = {S.u.gs.a, S.u.gs.b, S.u.gs.c};
        int k = 0;
        bool stk = false;
        while (len > kGOne && !stk) {
            const uint32_t ch = max(8u, (len + kBB - 1) / kBB);
            uint16_t* st = b16[k % 3] == cur ? b16[(k + 1) % 3] : b16[k % 3];
            uint16_t* dst = nullptr;
            for (int q = 0; q < 3; ++q)
                if (b16[q] != cur && b16[q] != st) dst = b16[q];
            const uint32_t beg = min(len, (uint32_t)tid * ch), end = min(len, beg + ch);
            const uint32_t h = graham_lds(S.u.gs.x, S.u.gs.y, cur, beg, end, st + beg, x0, y0);
            uint32_t tot;
            const uint32_t at = bexcl(h, S, tot);
            for (uint32_t j = 0; j < h; ++j) dst[at + j] = st[beg + j];
            __syncthreads();
            stk = (uint64_t)tot * 10u > (uint64_t)len * 9u;
            cur = dst;
            len = tot;
            ++k;
        }
        fin16 = S.u.gs.a;
        for (int q = 0; q < 3; ++q)
            if (b16[q] != cur) fin16 = b16[q];
        if (tid == 0) S.h = graham_lds(S.u.gs.x, S.u.gs.y, cur, 0, len, fin16, x0, y0) + 1u;
    } else {
        for (int q = 0; q < 3; ++q)
            if (bufs[q] != cur_a) fin = bufs[q];
        if (tid == 0) S.h = graham_run(sv_xy, cur_a, 0, len, fin, x0, y0) + 1u;
    }
    __syncthreads();
    const uint32_t h = S.h;
    // stack entry k >= 1: its point and its kept-list position
    auto vpos = [&](uint32_t k) -> uint32_t { return in_lds ? S.u.gs.pos[fin16[k - 1]] : fin[k - 1]; };
    // canonical start: the lexicographically smallest vertex (P_0 is entry 0)
    {
        double bx = INFINITY, by = INFINITY;
        uint32_t bk = kNone;
        for (uint32_t k = (uint32_t)tid; k < h; k += kBB) {
            double x, y;
            if (k == 0) {
                x = x0;
                y = y0;
            } else if (in_lds) {
                x = S.u.gs.x[fin16[k - 1]];
                y = S.u.gs.y[fin16[k - 1]];
            } else {
                const double2 q = sv_xy[fin[k - 1]];
                x = q.x;
                y = q.y;
            }
            const bool tk = (x < bx) | ((x == bx) & (y < by));
            bx = tk ? x : bx;
            by = tk ? y : by;
            bk = tk ? k : bk;
        }
#pragma unroll
        for (int msk = 32; msk > 0; msk >>= 1) {
            const double ox = __shfl_xor(bx, msk), oy = __shfl_xor(by, msk);
            const uint32_t ok = __shfl_xor(bk, msk);
            const bool tk = (ox < bx) | ((ox == bx) & (oy < by));
            bx = tk ? ox : bx;
            by = tk ? oy : by;
            bk = tk ? ok : bk;
        }
        if (lane == 0) {
            S.bd2[wave] = bx;
            S.wx[wave] = by;
            S.bidx[wave] = bk;
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < kBW; ++w) {
                const bool tk = (S.bd2[w] < bx) | ((S.bd2[w] == bx) & (S.wx[w] < by));
                bx = tk ? S.bd2[w] : bx;
                by = tk ? S.wx[w] : by;
                bk = tk ? S.bidx[w] : bk;
            }
            S.start = bk;
            S.hpos = atomicAdd(A.hull_cursor, h);
        }
        __syncthreads();
    }
    const uint32_t start = S.start, at = S.hpos;
    for (uint32_t k = (uint32_t)tid; k < h; k += kBB) {
        const uint32_t e = (start + k) % h;
        A.hull[at + k] = e == 0 ? p0_idx : (int32_t)sv_idx[vpos(e)];
    }
    if (tid == 0) {
        A.h_count[s] = (int32_t)h;
        A.h_start[s] = (int32_t)at;
        A.h_flags[s] = 0;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kBB) __attribute__((amdgpu_waves_per_eu(4))) void k_batch(BatchArgs A) {
    __shared__ BatchLds S;
    uint32_t* counter = &A.ctr->ticket[16 * kTicketBatch];
    const uint32_t players = gridDim.x;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t t = take_ticket(counter);
            if (t == (uint32_t)A.S + players - 1) reset_ticket(counter);
            S.ticket = t;
        }
        __syncthreads();
        const uint32_t t = S.ticket;
        if (t >= (uint32_t)A.S) break;
        batch_set(A, S, A.order[t]);
    }
}

}  // namespace

hipError_t launch_batch(const double2* xy, const int64_t* offs, const int32_t* order, int32_t S,
                        double2* sv_xy, uint32_t* sv_idx, uint32_t* sv_key, double2* cd_xy,
                        uint32_t* cd_idx, uint32_t* cd_key, uint32_t* ka, uint32_t* kb,
                        uint32_t* va, uint32_t* vb, uint8_t* flag, int32_t* hull,
                        uint32_t* hull_cursor, int32_t* h_count, int32_t* h_start,
                        uint32_t* h_flags, Counters* ctr, int grid, hipStream_t s) {
    BatchArgs A;
    A.xy = xy;
    A.offs = offs;
    A.order = order;
    A.S = S;
    A.sv_xy = sv_xy;
    A.sv_idx = sv_idx;
    A.sv_key = sv_key;
    A.cd_xy = cd_xy;
    A.cd_idx = cd_idx;
    A.cd_key = cd_key;
    A.ka = ka;
    A.kb = kb;
    A.va = va;
    A.vb = vb;
    A.flag = flag;
    A.hull = hull;
    A.hull_cursor = hull_cursor;
    A.h_count = h_count;
    A.h_start = h_start;
    A.h_flags = h_flags;
    A.ctr = ctr;
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kBB), 0, s, A);
    return hipGetLastError();
}

namespace {
__global__ void k_batch_clear(uint32_t* __restrict__ meta) { meta[0] = 0; }
}  // namespace

hipError_t launch_batch_clear(uint32_t* meta, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_clear, dim3(1), dim3(1), 0, s, meta);
    return hipGetLastError();
}

int batch_blocks_per_cu() {
    return resident_blocks(reinterpret_cast<const void*>(k_batch), kBB);
}

}  // namespace hx
