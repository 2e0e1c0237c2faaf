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
__device__ __forceinline__ int wg_radix(BatchLds& S, uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
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
__device__ __forceinline__ bool wg_ties(BatchLds& S, const uint32_t* K, uint32_t* V, uint32_t cnt, const double2* cxy,
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
__device__ __forceinline__ void wg_walk(BatchLds& S, const uint32_t* V, uint32_t cnt, int region,
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
__device__ __forceinline__ uint32_t wg_compact(BatchLds& S, const uint32_t* V, const uint8_t* flag, uint32_t cnt,
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

// Where entry i of a set's kept list lies in its kept-point arrays: the
// right region's k0 points from lo0, then the left region's from lo1.
struct KeptMap {
    uint32_t lo0, k0, lo1;
    __device__ uint32_t operator()(uint32_t i) const { return i < k0 ? lo0 + i : lo1 + (i - k0); }
};

// Step 8 on a chunk: Graham scan of P_0 followed by K[A[beg..end)) (or the
// kept list's own entries beg..end when A is null; pop while the last two
// stack points and the new one do not turn left, skip a point equal to the
// top).  The stack, without P_0, goes to st[0..); returns its size.  The
// result is the hull of P_0 and the chunk, so a point it drops is no vertex
// of the whole hull either.
__device__ __forceinline__ uint32_t graham_run(const double2* K, const uint32_t* A, const KeptMap& M, uint32_t beg,
                               uint32_t end, uint32_t* st, double x0, double y0) {
    uint32_t top = 0;              // stack entries above P_0
    double tx = x0, ty = y0;       // top of the stack (P_0 when top == 0)
    double sx = x0, sy = y0;       // the entry below it (valid when top >= 1)
    for (uint32_t i = beg; i < end; ++i) {
        const uint32_t pos = A ? A[i] : M(i);
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

// graham_run with its stack in LDS, as 16-bit offsets from beg (ls, room for
// kLdsStack entries: chunks of at most that many points): a pop then reads
// LDS for the entry below instead of global memory written moments before.
constexpr uint32_t kLdsStack = 51;
__device__ __forceinline__ uint32_t graham_run_ls(const double2* K, const uint32_t* A, const KeptMap& M,
                                                  uint32_t beg, uint32_t end, uint16_t* ls, double x0, double y0) {
    uint32_t top = 0;
    double tx = x0, ty = y0, sx = x0, sy = y0;
    for (uint32_t i = beg; i < end; ++i) {
        const double2 p = K[A ? A[i] : M(i)];
        if (p.x == tx && p.y == ty) continue;
        while (top >= 1) {
            if (orient(sx, sy, tx, ty, p.x, p.y) > 0) break;
            --top;
            tx = sx;
            ty = sy;
            if (top >= 2) {
                const uint32_t j = beg + ls[top - 2];
                const double2 q = K[A ? A[j] : M(j)];
                sx = q.x;
                sy = q.y;
            } else {
                sx = x0;
                sy = y0;
            }
        }
        ls[top++] = (uint16_t)(i - beg);
        sx = tx;
        sy = ty;
        tx = p.x;
        ty = p.y;
    }
    return top;
}

// graham_run on points staged in LDS (positions are u16 indices into x, y).
__device__ __forceinline__ uint32_t graham_lds(const double* __restrict__ gx, const double* __restrict__ gy,
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

// Joins T neighbouring chains pairwise until one is left.  Chain t (each
// the stack scan of P_0 followed by chunk t of ch points of the list, a
// convex chain after P_0) starts at position t * ch of P[0]; its length is
// len0[t].  Two neighbouring chains A (earlier) and B combine into the chain
// of their union by keeping a prefix a_1..a_i of A and a suffix b_j..b_q of
// B: for a point b of B, the prefix of A the scan keeps when b arrives is the
// longest whose every step turns left before b (orient(a_{k-1}, a_k, b) > 0,
// a_0 = P_0), a test monotone in k, so a binary search finds it; the bridge
// is the one b_j whose a = a_i has a -> b_{j-1} -> b_j not a left turn and
// a -> b_j -> b_{j+1} a left turn.  np positions in use; entries are LDS
// indices into (X, Y).  Returns the buffer (0: P0, 1: P1) holding the result
// as its chain 0, whose length is then len0[0] or len1[0].
__device__ __forceinline__ int lds_combine(const double* X, const double* Y, uint16_t* P0, uint16_t* P1,
                                           uint16_t* len0, uint16_t* len1, uint16_t* bi, uint16_t* bj, int T,
                                           int np, int ch, double x0, double y0) {
    const int tid = (int)threadIdx.x;
    int cur = 0;
    for (int L = 0; (1 << L) < T; ++L) {
        const int TL = (T + (1 << L) - 1) >> L;
        const uint16_t* P = cur ? P1 : P0;
        uint16_t* Q = cur ? P0 : P1;
        const uint16_t* len = cur ? len1 : len0;
        uint16_t* nlen = cur ? len0 : len1;
        // no bridge found (B empty): all of A, none of B
        for (int t = tid; t < TL / 2; t += kBB) {
            bi[t] = len[2 * t];
            bj[t] = len[2 * t + 1];
        }
        __syncthreads();
        for (int s = tid; s < np; s += kBB) {
            const int c = (s / ch) >> L;
            if ((c & 1) == 0) continue;
            const int j = s - ((c * ch) << L);
            const int q = len[c];
            if (j >= q) continue;
            const int sa = ((c - 1) * ch) << L;
            const int p = len[c - 1];
            const int pb = P[s];
            const double bx = X[pb], by = Y[pb];
            int lo = 0, hi = p;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                const int pk = P[sa + mid];
                double px = x0, py = y0;
                if (mid > 0) {
                    const int pp = P[sa + mid - 1];
                    px = X[pp];
                    py = Y[pp];
                }
                if (orient(px, py, X[pk], Y[pk], bx, by) > 0) lo = mid + 1;
                else hi = mid;
            }
            const int i = lo;
            double ax = x0, ay = y0;
            if (i > 0) {
                const int pa = P[sa + i - 1];
                ax = X[pa];
                ay = Y[pa];
            }
            bool bridge = true;
            if (j > 0) {
                const int pp = P[s - 1];
                bridge = orient(ax, ay, X[pp], Y[pp], bx, by) <= 0;
            }
            if (bridge && j + 1 < q) {
                const int pn = P[s + 1];
                bridge = orient(ax, ay, bx, by, X[pn], Y[pn]) > 0;
            }
            if (bridge) {
                bi[c >> 1] = (uint16_t)i;
                bj[c >> 1] = (uint16_t)j;
            }
        }
        __syncthreads();
        for (int s = tid; s < np; s += kBB) {
            const int c = (s / ch) >> L;
            const int k = s - ((c * ch) << L);
            if (k >= len[c]) continue;
            int dst = -1;
            if ((c & 1) == 0) {
                if (c + 1 >= TL || k < bi[c >> 1]) dst = s;
            } else if (k >= bj[c >> 1]) {
                dst = (((c - 1) * ch) << L) + bi[c >> 1] + (k - bj[c >> 1]);
            }
            if (dst >= 0) Q[dst] = P[s];
        }
        for (int t = tid; t < (TL + 1) / 2; t += kBB) {
            const int b = 2 * t + 1;
            nlen[t] = b < TL ? (uint16_t)(bi[t] + (len[b] - bj[t])) : len[2 * t];
        }
        __syncthreads();
        cur ^= 1;
    }
    return cur;
}

// Where a set's hull goes: hull[start[s] ..+ count[s]], flags[s] = 0.
struct HullSink {
    int32_t* hull;
    uint32_t* cursor;
    int32_t* count;
    int32_t* start;
    uint32_t* flags;
};

// Step 8 of one set and its output.  The kept list (angular order, P_0 not
// in it) is entries 0..m-1 of (kxy, kidx) as M places them; b0, b1, b2 hold
// m positions each.  kLdsStacks: chunk stacks in LDS where they fit (the
// persistent engine keeps them in global memory: its kernel is already at
// its register limit).
template <bool kLdsStacks>
__device__ __forceinline__ void batch_step8(BatchLds& S, const HullSink& H, int32_t s, const double2* kxy,
                            const uint32_t* kidx, const KeptMap& M, uint32_t m, uint32_t* b0,
                            uint32_t* b1, uint32_t* b2, double x0, double y0, int32_t p0_idx) {
    const int tid = (int)threadIdx.x, lane = (int)__lane_id(), wave = tid >> 6;
    // reduce chunks in parallel (in HBM while many points are left, then in
    // LDS), then one thread
    uint32_t* cur_a = nullptr;  // positions into the kept arrays (null: the kept list through M)
    uint32_t len = m;
    uint32_t* bufs[3] = {b0, b1, b2};
    int nb = 0;
    bool stuck = false;
    while (len > kGLds && !stuck) {
        const uint32_t ch = max(16u, (len + kBB - 1) / kBB);
        uint32_t len_next;
        uint32_t* st = bufs[nb % 3] == cur_a ? bufs[(nb + 1) % 3] : bufs[nb % 3];
        uint32_t* dst = nullptr;
        for (int q = 0; q < 3; ++q)
            if (bufs[q] != cur_a && bufs[q] != st) dst = bufs[q];
        const uint32_t beg = min(len, (uint32_t)tid * ch), end = min(len, beg + ch);
        if (kLdsStacks && ch <= kLdsStack) {
            // the stacks in the LDS the final stage has not taken yet
            static_assert(sizeof(S.u) >= (size_t)kBB * kLdsStack * sizeof(uint16_t), "LDS stacks");
            uint16_t* ls = reinterpret_cast<uint16_t*>(&S.u) + (size_t)tid * kLdsStack;
            const uint32_t h = graham_run_ls(kxy, cur_a, M, beg, end, ls, x0, y0);
            uint32_t tot;
            const uint32_t at = bexcl(h, S, tot);
            for (uint32_t j = 0; j < h; ++j) {
                const uint32_t i = beg + ls[j];
                dst[at + j] = cur_a ? cur_a[i] : M(i);
            }
            len_next = tot;
        } else {
            const uint32_t h = graham_run(kxy, cur_a, M, beg, end, st + beg, x0, y0);
            uint32_t tot;
            const uint32_t at = bexcl(h, S, tot);
            for (uint32_t j = 0; j < h; ++j) dst[at + j] = st[beg + j];
            len_next = tot;
        }
        __syncthreads();
        const uint32_t tot = len_next;
        stuck = (uint64_t)tot * 10u > (uint64_t)len * 9u;
        cur_a = dst;
        len = tot;
        ++nb;
    }
    const bool in_lds = len <= kGLds;
    uint32_t* fin = b0;       // final stack (HBM path)
    uint16_t* fin16 = nullptr;  // final stack (LDS path)
    if (in_lds) {
        for (uint32_t i = (uint32_t)tid; i < len; i += kBB) {
            const uint32_t pos = cur_a ? cur_a[i] : M(i);
            const double2 q = kxy[pos];
            S.u.gs.x[i] = q.x;
            S.u.gs.y[i] = q.y;
            S.u.gs.pos[i] = pos;
        }
        __syncthreads();
        // repeats dropped (copies of a point are adjacent): a[] lists the
        // LDS entries of the first copy of each point, in order
        uint32_t keep = 0;
        const uint32_t per = (len + kBB - 1) / kBB;  // at most kGLds / kBB
        const uint32_t i0 = min(len, (uint32_t)tid * per), i1 = min(len, i0 + per);
        for (uint32_t i = i0; i < i1; ++i)
            keep += (i == 0 || S.u.gs.x[i] != S.u.gs.x[i - 1] || S.u.gs.y[i] != S.u.gs.y[i - 1]) ? 1u : 0u;
        uint32_t np;
        uint32_t at = bexcl(keep, S, np);
        for (uint32_t i = i0; i < i1; ++i)
            if (i == 0 || S.u.gs.x[i] != S.u.gs.x[i - 1] || S.u.gs.y[i] != S.u.gs.y[i - 1])
                S.u.gs.a[at++] = (uint16_t)i;
        __syncthreads();
        // chunk scans, then neighbouring chains joined at their common
        // tangent, level by level
        uint16_t* lens = S.u.gs.c;  // [2][kBB] chain lengths, then the bridges
        const uint32_t ch = max(4u, (np + kBB - 1) / kBB);
        const int T = np == 0 ? 0 : (int)((np + ch - 1) / ch);
        if (tid < T) {
            const uint32_t beg = (uint32_t)tid * ch, end = min(np, beg + ch);
            lens[tid] = (uint16_t)graham_lds(S.u.gs.x, S.u.gs.y, S.u.gs.a, beg, end, S.u.gs.b + beg, x0, y0);
        }
        __syncthreads();
        const int cur = lds_combine(S.u.gs.x, S.u.gs.y, S.u.gs.b, S.u.gs.a, lens, lens + kBB,
                                    lens + 2 * kBB, lens + 2 * kBB + kBB / 2, T, (int)np, (int)ch, x0, y0);
        fin16 = cur == 0 ? S.u.gs.b : S.u.gs.a;
        if (tid == 0) S.h = (T == 0 ? 0u : (uint32_t)lens[cur * kBB]) + 1u;
    } else {
        for (int q = 0; q < 3; ++q)
            if (bufs[q] != cur_a) fin = bufs[q];
        if (tid == 0) S.h = graham_run(kxy, cur_a, M, 0, len, fin, x0, y0) + 1u;
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
                const double2 q = kxy[fin[k - 1]];
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
            S.hpos = atomicAdd(H.cursor, h);
        }
        __syncthreads();
    }
    const uint32_t start = S.start, at = S.hpos;
    for (uint32_t k = (uint32_t)tid; k < h; k += kBB) {
        const uint32_t e = (start + k) % h;
        H.hull[at + k] = e == 0 ? p0_idx : (int32_t)kidx[vpos(e)];
    }
    if (tid == 0) {
        H.count[s] = (int32_t)h;
        H.start[s] = (int32_t)at;
        H.flags[s] = 0;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// One set, start to end.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void batch_set(const BatchArgs& A, BatchLds& S, int32_t s) {
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

    HullSink H;
    H.hull = A.hull;
    H.cursor = A.hull_cursor;
    H.count = A.h_count;
    H.start = A.h_start;
    H.flags = A.h_flags;
    batch_step8<false>(S, H, s, sv_xy, sv_idx, KeptMap{0u, m, 0u}, m, ka, kb, va, x0, y0, p0_idx);
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

// ===========================================================================
// The tiled engine.  Passes over points (Step 1, Steps 2-3, the bucket
// maxima, the candidates, their grouping by bucket) run one workgroup per
// tile of points (kWideTile by default) over the tiles of all sets; the reductions and
// bucket prefixes of a set take one workgroup per set; each region of a set
// is sorted and walked by one workgroup (candidates already grouped by their
// angle bucket, so a tile of whole buckets is sorted in LDS bucket by
// bucket); Step 8 takes one workgroup per set.
// ===========================================================================
namespace {

constexpr int kWB = 256;              // threads of the tile passes
constexpr int kWW = kWB / 64;
// entries per thread per round of the candidates' grouping (the passes over
// points take kI of 2, 4 or 8, a schedule option)
constexpr int kWI = 4;
constexpr uint32_t kCT = 2048;        // candidates per walk tile
constexpr int kCI = (int)kCT / kBB;   // walk positions per thread
constexpr uint32_t kSortOne = 32;     // buckets up to this size: one thread sorts them
constexpr uint16_t kInf16 = 0xFFFFu;  // bitonic padding (after every real entry)
static_assert(kCI * kBB == (int)kCT, "walk tile");
static_assert(kBuckets == 1 << kWideSortBits, "sort buckets per region");
static_assert(kCT < kInf16, "16-bit tile positions");

struct WalkTile {
    uint32_t key[kCT], key2[kCT];  // radix ping-pong (the sort overwrites both)
    uint16_t perm[kCT];  // tile positions in sorted order
    uint16_t tmp[kCT];   // radix ping-pong, bitonic buffer
    uint32_t base[256];
    uint16_t wc[kBW][256];
    uint32_t cpos[kCT];       // each entry's position in the candidate arrays
    uint32_t bend[kBuckets];  // the region's bucket ends
    const double2* xy;        // the set's candidates (global memory)
    const uint32_t* idx;
};

struct alignas(16) WalkLds {
    union {
        WalkTile t;
    } u;
    double wx[kBW], wy[kBW];
    uint32_t wv[kBW], wsum[kBW];
    uint32_t tlo, thi, nbig;
    uint32_t big[kCT / (kSortOne + 1) + 1];
};

// Tile t (global numbering) -> its set, the set's layout and the tile's
// point range within the set.
__device__ inline uint32_t wide_tile_set(const WideArgs& A, uint32_t t, WSetIn& in, uint32_t& lo, uint32_t& hi) {
    const int32_t s = A.tile_set[t];
    in = A.in[s];
    lo = (t - in.t0) * in.tile;
    hi = min(lo + in.tile, in.n);
    return (uint32_t)s;
}

// ---- prep: tile owners and cleared counters (one workgroup per set)
__global__ __launch_bounds__(kWB) void k_wprep(WideArgs A) {
    const int32_t s = A.order[blockIdx.x];
    const WSetIn in = A.in[s];
    const uint32_t tid = threadIdx.x;
    for (uint32_t j = tid; j < in.nt; j += kWB) A.tile_set[in.t0 + j] = s;
    if (tid == 0) {
        WSet& W = A.ws[s];
        W.flags = 0u;
        W.m1 = 0u;
        W.lslot = 0u;
        for (int r = 0; r < 2; ++r) {
            W.c[r] = 0u;
            W.big[r] = 0u;
            W.k[r] = 0u;
            W.klo[r] = 0u;
        }
    }
}

// ---- Step 1 on a tile: its four extreme points and domain flags
template <int kI>
__global__ __launch_bounds__(kWB) void k_wext(WideArgs A) {
    __shared__ Cand s_ext[kWW][4];
    __shared__ uint32_t s_bad;
    const int tid = (int)threadIdx.x, lane = (int)__lane_id(), wave = tid >> 6;
    const uint32_t t = A.t_base + blockIdx.x;
    WSetIn in;
    uint32_t lo, hi;
    wide_tile_set(A, t, in, lo, hi);
    const double2* xy = A.xy + in.o;
    if (tid == 0) s_bad = 0u;
    Cand c[4] = {sentinel(0), sentinel(1), sentinel(2), sentinel(3)};
    uint32_t bad = 0;
    for (uint32_t b0 = lo; b0 < hi; b0 += kWB * kI) {
        double2 p[kI];
#pragma unroll
        for (int k = 0; k < kI; ++k) {
            const uint32_t i = b0 + (uint32_t)(k * kWB + tid);
            p[k] = make_double2(0.0, 0.0);
            if (i < hi) p[k] = load_stream(&xy[i]);
        }
#pragma unroll
        for (int k = 0; k < kI; ++k) {
            const uint32_t i = b0 + (uint32_t)(k * kWB + tid);
            if (i < hi) {
                const bool need = (p[k].x <= c[0].x) | (p[k].y <= c[1].y) | (p[k].x >= c[2].x) |
                                  (p[k].y >= c[3].y);
                if (need) offer(c, p[k].x, p[k].y, (int32_t)i);
                bad |= domain_flags(p[k].x) | domain_flags(p[k].y);
            }
        }
    }
    reduce4_wave(c);
    __syncthreads();
    if (bad) atomicOr(&s_bad, bad);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s_ext[wave][k] = c[k];
    }
    __syncthreads();
    if (tid == 0) {
        Cand e[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] = s_ext[0][k];
        for (int w = 1; w < kWW; ++w) {
            take_better<0>(e[0], s_ext[w][0]);
            take_better<1>(e[1], s_ext[w][1]);
            take_better<2>(e[2], s_ext[w][2]);
            take_better<3>(e[3], s_ext[w][3]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) A.tile_ext[4 * t + k] = e[k];
        A.tile_flags[t] = s_bad;
    }
}

// ---- Step 1 of a set: its tiles' extremes, the quadrilateral, P_0
__global__ __launch_bounds__(64) void k_wparams(WideArgs A) {
    const int32_t s = A.order[blockIdx.x];
    const WSetIn in = A.in[s];
    const uint32_t lane = threadIdx.x;
    if (in.n == 0) return;
    Cand c[4] = {sentinel(0), sentinel(1), sentinel(2), sentinel(3)};
    uint32_t bad = 0;
    for (uint32_t j = lane; j < in.nt; j += 64) {
        const uint32_t t = in.t0 + j;
        take_better<0>(c[0], A.tile_ext[4 * t + 0]);
        take_better<1>(c[1], A.tile_ext[4 * t + 1]);
        take_better<2>(c[2], A.tile_ext[4 * t + 2]);
        take_better<3>(c[3], A.tile_ext[4 * t + 3]);
        bad |= A.tile_flags[t];
    }
    reduce4_wave(c);
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) bad |= __shfl_xor(bad, m);
    if (lane == 0) {
        make_params(A.ws[s].P, c, bad);
        A.ws[s].flags = bad;
    }
}

// ---- Steps 2-3 on a tile: survivors (packed at the tile's first position)
//      with their angle keys, and the tile's farthest survivor (Step 5)
template <int kI>
__global__ __launch_bounds__(kWB) void k_wfilter(WideArgs A) {
    __shared__ uint32_t s_cnt;
    __shared__ double s_d2[kWW];
    __shared__ uint32_t s_i[kWW], s_sl[kWW];
    const int tid = (int)threadIdx.x, lane = (int)__lane_id(), wave = tid >> 6;
    const uint32_t t = A.t_base + blockIdx.x;
    WSetIn in;
    uint32_t lo, hi;
    const uint32_t s = wide_tile_set(A, t, in, lo, hi);
    const WSet& W = A.ws[s];
    if (W.flags != 0u) return;
    double qx[4], qy[4], ex[4], ey[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        qx[j] = W.P.qx[j];
        qy[j] = W.P.qy[j];
        ex[j] = W.P.ex[j];
        ey[j] = W.P.ey[j];
    }
    const double qb = W.P.qbound, x0 = W.P.x0, y0 = W.P.y0;
    const int nc = W.P.ncorner;
    const double2* xy = A.xy + in.o;
    double2* sv_xy = A.sv_xy + in.o;
    uint32_t* sv_idx = A.sv_idx + in.o;
    uint32_t* sv_key = A.sv_key + in.o;
    if (tid == 0) s_cnt = 0u;
    __syncthreads();
    double bd2 = -1.0;
    uint32_t bidx = kNone, bslot = kNone;
    for (uint32_t b0 = lo; b0 < hi; b0 += kWB * kI) {
        double2 p[kI];
#pragma unroll
        for (int k = 0; k < kI; ++k) {
            const uint32_t i = b0 + (uint32_t)(k * kWB + tid);
            p[k] = make_double2(0.0, 0.0);
            if (i < hi) p[k] = load_stream(&xy[i]);
        }
#pragma unroll
        for (int k = 0; k < kI; ++k) {
            const uint32_t i = b0 + (uint32_t)(k * kWB + tid);
            bool surv = false;
            if (i < hi) {
                surv = !quad_inside(qx, qy, ex, ey, qb, nc, p[k].x, p[k].y) &&
                       !(p[k].x == x0 && p[k].y == y0);
            }
            const uint32_t at = wave_append(surv, &s_cnt);
            if (surv) {
                const uint32_t pos = lo + at;
                sv_xy[pos] = p[k];
                sv_idx[pos] = i;
                sv_key[pos] = angle_key(p[k].x, p[k].y, x0, y0);
                const double d2 = dist2(p[k].x, p[k].y, x0, y0);
                const bool tk = (d2 > bd2) | ((d2 == bd2) & (i < bidx));
                bd2 = tk ? d2 : bd2;
                bidx = tk ? i : bidx;
                bslot = tk ? pos : bslot;
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
        s_d2[wave] = bd2;
        s_i[wave] = bidx;
        s_sl[wave] = bslot;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < kWW; ++w) {
            const bool tk = (s_d2[w] > bd2) | ((s_d2[w] == bd2) & (s_i[w] < bidx));
            bd2 = tk ? s_d2[w] : bd2;
            bidx = tk ? s_i[w] : bidx;
            bslot = tk ? s_sl[w] : bslot;
        }
        WFar f;
        f.d2 = bd2;
        f.idx = bidx;
        f.slot = bslot;
        A.tile_far[t] = f;
        A.tile_cnt[t] = s_cnt;
    }
}

// ---- Step 5 of a set: P_l, the farthest survivor (smallest index on ties)
__global__ __launch_bounds__(64) void k_wfar(WideArgs A) {
    const int32_t s = A.order[blockIdx.x];
    const WSetIn in = A.in[s];
    const uint32_t lane = threadIdx.x;
    if (in.n == 0) return;
    WSet& W = A.ws[s];
    if (W.flags != 0u) return;
    double bd2 = -1.0;
    uint32_t bidx = kNone, bslot = kNone, m1 = 0;
    for (uint32_t j = lane; j < in.nt; j += 64) {
        const uint32_t t = in.t0 + j;
        const WFar f = A.tile_far[t];
        m1 += A.tile_cnt[t];
        const bool tk = (f.d2 > bd2) | ((f.d2 == bd2) & (f.idx < bidx));
        bd2 = tk ? f.d2 : bd2;
        bidx = tk ? f.idx : bidx;
        bslot = tk ? f.slot : bslot;
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        const double od = __shfl_xor(bd2, m);
        const uint32_t oi = __shfl_xor(bidx, m);
        const uint32_t os = __shfl_xor(bslot, m);
        m1 += __shfl_xor(m1, m);
        const bool tk = (od > bd2) | ((od == bd2) & (oi < bidx));
        bd2 = tk ? od : bd2;
        bidx = tk ? oi : bidx;
        bslot = tk ? os : bslot;
    }
    if (lane == 0) {
        W.m1 = m1;
        if (m1 > 0) {
            const double2 q = A.sv_xy[in.o + bslot];
            W.P.lx = q.x;
            W.P.ly = q.y;
            W.P.l_idx = (int32_t)bidx;
            W.P.kl = A.sv_key[in.o + bslot];
            const uint32_t tu = turn_key(W.P.x0, W.P.y0, q.x, q.y);
            W.P.turn_u = tu;
            W.P.turn_v = tu + 0x80000000u;
            W.lslot = bslot;
        }
    }
}

// The fields of Step 6-7's classification, read once per workgroup.
struct WCls {
    double x0, y0, lx, ly;
    uint32_t kl, tu, tv;
    int32_t l_idx;
    __device__ explicit WCls(const Params& P)
        : x0(P.x0), y0(P.y0), lx(P.lx), ly(P.ly), kl(P.kl), tu(P.turn_u), tv(P.turn_v), l_idx(P.l_idx) {}
    __device__ Cls operator()(double x, double y, uint32_t key) const {
        return classify_at(x, y, key, x0, y0, lx, ly, kl, tu, tv);
    }
    __device__ Cls near(double x, double y, uint32_t key) const {
        return classify_near(x, y, key, x0, y0, lx, ly, kl, tu, tv);
    }
};

// Exclusive block scan over kT threads (sum or max); all threads call it.
template <bool kMax, int kT>
__device__ inline uint32_t wblock_scan(uint32_t v, uint32_t* s_w, uint32_t& total) {
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d);
        if (lane >= d) inc = kMax ? max(inc, o) : inc + o;
    }
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kT / 64; ++w) {
        const uint32_t x = s_w[w];
        if (w < wave) pre = kMax ? max(pre, x) : pre + x;
        tot = kMax ? max(tot, x) : tot + x;
    }
    __syncthreads();
    total = tot;
    const uint32_t ex = __shfl_up(inc, 1);
    const uint32_t lane_ex = lane == 0 ? 0u : ex;
    return kMax ? max(pre, lane_ex) : pre + lane_ex;
}

// ---- Steps 6-7 of one set in one workgroup (sets largest first): the
//      bucket maxima of its survivors' direction keys (an LDS table of 2^bf
//      buckets per region; the keys from turn_key_near, each within
//      kTurnSlack / 8 of the exact one, and each survivor's key and region
//      kept in ka and the bytes of vb), their exclusive prefix maxima in
//      walking order (right region ascending from kappa(P_0) = 0, left
//      region descending), the candidates (every survivor whose key plus
//      kTurnSlack reaches the prefix maximum: a point dropped has an exact
//      key below that of a point in an earlier bucket, so the exact walk
//      drops it too; packed at the set's first
//      positions of cd_*, with their sort region in flag: before P_l in the
//      exact angular order 0, P_l and after 1), then the candidates grouped
//      by sort bucket: counted in LDS, the bucket starts (region 0 from 0,
//      region 1 after it), every candidate's angle key and position placed
//      in its bucket of gk (order within a bucket arbitrary: the walk sorts
//      each tile); the bucket ends, region sizes and largest buckets go to
//      global memory for the walk.
//      Two instances: sets of more than 2^kSmallBits buckets per region get
//      1024 threads and the 128 KB table (one workgroup per compute unit),
//      the others 256 threads and a 16 KB table.  Each instance's grid covers
//      its own sets only (the first S_large sets of the launch, sizes
//      descending, and the rest), so that no workgroup reserves a table only
//      to return.
constexpr int kSmallBits = kWideSmallBits;
constexpr uint32_t kPreTiles = 2048;  // sets of up to this many tiles spread their survivors evenly

template <int kBits, int kMB>
__global__ __launch_bounds__(kMB) void k_wset(WideArgs A) {
    constexpr int kMW = kMB / 64;
    constexpr uint32_t kFiltMax = 1u << kBits;
    constexpr uint32_t kSortMax = 1u << (kBits < kWideSortBits ? kBits : kWideSortBits);
    static_assert(kFiltMax % kMB == 0 && kSortMax % kMB == 0, "whole buckets per thread");
    __shared__ uint32_t s_tab[2 * kFiltMax];
    __shared__ uint32_t s_pre[kPreTiles + 1];  // survivors before each tile
    __shared__ uint32_t s_w[kMW];
    __shared__ uint32_t s_nc;
    const int tid = (int)threadIdx.x;
    const int32_t s = A.order[blockIdx.x + (kBits > kSmallBits ? 0u : (uint32_t)A.S_large)];
    const WSetIn in = A.in[s];
    if (in.n == 0) return;
    if (kBits > kSmallBits ? in.bf <= (uint32_t)kSmallBits : in.bf > (uint32_t)kSmallBits) return;
    WSet& W = A.ws[s];
    if (W.flags != 0u || W.m1 == 0u) return;
    const WCls C(W.P);
    const uint32_t lslot = W.lslot;
    const size_t o = (size_t)in.o;
    const double2* sv_xy = A.sv_xy + o;
    const uint32_t* sv_key = A.sv_key + o;
    const uint32_t* sv_idx = A.sv_idx + o;
    uint32_t* kap = A.ka + o;
    uint8_t* reg = reinterpret_cast<uint8_t*>(A.vb) + o;
    const uint32_t bf = in.bf, shf = 32u - bf, B = 1u << bf;
    for (uint32_t j = (uint32_t)tid; j < 2u * B; j += kMB) s_tab[j] = 0u;
    if (tid == 0) s_nc = 0u;
    __syncthreads();

    // the survivors of all tiles numbered 0..m1-1 in tile order (sets of
    // more than kPreTiles tiles go tile by tile instead)
    const bool flat = in.nt <= kPreTiles;
    if (flat) {
        constexpr int kPT = (int)(kPreTiles + kMB - 1) / kMB;
        uint32_t c[kPT], tsum = 0;
#pragma unroll
        for (int k = 0; k < kPT; ++k) {
            const uint32_t j = (uint32_t)tid * kPT + (uint32_t)k;
            c[k] = j < in.nt ? A.tile_cnt[in.t0 + j] : 0u;
            tsum += c[k];
        }
        uint32_t tot;
        uint32_t run = wblock_scan<false, kMB>(tsum, s_w, tot);
#pragma unroll
        for (int k = 0; k < kPT; ++k) {
            const uint32_t j = (uint32_t)tid * kPT + (uint32_t)k;
            if (j < in.nt) s_pre[j] = run;
            run += c[k];
        }
        if (tid == 0) s_pre[in.nt] = tot;
        __syncthreads();
    }
    const uint32_t nt = in.nt;
    // survivor f of the flat numbering -> its position
    auto spos = [&](uint32_t f) -> uint32_t {
        uint32_t a = 0, z = nt - 1;  // last tile whose first survivor is at or before f
        while (a < z) {
            const uint32_t mid = (a + z + 1) >> 1;
            if (s_pre[mid] <= f) a = mid;
            else z = mid - 1;
        }
        return a * in.tile + (f - s_pre[a]);
    };
    const uint32_t ntile_loops = flat ? 1u : nt;

    // bucket maxima, every thread taking kSI survivors at a time
    constexpr int kSI = 4;
    for (uint32_t tl = 0; tl < ntile_loops; ++tl) {
        const uint32_t fend = flat ? s_pre[nt] : A.tile_cnt[in.t0 + tl];
        for (uint32_t b0 = 0; b0 < fend; b0 += (uint32_t)kMB * kSI) {
            double2 p[kSI];
            uint32_t key[kSI], at[kSI];
#pragma unroll
            for (int k = 0; k < kSI; ++k) {
                const uint32_t f = b0 + (uint32_t)(k * kMB + tid);
                p[k] = make_double2(0.0, 0.0);
                key[k] = 0;
                at[k] = 0;
                if (f < fend) {
                    at[k] = flat ? spos(f) : tl * in.tile + f;
                    p[k] = sv_xy[at[k]];
                    key[k] = sv_key[at[k]];
                }
            }
#pragma unroll
            for (int k = 0; k < kSI; ++k) {
                const uint32_t f = b0 + (uint32_t)(k * kMB + tid);
                if (f < fend) {
                    const Cls cl = C.near(p[k].x, p[k].y, key[k]);
                    if (cl.region < 2) atomicMax(&s_tab[((uint32_t)cl.region << bf) + (key[k] >> shf)], cl.kappa);
                    kap[at[k]] = cl.kappa;
                    reg[at[k]] = (uint8_t)cl.region;
                }
            }
        }
    }
    __syncthreads();

    // prefix maxima in walking order, in place
    {
        const uint32_t per = B > (uint32_t)kMB ? B / kMB : 1u;
        constexpr int kPer = (int)kFiltMax / kMB;
        for (int region = 0; region < 2; ++region) {
            uint32_t* T = s_tab + ((uint32_t)region << bf);
            uint32_t v[kPer];
            uint32_t tmax = 0;
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const uint32_t w = (uint32_t)tid * per + (uint32_t)k;
                v[k] = 0;
                if ((uint32_t)k < per && w < B) {
                    v[k] = T[region == 0 ? w : B - 1 - w];
                    tmax = max(tmax, v[k]);
                }
            }
            uint32_t tot;
            uint32_t run = wblock_scan<true, kMB>(tmax, s_w, tot);
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const uint32_t w = (uint32_t)tid * per + (uint32_t)k;
                if ((uint32_t)k < per && w < B) {
                    T[region == 0 ? w : B - 1 - w] = run;
                    run = max(run, v[k]);
                }
            }
        }
    }
    __syncthreads();

    // candidates, likewise
    for (uint32_t tl = 0; tl < ntile_loops; ++tl) {
        const uint32_t fend = flat ? s_pre[nt] : A.tile_cnt[in.t0 + tl];
        for (uint32_t b0 = 0; b0 < fend; b0 += (uint32_t)kMB * kSI) {
            uint32_t key[kSI], kp[kSI], rg[kSI], at[kSI];
#pragma unroll
            for (int k = 0; k < kSI; ++k) {
                const uint32_t f = b0 + (uint32_t)(k * kMB + tid);
                key[k] = kp[k] = at[k] = 0;
                rg[k] = 3u;
                if (f < fend) {
                    at[k] = flat ? spos(f) : tl * in.tile + f;
                    key[k] = sv_key[at[k]];
                    kp[k] = kap[at[k]];
                    rg[k] = reg[at[k]];
                }
            }
            // keep flags first, then one LDS reservation per wave for all
            // kSI rounds, then the loads and stores of the candidates
            bool keep[kSI];
            uint64_t mk[kSI];
            uint32_t cnt = 0;
#pragma unroll
            for (int k = 0; k < kSI; ++k) {
                keep[k] = rg[k] == 2u ||
                          (rg[k] < 2u && (uint64_t)kp[k] + kTurnSlack >= s_tab[(rg[k] << bf) + (key[k] >> shf)]);
                mk[k] = __ballot(keep[k]);
                cnt += (uint32_t)__popcll(mk[k]);
            }
            uint32_t base = 0;
            if (__lane_id() == 0 && cnt > 0) base = atomicAdd(&s_nc, cnt);
            base = __shfl(base, 0);
#pragma unroll
            for (int k = 0; k < kSI; ++k) {
                const uint32_t i = at[k];
                if (keep[k]) {
                    const double2 p = sv_xy[i];
                    const uint32_t idx = sv_idx[i];
                    uint32_t sreg;
                    if (key[k] != C.kl) sreg = key[k] < C.kl ? 0u : 1u;
                    else if (i == lslot) sreg = 1u;
                    else sreg = angle_less(p.x, p.y, idx, C.lx, C.ly, (uint32_t)C.l_idx, C.x0, C.y0) ? 0u : 1u;
                    const uint32_t pos = base + (uint32_t)__popcll(mk[k] & lanemask_lt());
                    A.cd_xy[o + pos] = p;
                    A.cd_idx[o + pos] = idx;
                    A.cd_key[o + pos] = key[k];
                    A.flag[o + pos] = (uint8_t)sreg;
                }
                base += (uint32_t)__popcll(mk[k]);
            }
        }
    }
    __syncthreads();
    const uint32_t nc = s_nc;

    // grouping by sort bucket (the table now counts, then places)
    const uint32_t bs = in.bs, shs = 32u - bs, BS = 1u << bs;
    for (uint32_t j = (uint32_t)tid; j < 2u * BS; j += kMB) s_tab[j] = 0u;
    __syncthreads();
    for (uint32_t b0 = 0; b0 < nc; b0 += kMB * kWI) {
        uint32_t key[kWI], sr[kWI];
#pragma unroll
        for (int k = 0; k < kWI; ++k) {
            const uint32_t i = b0 + (uint32_t)(k * kMB + tid);
            key[k] = sr[k] = 0;
            if (i < nc) {
                key[k] = A.cd_key[o + i];
                sr[k] = A.flag[o + i];
            }
        }
#pragma unroll
        for (int k = 0; k < kWI; ++k) {
            const uint32_t i = b0 + (uint32_t)(k * kMB + tid);
            if (i < nc) atomicAdd(&s_tab[(sr[k] << bs) + (key[k] >> shs)], 1u);
        }
    }
    __syncthreads();
    {
        const uint32_t per = BS > (uint32_t)kMB ? BS / kMB : 1u;
        constexpr int kPer = (int)kSortMax / kMB;
        uint32_t base = 0;
        for (int region = 0; region < 2; ++region) {
            uint32_t* T = s_tab + ((uint32_t)region << bs);
            uint32_t v[kPer];
            uint32_t tsum = 0, tmax = 0;
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const uint32_t w = (uint32_t)tid * per + (uint32_t)k;
                v[k] = 0;
                if ((uint32_t)k < per && w < BS) v[k] = T[w];
                tsum += v[k];
                tmax = max(tmax, v[k]);
            }
            uint32_t tot, big;
            uint32_t run = base + wblock_scan<false, kMB>(tsum, s_w, tot);
            (void)wblock_scan<true, kMB>(tmax, s_w, big);
            uint32_t* ends = A.bcnt + in.soff + ((uint32_t)region << bs);
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const uint32_t w = (uint32_t)tid * per + (uint32_t)k;
                if ((uint32_t)k < per && w < BS) {
                    T[w] = run;
                    run += v[k];
                    ends[w] = run;
                }
            }
            if (tid == 0) {
                W.c[region] = tot;
                W.big[region] = big;
            }
            base += tot;
        }
    }
    __syncthreads();
    for (uint32_t b0 = 0; b0 < nc; b0 += kMB * kWI) {
        uint32_t key[kWI], sr[kWI];
#pragma unroll
        for (int k = 0; k < kWI; ++k) {
            const uint32_t i = b0 + (uint32_t)(k * kMB + tid);
            key[k] = sr[k] = 0;
            if (i < nc) {
                key[k] = A.cd_key[o + i];
                sr[k] = A.flag[o + i];
            }
        }
#pragma unroll
        for (int k = 0; k < kWI; ++k) {
            const uint32_t i = b0 + (uint32_t)(k * kMB + tid);
            if (i < nc) {
                const uint32_t pos = atomicAdd(&s_tab[(sr[k] << bs) + (key[k] >> shs)], 1u);
                A.gk[o + pos] = make_uint2(key[k], i);
            }
        }
    }
}

// The exact order of Step 4 between two tile entries of equal angle key.
__device__ inline bool tile_less(const WalkTile& T, uint32_t a, uint32_t b, double x0, double y0) {
    const double2 p = T.xy[T.cpos[a]], q = T.xy[T.cpos[b]];
    return angle_less(p.x, p.y, T.idx[T.cpos[a]], q.x, q.y, T.idx[T.cpos[b]], x0, y0);
}
__device__ inline bool tile_less_pad(const WalkTile& T, uint16_t a, uint16_t b, double x0, double y0) {
    if (a == kInf16) return false;
    if (b == kInf16) return true;
    return tile_less(T, a, b, x0, y0);
}

// Stable LSD radix sort (8-bit digits) of the tile's angle keys with their
// positions, in LDS: T.perm[0..nt) ends as the positions in key order (equal
// keys in position order); returns the sorted keys (T.key or T.key2).  A
// pass is skipped when the smallest and largest key agree on that digit and
// every digit above it (then every key does).
__device__ __forceinline__ const uint32_t* tile_radix(WalkTile& T, uint32_t* s_wsum, uint32_t nt) {
    const int tid = (int)threadIdx.x, lane = (int)__lane_id(), wave = tid >> 6;
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
    for (uint32_t j = (uint32_t)tid; j < nt; j += kBB) {
        kmin = min(kmin, T.key[j]);
        kmax = max(kmax, T.key[j]);
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        kmin = min(kmin, __shfl_xor(kmin, d));
        kmax = max(kmax, __shfl_xor(kmax, d));
    }
    if (lane == 0) {
        s_wsum[wave] = kmin;
        T.base[wave] = kmax;
    }
    __syncthreads();
    for (int w = 0; w < kBW; ++w) {
        kmin = min(kmin, s_wsum[w]);
        kmax = max(kmax, T.base[w]);
    }
    const uint32_t diff = kmin ^ kmax;  // every key lies in [kmin, kmax]
    __syncthreads();
    uint32_t* ks = T.key;
    uint16_t* vs = T.perm;
    uint32_t* kd = T.key2;
    uint16_t* vd = T.tmp;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        // the smallest and largest key agree on this digit and above: so
        // does every key, and the pass would not move anything
        if ((diff >> shift) == 0u) continue;
        for (int j = tid; j < kBW * 256; j += kBB) (&T.wc[0][0])[j] = 0;
        __syncthreads();
        uint32_t key[kCI], rank[kCI];
        uint16_t val[kCI];
#pragma unroll
        for (int k = 0; k < kCI; ++k) {
            const uint32_t p = (uint32_t)(wave * 64 * kCI + k * 64 + lane);
            key[k] = 0;
            val[k] = 0;
            if (p < nt) {
                key[k] = ks[p];
                val[k] = vs[p];
            }
        }
#pragma unroll
        for (int k = 0; k < kCI; ++k) {
            const uint32_t p = (uint32_t)(wave * 64 * kCI + k * 64 + lane);
            const bool valid = p < nt;
            const uint32_t dig = (key[k] >> shift) & 0xFFu;
            const uint64_t m = match_digit8(dig, valid);
            uint32_t prior = 0;
            if (valid) prior = T.wc[wave][dig];
            const uint32_t below = (uint32_t)__popcll(m & lanemask_lt());
            __builtin_amdgcn_wave_barrier();
            if (valid && below == 0u) T.wc[wave][dig] = (uint16_t)(prior + (uint32_t)__popcll(m));
            __builtin_amdgcn_wave_barrier();
            rank[k] = prior + below;
        }
        __syncthreads();
        if (tid < 256) {
            uint32_t tot = 0;
            for (int w = 0; w < kBW; ++w) {
                const uint32_t c = T.wc[w][tid];
                T.wc[w][tid] = (uint16_t)tot;
                tot += c;
            }
            const uint32_t inc = bw_incl(tot);
            if (lane == 63) s_wsum[wave] = inc;
            T.base[tid] = inc - tot;
        }
        __syncthreads();
        if (tid < 256) {
            uint32_t pre = 0;
            for (int w = 0; w < wave; ++w) pre += s_wsum[w];
            T.base[tid] += pre;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kCI; ++k) {
            const uint32_t p = (uint32_t)(wave * 64 * kCI + k * 64 + lane);
            if (p < nt) {
                const uint32_t dig = (key[k] >> shift) & 0xFFu;
                const uint32_t q = T.base[dig] + T.wc[wave][dig] + rank[k];
                kd[q] = key[k];
                vd[q] = val[k];
            }
        }
        __syncthreads();
        uint32_t* tk = ks;
        ks = kd;
        kd = tk;
        uint16_t* tv = vs;
        vs = vd;
        vd = tv;
    }
    if (vs != T.perm) {
        for (uint32_t j = (uint32_t)tid; j < nt; j += kBB) T.perm[j] = vs[j];
        __syncthreads();
    }
    return ks;
}

// Bitonic sort of perm[bs, bs + len) in LDS by the whole workgroup.
__device__ __forceinline__ void tile_bitonic(WalkTile& T, uint32_t bs, uint32_t len, double x0, double y0) {
    const uint32_t tid = threadIdx.x;
    uint32_t P2 = 1;
    while (P2 < len) P2 <<= 1;
    for (uint32_t a = tid; a < P2; a += kBB) T.tmp[a] = a < len ? T.perm[bs + a] : kInf16;
    __syncthreads();
    for (uint32_t kb = 2; kb <= P2; kb <<= 1) {
        for (uint32_t jj = kb >> 1; jj > 0; jj >>= 1) {
            for (uint32_t a = tid; a < P2; a += kBB) {
                const uint32_t b = a ^ jj;
                if (b > a) {
                    const uint16_t ia = T.tmp[a], ib = T.tmp[b];
                    const bool asc = (a & kb) == 0;
                    const bool swap = asc ? tile_less_pad(T, ib, ia, x0, y0) : tile_less_pad(T, ia, ib, x0, y0);
                    if (swap) {
                        T.tmp[a] = ib;
                        T.tmp[b] = ia;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t a = tid; a < len; a += kBB) T.perm[bs + a] = T.tmp[a];
    __syncthreads();
}

// The region a walk workgroup takes: sets largest first, two regions each.
struct WRegion {
    int32_t s;
    int r;
    uint32_t cnt, rs, re;
};
__device__ inline bool wide_region(const WideArgs& A, WRegion& R, uint32_t g = blockIdx.x) {
    R.s = A.order[g >> 1];
    R.r = (int)(g & 1u);
    const WSet& W = A.ws[R.s];
    if (A.in[R.s].n == 0 || W.flags != 0u || W.m1 == 0u) return false;
    R.cnt = W.c[R.r];
    R.rs = R.r == 0 ? 0u : W.c[0];
    R.re = R.rs + R.cnt;
    return true;
}

// ---- Step 4 and the walk of Figure 2 on one region of one set whose
//      buckets all fit a tile: tiles of whole buckets in walking order, each
//      sorted bucket by bucket in LDS, then walked as a max-scan with the
//      running maximum carried from tile to tile; kept points to (sv_xy,
//      sv_idx): the right region ascending from its first position, the left
//      region descending from its last (P_l, always kept, last of all)
__global__ __launch_bounds__(kBB) __attribute__((amdgpu_waves_per_eu(4))) void k_wwalk(WideArgs A) {
    __shared__ WalkLds L;
    const int tid = (int)threadIdx.x, lane = (int)__lane_id(), wave = tid >> 6;
    WRegion R;
    if (!wide_region(A, R)) return;
    WSet& W = A.ws[R.s];
    if (W.big[R.r] > kCT || R.cnt <= 64u) return;
    const WSetIn in = A.in[R.s];
    const size_t o = (size_t)in.o;
    const int r = R.r;
    const uint32_t rs = R.rs, re = R.re;
    const double x0 = W.P.x0, y0 = W.P.y0, lx = W.P.lx, ly = W.P.ly;
    const int sgn = r == 0 ? 1 : -1;

    WalkTile& T = L.u.t;
    const uint32_t B = 1u << in.bs;
    const uint32_t* ends = A.bcnt + in.soff + ((uint32_t)r << in.bs);
    for (uint32_t b = (uint32_t)tid; b < B; b += kBB) T.bend[b] = ends[b];
    __syncthreads();
    auto bstart = [&](uint32_t b) -> uint32_t { return b == 0 ? rs : T.bend[b - 1]; };
    BPt carry = bpt_none();
    if (r == 0) {
        carry.x = x0;
        carry.y = y0;
        carry.v = true;
    }
    uint32_t kept = 0;
    uint32_t lo_p = rs, hi_p = re;  // positions not walked yet
    while (lo_p < hi_p) {
        if (tid == 0) {
            uint32_t plo, phi;
            if (r == 0) {
                // [lo_p, e): e the last bucket end within lo_p + kCT
                const uint32_t lim = lo_p + min(kCT, hi_p - lo_p);
                uint32_t a = 0, z = B - 1;  // largest b with bend[b] <= lim (bend[B-1] = re <= lim or not)
                while (a < z) {
                    const uint32_t mid = (a + z + 1) >> 1;
                    if (T.bend[mid] <= lim) a = mid;
                    else z = mid - 1;
                }
                plo = lo_p;
                phi = T.bend[a];
            } else {
                // [e, hi_p): e the first bucket start at or after hi_p - kCT
                const uint32_t lim = hi_p - min(kCT, hi_p - lo_p);
                uint32_t a = 0, z = B - 1;  // smallest b with bstart(b) >= lim
                while (a < z) {
                    const uint32_t mid = (a + z) >> 1;
                    if (bstart(mid) >= lim) z = mid;
                    else a = mid + 1;
                }
                plo = bstart(a);
                phi = hi_p;
            }
            L.tlo = plo;
            L.thi = phi;
            L.nbig = 0;
            T.idx = A.cd_idx + o;
            T.xy = A.cd_xy + o;
        }
        __syncthreads();
        const uint32_t plo = L.tlo, phi = L.thi, nt = phi - plo;
        for (uint32_t j = (uint32_t)tid; j < nt; j += kBB) {
            const uint2 g = A.gk[o + plo + j];
            T.key[j] = g.x;
            T.cpos[j] = g.y;
            T.perm[j] = (uint16_t)j;
        }
        __syncthreads();
        // sorted by angle key, then the exact order within runs of equal keys:
        // short runs by one thread each, longer ones by the workgroup
        const uint32_t* K = tile_radix(T, L.wsum, nt);
        for (uint32_t j = (uint32_t)tid; j < nt; j += kBB) {
            if (j > 0 && K[j - 1] == K[j]) continue;
            if (!(j + 1 < nt && K[j + 1] == K[j])) continue;
            uint32_t e = j + 2;
            while (e < nt && e - j <= kSortOne && K[e] == K[j]) ++e;
            if (e - j > kSortOne) {
                const uint32_t at = atomicAdd(&L.nbig, 1u);
                L.big[at] = j;
                continue;
            }
            for (uint32_t a = j + 1; a < e; ++a) {
                const uint16_t v = T.perm[a];
                uint32_t q = a;
                while (q > j && tile_less(T, v, T.perm[q - 1], x0, y0)) {
                    T.perm[q] = T.perm[q - 1];
                    --q;
                }
                T.perm[q] = v;
            }
        }
        __syncthreads();
        const uint32_t nbig = L.nbig;
        for (uint32_t jb = 0; jb < nbig; ++jb) {
            const uint32_t j = L.big[jb];
            uint32_t e = j + 1;
            while (e < nt && K[e] == K[j]) ++e;
            tile_bitonic(T, j, e - j, x0, y0);
        }
        // the walk: position w of the tile in walking order is sorted rank w
        // (right region) or nt - 1 - w (left region); P_l, rank 0 of the left
        // region, is not walked
        const uint32_t nw = (r == 1 && plo == rs) ? nt - 1u : nt;
        BPt it[kCI];
        bool kp[kCI];
        BPt agg = bpt_none();
#pragma unroll
        for (int k = 0; k < kCI; ++k) {
            const uint32_t w = (uint32_t)(tid * kCI + k);
            it[k] = bpt_none();
            if (w < nw) {
                const double2 v = A.cd_xy[o + T.cpos[T.perm[r == 0 ? w : nt - 1u - w]]];
                it[k].x = v.x;
                it[k].y = v.y;
                it[k].v = true;
            }
            agg = bmax(agg, it[k], lx, ly, sgn);
        }
        BPt inc = agg;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const BPt q = shfl_up_bpt(inc, d);
            if (lane >= d) inc = bmax(q, inc, lx, ly, sgn);
        }
        BPt ex = shfl_up_bpt(inc, 1);
        if (lane == 0) ex = bpt_none();
        if (lane == 63) {
            L.wx[wave] = inc.x;
            L.wy[wave] = inc.y;
            L.wv[wave] = inc.v ? 1u : 0u;
        }
        __syncthreads();
        BPt run = carry, all = carry;
        for (int w = 0; w < kBW; ++w) {
            BPt q;
            q.x = L.wx[w];
            q.y = L.wy[w];
            q.v = L.wv[w] != 0u;
            if (w < wave) run = bmax(run, q, lx, ly, sgn);
            all = bmax(all, q, lx, ly, sgn);
        }
        run = bmax(run, ex, lx, ly, sgn);
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < kCI; ++k) {
            const uint32_t w = (uint32_t)(tid * kCI + k);
            kp[k] = false;
            if (w < nw) {
                kp[k] = (!run.v) || sgn * orient(lx, ly, run.x, run.y, it[k].x, it[k].y) >= 0;
                run = bmax(run, it[k], lx, ly, sgn);
                c += kp[k] ? 1u : 0u;
            }
        }
        // kept points in walking order
        const int lane_ = lane;
        (void)lane_;
        uint32_t tot;
        uint32_t off;
        {
            uint32_t incs = c;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t q = __shfl_up(incs, d);
                if (lane >= d) incs += q;
            }
            if (lane == 63) L.wsum[wave] = incs;
            __syncthreads();
            uint32_t pre = 0, t2 = 0;
            for (int w = 0; w < kBW; ++w) {
                const uint32_t x = L.wsum[w];
                if (w < wave) pre += x;
                t2 += x;
            }
            tot = t2;
            off = kept + pre + incs - c;
        }
#pragma unroll
        for (int k = 0; k < kCI; ++k) {
            const uint32_t w = (uint32_t)(tid * kCI + k);
            if (w < nw && kp[k]) {
                const uint32_t e = T.perm[r == 0 ? w : nt - 1u - w];
                const uint32_t pos = r == 0 ? rs + off : re - 1u - off;
                A.sv_xy[o + pos] = make_double2(it[k].x, it[k].y);
                A.sv_idx[o + pos] = T.idx[T.cpos[e]];
                ++off;
            }
        }
        kept += tot;
        carry = all;
        if (r == 0) lo_p = phi;
        else hi_p = plo;
        __syncthreads();
    }
    if (r == 1 && tid == 0) {
        const uint32_t pos = re - 1u - kept;
        A.sv_xy[o + pos] = make_double2(lx, ly);
        A.sv_idx[o + pos] = (uint32_t)W.P.l_idx;
    }
    if (r == 1) ++kept;
    if (tid == 0) {
        W.k[r] = kept;
        W.klo[r] = r == 0 ? rs : re - kept;
    }
}

// ---- the same for a region of at most 64 candidates, one wave per region
//      (eight per workgroup): a bitonic sort across the lanes, the walk as a
//      wave max-scan, the kept points by ballot
struct WItem {
    double x, y;
    uint32_t idx, key;
    bool inf;  // padding after every real entry
};

__device__ inline WItem shfl_item(const WItem& a, int src) {
    WItem r;
    r.x = __shfl(a.x, src);
    r.y = __shfl(a.y, src);
    r.idx = __shfl(a.idx, src);
    r.key = __shfl(a.key, src);
    r.inf = __shfl((int)a.inf, src) != 0;
    return r;
}

__device__ inline bool item_less(const WItem& a, const WItem& b, double x0, double y0) {
    if (a.inf) return false;
    if (b.inf) return true;
    if (a.key != b.key) return a.key < b.key;
    return angle_less(a.x, a.y, a.idx, b.x, b.y, b.idx, x0, y0);
}

__global__ __launch_bounds__(kBB) void k_wwalk_small(WideArgs A) {
    const int lane = (int)__lane_id();
    const uint32_t g = blockIdx.x * (uint32_t)kBW + (threadIdx.x >> 6);
    if (g >= 2u * (uint32_t)A.S) return;
    const int32_t s = A.order[g >> 1];
    const int r = (int)(g & 1u);
    const WSetIn in = A.in[s];
    if (in.n == 0) return;
    WSet& W = A.ws[s];
    if (W.flags != 0u || W.m1 == 0u) return;
    const uint32_t cnt = W.c[r];
    if (cnt > 64u) return;
    const uint32_t rs = r == 0 ? 0u : W.c[0], re = rs + cnt;
    const size_t o = (size_t)in.o;
    const double x0 = W.P.x0, y0 = W.P.y0, lx = W.P.lx, ly = W.P.ly;
    const int sgn = r == 0 ? 1 : -1;
    WItem me;
    me.x = me.y = 0.0;
    me.idx = me.key = 0;
    me.inf = (uint32_t)lane >= cnt;
    if (!me.inf) {
        const uint2 g = A.gk[o + rs + lane];
        const double2 v = A.cd_xy[o + g.y];
        me.x = v.x;
        me.y = v.y;
        me.idx = A.cd_idx[o + g.y];
        me.key = g.x;
    }
    for (int k = 2; k <= 64; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const WItem ot = shfl_item(me, lane ^ j);
            const bool low = (lane & j) == 0, asc = (lane & k) == 0;
            const bool take = low == asc ? item_less(ot, me, x0, y0) : item_less(me, ot, x0, y0);
            if (take) me = ot;
        }
    }
    // walking order: rank w (right region) or cnt - 1 - w (left region, whose
    // rank 0 is P_l: kept, not walked)
    const uint32_t nw = r == 0 ? cnt : (cnt > 0 ? cnt - 1u : 0u);
    const int src = r == 0 ? lane : (int)cnt - 1 - lane;
    const WItem w = shfl_item(me, src < 0 ? 0 : src);
    BPt it = bpt_none();
    if ((uint32_t)lane < nw) {
        it.x = w.x;
        it.y = w.y;
        it.v = true;
    }
    BPt inc = it;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const BPt q = shfl_up_bpt(inc, d);
        if (lane >= d) inc = bmax(q, inc, lx, ly, sgn);
    }
    BPt ex = shfl_up_bpt(inc, 1);
    if (lane == 0) ex = bpt_none();
    BPt run = bpt_none();
    if (r == 0) {
        run.x = x0;
        run.y = y0;
        run.v = true;
    }
    run = bmax(run, ex, lx, ly, sgn);
    const bool kp = (uint32_t)lane < nw &&
                    ((!run.v) || sgn * orient(lx, ly, run.x, run.y, it.x, it.y) >= 0);
    const uint64_t mask = __ballot(kp);
    const uint32_t off = (uint32_t)__popcll(mask & lanemask_lt());
    if (kp) {
        const uint32_t pos = r == 0 ? rs + off : re - 1u - off;
        A.sv_xy[o + pos] = make_double2(w.x, w.y);
        A.sv_idx[o + pos] = w.idx;
    }
    uint32_t kept = (uint32_t)__popcll(mask);
    if (r == 1) {
        if (lane == 0) {
            const uint32_t pos = re - 1u - kept;
            A.sv_xy[o + pos] = make_double2(lx, ly);
            A.sv_idx[o + pos] = (uint32_t)W.P.l_idx;
        }
        ++kept;
    }
    if (lane == 0) {
        W.k[r] = kept;
        W.klo[r] = r == 0 ? rs : re - kept;
    }
}

// ---- the same for a region with a bucket larger than a walk tile: the
//      per-set engine's stable radix sort in HBM, the exact order of equal
//      keys, its walk and removal (kept points ascending from the region's
//      first position); an equal-key run too long for the workgroup sends the
//      set to the host
__device__ __forceinline__ void walk_radix_region(const WideArgs& A, BatchLds& S, uint32_t g) {
    const int tid = (int)threadIdx.x;
    WRegion R;
    if (!wide_region(A, R, g)) return;
    WSet& W = A.ws[R.s];
    const WSetIn in = A.in[R.s];
    const size_t o = (size_t)in.o;
    const uint32_t cnt = R.cnt, rs = R.rs;
    const double x0 = W.P.x0, y0 = W.P.y0;
    uint32_t* K0 = A.ka + o + rs;
    uint32_t* V0 = A.va + o + rs;
    uint32_t* K1 = A.kb + o + rs;
    uint32_t* V1 = A.vb + o + rs;
    for (uint32_t i = (uint32_t)tid; i < cnt; i += kBB) {
        const uint2 gg = A.gk[o + rs + i];
        K0[i] = gg.x;
        V0[i] = gg.y;
    }
    __syncthreads();
    const int cur = wg_radix(S, K0, V0, K1, V1, cnt);
    const uint32_t* K = cur ? K1 : K0;
    uint32_t* V = cur ? V1 : V0;
    if (!wg_ties(S, K, V, cnt, A.cd_xy + o, A.cd_idx + o, x0, y0)) {
        if (tid == 0) atomicOr(&W.flags, kSetFallback);
        return;
    }
    wg_walk(S, V, cnt, R.r, A.cd_xy + o, A.flag + o + rs, x0, y0, W.P.lx, W.P.ly);
    const uint32_t end =
        wg_compact(S, V, A.flag + o + rs, cnt, A.cd_xy + o, A.cd_idx + o, A.sv_xy + o, A.sv_idx + o, rs);
    if (tid == 0) {
        W.k[R.r] = end - rs;
        W.klo[R.r] = rs;
    }
}

// ---- The regions with a sort bucket larger than a walk tile: Step 4 by the
//      persistent engine's radix sort in HBM, then the walk.  Such regions
//      are rare, so a small grid scans all regions (one per thread, kBB at a
//      time) and walks the ones found, one after another; a grid of one
//      workgroup per region would reserve this kernel's LDS for every region
//      only to return.
constexpr uint32_t kRadixGrid = 32;

__global__ __launch_bounds__(kBB) void k_wwalk_radix(WideArgs A) {
    __shared__ BatchLds S;
    __shared__ uint32_t s_list[kBB];
    __shared__ uint32_t s_n;
    const int tid = (int)threadIdx.x;
    const uint32_t nreg = 2u * (uint32_t)A.S;
    for (uint32_t base = blockIdx.x * (uint32_t)kBB; base < nreg; base += gridDim.x * (uint32_t)kBB) {
        if (tid == 0) s_n = 0u;
        __syncthreads();
        const uint32_t g = base + (uint32_t)tid;
        WRegion R;
        if (g < nreg && wide_region(A, R, g) && A.ws[R.s].big[R.r] > kCT) s_list[atomicAdd(&s_n, 1u)] = g;
        __syncthreads();
        const uint32_t nl = s_n;
        for (uint32_t q = 0; q < nl; ++q) {
            walk_radix_region(A, S, s_list[q]);
            __syncthreads();
        }
    }
}

// ---- Step 8 of a set over its kept points (right region, then the left)
constexpr uint32_t kStep8Wave = 63;  // kept lists up to this size: one wave per set (P_0 makes 64 entries)

// Kept points of a set after the walk (0 when nothing survived round 1).
__device__ inline uint32_t wide_kept(const WSet& W) { return W.m1 > 0 ? W.k[0] + W.k[1] : 0u; }

__global__ __launch_bounds__(kBB) __attribute__((amdgpu_waves_per_eu(4))) void k_wstep8(WideArgs A) {
    __shared__ BatchLds S;
    const int32_t s = A.order[blockIdx.x];
    const WSetIn in = A.in[s];
    const WSet& W = A.ws[s];
    // empty and flagged sets, and short kept lists: k_wstep8_small
    if (in.n == 0 || W.flags != 0u || wide_kept(W) <= kStep8Wave) return;
    const size_t o = (size_t)in.o;
    const uint32_t k0 = W.k[0], k1 = W.k[1];
    const uint32_t lo0 = W.klo[0], lo1 = W.klo[1];
    const uint32_t m = k0 + k1;
    HullSink H;
    H.hull = A.hull;
    H.cursor = A.hull_cursor;
    H.count = A.h_count;
    H.start = A.h_start;
    H.flags = A.h_flags;
    batch_step8<true>(S, H, s, A.sv_xy + o, A.sv_idx + o, KeptMap{lo0, k0, lo1}, m, A.ka + o, A.kb + o,
                      A.va + o, W.P.x0, W.P.y0, W.P.p0_idx);
}

// ---- Step 8 of a set whose kept list has at most kStep8Wave points, one
//      wave per set (eight per workgroup): the stack scan of P_0 and the kept
//      points run by the whole wave in step (every lane takes the same
//      decisions, points fetched from the lane that holds them), then the
//      rotation to the smallest vertex and the output.  Also writes the
//      result of empty and flagged sets.
__global__ __launch_bounds__(kBB) void k_wstep8_small(WideArgs A) {
    __shared__ uint8_t s_st[kBW][kStep8Wave];
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    const uint32_t g = blockIdx.x * (uint32_t)kBW + (uint32_t)wave;
    if (g >= (uint32_t)A.S) return;
    const int32_t s = A.order[g];
    const WSetIn in = A.in[s];
    const WSet& W = A.ws[s];
    if (in.n == 0 || W.flags != 0u) {
        if (lane == 0) {
            A.h_count[s] = 0;
            A.h_start[s] = 0;
            A.h_flags[s] = in.n == 0 ? 0u : W.flags;
        }
        return;
    }
    const uint32_t m = wide_kept(W);
    if (m > kStep8Wave) return;
    const size_t o = (size_t)in.o;
    const double x0 = W.P.x0, y0 = W.P.y0;
    double px = 0.0, py = 0.0;
    uint32_t pid = 0;
    if ((uint32_t)lane < m) {
        const uint32_t q = (uint32_t)lane < W.k[0] ? W.klo[0] + (uint32_t)lane : W.klo[1] + ((uint32_t)lane - W.k[0]);
        const double2 v = A.sv_xy[o + q];
        px = v.x;
        py = v.y;
        pid = A.sv_idx[o + q];
    }
    uint8_t* st = s_st[wave];
    uint32_t top = 0;                // stack entries above P_0
    double tx = x0, ty = y0, sx = x0, sy = y0;
    for (uint32_t i = 0; i < m; ++i) {
        const double qx = __shfl(px, (int)i), qy = __shfl(py, (int)i);
        if (qx == tx && qy == ty) continue;
        while (top >= 1) {
            if (orient(sx, sy, tx, ty, qx, qy) > 0) break;
            --top;
            tx = sx;
            ty = sy;
            if (top >= 2) {
                const int e = st[top - 2];
                sx = __shfl(px, e);
                sy = __shfl(py, e);
            } else {
                sx = x0;
                sy = y0;
            }
        }
        if (lane == 0) st[top] = (uint8_t)i;
        __builtin_amdgcn_wave_barrier();
        ++top;
        sx = tx;
        sy = ty;
        tx = qx;
        ty = qy;
    }
    __builtin_amdgcn_wave_barrier();
    const uint32_t h = top + 1;  // with P_0 as entry 0
    // entry k's point: P_0 for k = 0, else stack entry k - 1
    const int ek = lane >= 1 && (uint32_t)lane < h ? (int)st[lane - 1] : 0;
    const double ex = __shfl(px, ek), ey = __shfl(py, ek);
    const uint32_t eid = __shfl(pid, ek);
    double bx = lane == 0 ? x0 : ex, by = lane == 0 ? y0 : ey;
    uint32_t bk = (uint32_t)lane < h ? (uint32_t)lane : 0xFFFFFFFFu;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        const double ox = __shfl_xor(bx, d), oy = __shfl_xor(by, d);
        const uint32_t ok = __shfl_xor(bk, d);
        const bool take = ok != 0xFFFFFFFFu &&
                          (bk == 0xFFFFFFFFu || ox < bx || (ox == bx && (oy < by || (oy == by && ok < bk))));
        bx = take ? ox : bx;
        by = take ? oy : by;
        bk = take ? ok : bk;
    }
    uint32_t at = 0;
    if (lane == 0) at = atomicAdd(A.hull_cursor, h);
    at = __shfl(at, 0);
    const int32_t id_k = lane == 0 ? W.P.p0_idx : (int32_t)eid;
    if ((uint32_t)lane < h) {
        const uint32_t r = ((uint32_t)lane + h - bk) % h;  // output position of entry `lane`
        A.hull[at + r] = id_k;
    }
    if (lane == 0) {
        A.h_count[s] = (int32_t)h;
        A.h_start[s] = (int32_t)at;
        A.h_flags[s] = 0;
    }
}

}  // namespace

hipError_t launch_wide(const WideArgs& a, hipStream_t s) {
    if (a.S <= 0) return hipSuccess;
    const dim3 S1((unsigned)a.S), NT((unsigned)a.NT), S2((unsigned)(2 * a.S));
    hipLaunchKernelGGL(k_wprep, S1, dim3(kWB), 0, s, a);
    if (a.NT > 0) {
        if (a.items == 2) hipLaunchKernelGGL(k_wext<2>, NT, dim3(kWB), 0, s, a);
        else if (a.items == 8) hipLaunchKernelGGL(k_wext<8>, NT, dim3(kWB), 0, s, a);
        else hipLaunchKernelGGL(k_wext<4>, NT, dim3(kWB), 0, s, a);
    }
    hipLaunchKernelGGL(k_wparams, S1, dim3(64), 0, s, a);
    if (a.NT > 0) {
        if (a.items == 2) hipLaunchKernelGGL(k_wfilter<2>, NT, dim3(kWB), 0, s, a);
        else if (a.items == 8) hipLaunchKernelGGL(k_wfilter<8>, NT, dim3(kWB), 0, s, a);
        else hipLaunchKernelGGL(k_wfilter<4>, NT, dim3(kWB), 0, s, a);
    }
    hipLaunchKernelGGL(k_wfar, S1, dim3(64), 0, s, a);
    if (a.S_large > 0)
        hipLaunchKernelGGL((k_wset<kWideFilterBits, 1024>), dim3((unsigned)a.S_large), dim3(1024), 0, s, a);
    if (a.S > a.S_large)
        hipLaunchKernelGGL((k_wset<kSmallBits, 256>), dim3((unsigned)(a.S - a.S_large)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_wwalk_small, dim3((unsigned)((2 * a.S + kBW - 1) / kBW)), dim3(kBB), 0, s, a);
    hipLaunchKernelGGL(k_wwalk, S2, dim3(kBB), 0, s, a);
    hipLaunchKernelGGL(k_wwalk_radix, dim3(kRadixGrid), dim3(kBB), 0, s, a);
    hipLaunchKernelGGL(k_wstep8_small, dim3((unsigned)((a.S + kBW - 1) / kBW)), dim3(kBB), 0, s, a);
    hipLaunchKernelGGL(k_wstep8, S1, dim3(kBB), 0, s, a);
    return hipGetLastError();
}

}  // namespace hx
