// kernels_scan.hip - Step 8 of gScan (the final stack scan, Section 3) on the
// device, for one hull.
//
// Input: the points kept by round 2 in angular order about the pivot P_0
// (Step 4's order: angle, then distance along the ray, then index), P_0
// itself excluded; copies of one point are adjacent, the first of them has
// the smallest index.  Output: the canonical hull (counter-clockwise from the
// lexicographically smallest vertex, collinear points and later copies
// dropped), the same list the sequential scan of the kept points produces.
//
// Why it can be split.  For a contiguous piece Q of the kept list, the stack
// scan of P_0 followed by Q returns the strict corners of conv(P_0 + Q) (P_0
// is a hull corner and Q is in angular order), a convex chain after P_0.  The
// chains of two adjacent pieces A (earlier) and B combine into the chain of
// A + B by keeping a prefix a_1..a_i of A and a suffix b_j..b_q of B: the
// bridge a_i -> b_j is the common tangent.  For a point b beyond A, the
// prefix of A the scan keeps when b arrives is the longest one whose every
// step turns left before b (orient(a_{k-1}, a_k, b) > 0, with a_0 = P_0);
// this test is monotone in k (the edges of conv(P_0 + A) seen from b form
// one run), so a binary search finds it: i(b).  Seen from a point a before
// B, the turn a -> b_j -> b_{j+1} is likewise first never left, then always
// left.  The bridge is the unique b_j whose a = a_{i(b_j)} has
// a -> b_{j-1} -> b_j not a left turn and a -> b_j -> b_{j+1} a left turn
// (a pair of mutual tangents is the supporting line of both chains).  Ties
// follow the scan: a point on a line between two others is dropped.
//
// Kernel: each workgroup takes up to kScanPart consecutive kept points into
// LDS, drops repeats, scans chunks of kScanChunk points per thread (level 0),
// then combines neighbouring chains pairwise, one level per step, every
// thread taking the points of the later chains (one binary search each).
// With several workgroups, the last to finish (ticket) combines their chains
// the same way, rotates the result to the lexicographically smallest vertex
// and writes the input indices to host-visible memory.  If the chains of the
// parts do not fit one workgroup's LDS, it reports an overflow instead and
// the host scans the kept points itself.
#include <hip/hip_runtime.h>

#include "exact.hpp"
#include "kernels.hpp"

namespace hx {
namespace {

constexpr int kSB = 1024;            // threads per workgroup
constexpr int kSP = kScanPart;       // kept points per workgroup
constexpr int kSC = kSP / kSB;       // level-0 chunk per thread
static_assert(kSC * kSB == kSP, "chunks tile the part");
static_assert(kSP <= 65535, "16-bit positions");

struct ScanLds {
    double x[kSP];          // coordinates of the part (phase 2: of the parts' chains)
    double y[kSP];
    uint16_t pos[2][kSP];   // chain contents (positions into x / y), ping-pong
    uint16_t len[2][kSB];   // chain lengths, ping-pong
    uint16_t bi[kSB / 2];   // per pair of chains: A points kept, first B point kept
    uint16_t bj[kSB / 2];
    int32_t poff[kScanMaxParts + 1];  // phase 2: where each part's chain starts
    double rx[kSB / 64], ry[kSB / 64];
    int32_t rk[kSB / 64];
    uint32_t misc[4];
};

// The kept list: positions q -> (point, input index).  Either the one-
// workgroup tail's kept slots into the candidate arrays (right region in
// walking order, P_l, left region in reverse), or contiguous arrays.
struct Kept {
    const double2* xy;
    const uint32_t* idx_u;   // tail form
    const int32_t* idx_i;    // contiguous form
    const uint16_t* oslot;   // tail form: [2][kTailCap] slots
    uint32_t nr, lslot;
    __device__ uint32_t slot(uint32_t q) const {
        if (!oslot) return q;
        return q < nr ? (uint32_t)oslot[q] : q == nr ? lslot : (uint32_t)oslot[kTailCap + (q - nr - 1u)];
    }
    __device__ double2 pt(uint32_t q) const { return xy[slot(q)]; }
    __device__ int32_t id(uint32_t q) const {
        const uint32_t s = slot(q);
        return oslot ? (int32_t)idx_u[s] : idx_i[s];
    }
};

struct ScanArgs {
    Kept kept;
    uint32_t m;                 // contiguous form: kept points (tail form: read from the statuses)
    const DevStatus* ds;        // [2]: round 1, candidates
    const uint32_t* ocount;     // tail form: kept per region
    double x0, y0;              // contiguous form: the pivot (tail form: from ds)
    int32_t p0_idx;
    double2* part_xy;           // the parts' chains (at each part's first position)
    uint32_t* part_idx;
    uint32_t* part_len;         // [kScanMaxParts]
    uint32_t* ticket;           // zero between launches
    int32_t* out;               // hull indices (host-visible)
    DevStatus* host_ds;         // tail form: both statuses are copied here; contiguous: [1] patched
};

// Chains of level-0 chunks: chain t of level L covers positions
// [t * kSC * 2^L, (t + 1) * kSC * 2^L) of the part.
struct FixedGeo {
    __device__ int start(int L, int t) const { return (t * kSC) << L; }
    __device__ int chain_of(int L, int s) const { return (s / kSC) >> L; }
};

// Chains of the parts (phase 2): chain t of level L starts where part
// t * 2^L's chain starts.
struct PartGeo {
    const int32_t* off;
    int parts;
    __device__ int start(int L, int t) const { return off[t << L]; }
    __device__ int chain_of(int L, int s) const {
        int lo = 0, hi = parts - 1;  // last part whose chain starts at or before s
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= s) lo = mid;
            else hi = mid - 1;
        }
        return lo >> L;
    }
};

// Combines the T chains in S.pos[cur] (lengths S.len[cur]) pairwise until
// one is left; np positions in use.  Returns the buffer holding the result
// (its chain 0).
template <class Geo>
__device__ int combine(ScanLds& S, const Geo& geo, int T, int np, double x0, double y0, int cur) {
    const int tid = (int)threadIdx.x;
    for (int L = 0; (1 << L) < T; ++L) {
        const int TL = (T + (1 << L) - 1) >> L;
        const uint16_t* P = S.pos[cur];
        const uint16_t* len = S.len[cur];
        // no bridge found (B empty): all of A, none of B
        for (int t = tid; t < TL / 2; t += kSB) {
            S.bi[t] = len[2 * t];
            S.bj[t] = len[2 * t + 1];
        }
        __syncthreads();
        for (int s = tid; s < np; s += kSB) {
            const int c = geo.chain_of(L, s);
            if ((c & 1) == 0) continue;
            const int j = s - geo.start(L, c);
            const int q = len[c];
            if (j >= q) continue;
            const int sa = geo.start(L, c - 1);
            const int p = len[c - 1];
            const int pb = P[s];
            const double bx = S.x[pb], by = S.y[pb];
            // i(b): the first k whose step a_{k-1} -> a_k does not turn left before b
            int lo = 0, hi = p;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                const int pk = P[sa + mid];
                double px = x0, py = y0;
                if (mid > 0) {
                    const int pp = P[sa + mid - 1];
                    px = S.x[pp];
                    py = S.y[pp];
                }
                if (orient(px, py, S.x[pk], S.y[pk], bx, by) > 0) lo = mid + 1;
                else hi = mid;
            }
            const int i = lo;
            double ax = x0, ay = y0;
            if (i > 0) {
                const int pa = P[sa + i - 1];
                ax = S.x[pa];
                ay = S.y[pa];
            }
            bool bridge = true;
            if (j > 0) {
                const int pp = P[s - 1];
                bridge = orient(ax, ay, S.x[pp], S.y[pp], bx, by) <= 0;
            }
            if (bridge && j + 1 < q) {
                const int pn = P[s + 1];
                bridge = orient(ax, ay, bx, by, S.x[pn], S.y[pn]) > 0;
            }
            if (bridge) {
                S.bi[c >> 1] = (uint16_t)i;
                S.bj[c >> 1] = (uint16_t)j;
            }
        }
        __syncthreads();
        uint16_t* Q = S.pos[cur ^ 1];
        for (int s = tid; s < np; s += kSB) {
            const int c = geo.chain_of(L, s);
            const int k = s - geo.start(L, c);
            if (k >= len[c]) continue;
            int dst = -1;
            if ((c & 1) == 0) {
                if (c + 1 >= TL || k < S.bi[c >> 1]) dst = s;
            } else if (k >= S.bj[c >> 1]) {
                dst = geo.start(L, c - 1) + S.bi[c >> 1] + (k - S.bj[c >> 1]);
            }
            if (dst >= 0) Q[dst] = P[s];
        }
        for (int t = tid; t < (TL + 1) / 2; t += kSB) {
            const int b = 2 * t + 1;
            S.len[cur ^ 1][t] = b < TL ? (uint16_t)(S.bi[t] + (len[b] - S.bj[t])) : len[2 * t];
        }
        __syncthreads();
        cur ^= 1;
    }
    return cur;
}

// The hull is P_0 followed by the chain (positions P[0..len)): rotated to its
// lexicographically smallest vertex, its input indices written to out.
template <class IdOf>
__device__ uint32_t emit(ScanLds& S, const uint16_t* P, int len, double x0, double y0, int32_t p0_idx,
                         const IdOf& id_of, int32_t* out) {
    const int tid = (int)threadIdx.x, lane = (int)__lane_id(), wave = tid >> 6;
    const int h = len + 1;
    double bx = 0.0, by = 0.0;
    int bk = -1;
    for (int k = tid; k < h; k += kSB) {
        double x = x0, y = y0;
        if (k > 0) {
            x = S.x[P[k - 1]];
            y = S.y[P[k - 1]];
        }
        const bool take = bk < 0 || x < bx || (x == bx && y < by);
        bx = take ? x : bx;
        by = take ? y : by;
        bk = take ? k : bk;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        const double ox = __shfl_xor(bx, d), oy = __shfl_xor(by, d);
        const int ok = __shfl_xor(bk, d);
        const bool take = ok >= 0 && (bk < 0 || ox < bx || (ox == bx && oy < by));
        bx = take ? ox : bx;
        by = take ? oy : by;
        bk = take ? ok : bk;
    }
    if (lane == 0) {
        S.rx[wave] = bx;
        S.ry[wave] = by;
        S.rk[wave] = bk;
    }
    __syncthreads();
    if (tid == 0) {
        double x = S.rx[0], y = S.ry[0];
        int k = S.rk[0];
        for (int w = 1; w < kSB / 64; ++w) {
            const int ok = S.rk[w];
            const bool take = ok >= 0 && (k < 0 || S.rx[w] < x || (S.rx[w] == x && S.ry[w] < y));
            x = take ? S.rx[w] : x;
            y = take ? S.ry[w] : y;
            k = take ? ok : k;
        }
        S.misc[0] = (uint32_t)k;
    }
    __syncthreads();
    const int start = (int)S.misc[0];
    for (int k = tid; k < h; k += kSB) {
        int v = start + k;
        v = v >= h ? v - h : v;
        out[k] = v == 0 ? p0_idx : id_of(P[v - 1]);
    }
    return (uint32_t)h;
}

// The statuses for the host: both problems' words, with the kept count, the
// hull size and the scan's state in the candidate problem's.
__device__ void publish(const DevStatus* ds, DevStatus* host_ds, bool full_copy, uint32_t m, uint32_t h,
                        uint32_t state) {
    const int tid = (int)threadIdx.x;
    constexpr int W = (int)(sizeof(DevStatus) / sizeof(uint32_t));
    if (full_copy && tid < 2 * W) {
        uint32_t v = reinterpret_cast<const uint32_t*>(ds)[tid];
        if (tid == W + (int)(offsetof(DevStatus, n_kept) / sizeof(uint32_t)) && state != kScanNone) v = m;
        if (tid == W + (int)(offsetof(DevStatus, n_hull) / sizeof(uint32_t))) v = h;
        if (tid == W + (int)(offsetof(DevStatus, scan_state) / sizeof(uint32_t))) v = state;
        reinterpret_cast<uint32_t*>(host_ds)[tid] = v;
    }
    if (!full_copy && tid == 0) {
        host_ds[1].n_hull = h;
        host_ds[1].scan_state = state;
    }
}

__global__ __launch_bounds__(kSB) void k_scan(ScanArgs A) {
    __shared__ ScanLds S;
    const int tid = (int)threadIdx.x;
    const int g = (int)blockIdx.x;
    const bool tail = A.kept.oslot != nullptr;
    Kept K = A.kept;
    uint32_t m = A.m;
    double x0 = A.x0, y0 = A.y0;
    int32_t p0_idx = A.p0_idx;
    if (tail) {
        const DevStatus* ds2 = A.ds + 1;
        if (ds2->tail_state != kTailDone) {
            // the tail gave up: the multi-kernel path follows on the host
            if (g == 0) publish(A.ds, A.host_ds, true, 0u, 0u, kScanNone);
            return;
        }
        const uint32_t nc = ds2->n_sorted;
        K.nr = nc > 0 ? A.ocount[0] : 0u;
        K.lslot = ds2->l_slot;
        m = nc > 0 ? K.nr + 1u + A.ocount[1] : 0u;
        x0 = A.ds[0].x0;
        y0 = A.ds[0].y0;
        p0_idx = A.ds[0].p0_idx;
    }
    const int parts = m == 0 ? 1 : (int)((m + kSP - 1) / kSP);
    if (g >= parts) return;
    const uint32_t base = (uint32_t)g * kSP;
    const int np = (int)min((uint32_t)kSP, m - min(m, base));

    // ---- the part's points, then the level-0 chunk scans ------------------
    for (int s = tid; s < np; s += kSB) {
        const double2 p = K.pt(base + (uint32_t)s);
        S.x[s] = p.x;
        S.y[s] = p.y;
    }
    if (tid == 0) {
        // the point before the part, for the repeat test of its first point
        uint32_t f = 0u;
        if (base > 0 && np > 0) {
            const double2 p = K.pt(base - 1u);
            f = (p.x == K.pt(base).x && p.y == K.pt(base).y) ? 1u : 0u;
        }
        S.misc[1] = f;
    }
    __syncthreads();
    const int T = (np + kSC - 1) / kSC;
    int cur = 0;
    if (tid < T) {
        uint16_t* stk = &S.pos[0][tid * kSC];
        int depth = 0;
        for (int k = 0; k < kSC; ++k) {
            const int s = tid * kSC + k;
            if (s >= np) break;
            const double px = S.x[s], py = S.y[s];
            const bool rep = s > 0 ? (S.x[s - 1] == px && S.y[s - 1] == py) : S.misc[1] != 0u;
            if (rep) continue;
            while (depth > 0) {
                const int b = stk[depth - 1];
                double ax = x0, ay = y0;
                if (depth > 1) {
                    const int a = stk[depth - 2];
                    ax = S.x[a];
                    ay = S.y[a];
                }
                if (orient(ax, ay, S.x[b], S.y[b], px, py) > 0) break;
                --depth;
            }
            stk[depth++] = (uint16_t)s;
        }
        S.len[0][tid] = (uint16_t)depth;
    }
    __syncthreads();
    cur = combine(S, FixedGeo{}, T, np, x0, y0, cur);
    const int clen = T > 0 ? (int)S.len[cur][0] : 0;

    if (parts == 1) {
        const uint32_t h = emit(S, S.pos[cur], clen, x0, y0, p0_idx,
                                [&](int s) { return K.id((uint32_t)s); }, A.out);
        __syncthreads();
        publish(A.ds, A.host_ds, tail, m, h, kScanDone);
        return;
    }

    // ---- several parts: store this part's chain, the last part combines ---
    for (int k = tid; k < clen; k += kSB) {
        const int s = S.pos[cur][k];
        A.part_xy[base + (uint32_t)k] = make_double2(S.x[s], S.y[s]);
        A.part_idx[base + (uint32_t)k] = (uint32_t)K.id(base + (uint32_t)s);
    }
    if (tid == 0) A.part_len[g] = (uint32_t)clen;
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        const uint32_t t = __hip_atomic_fetch_add(A.ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        const bool last = t == (uint32_t)parts - 1u;
        if (last) __hip_atomic_store(A.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        S.misc[2] = last ? 1u : 0u;
    }
    __syncthreads();
    if (S.misc[2] == 0u) return;
    __threadfence();

    // ---- phase 2 (last workgroup): the parts' chains into LDS --------------
    if (tid == 0) {
        int o = 0;
        for (int p = 0; p < parts; ++p) {
            S.poff[p] = o;
            o += (int)__hip_atomic_load(&A.part_len[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        S.poff[parts] = o;
    }
    __syncthreads();
    const int total = S.poff[parts];
    if (total > kSP) {
        // does not fit: the host scans the kept points
        publish(A.ds, A.host_ds, tail, m, 0u, kScanOverflow);
        return;
    }
    for (int p = 0; p < parts; ++p) {
        const int o = S.poff[p], L = S.poff[p + 1] - o;
        for (int k = tid; k < L; k += kSB) {
            const double2 v = A.part_xy[(uint32_t)p * kSP + (uint32_t)k];
            S.x[o + k] = v.x;
            S.y[o + k] = v.y;
            S.pos[0][o + k] = (uint16_t)(o + k);
        }
        if (tid == 0) S.len[0][p] = (uint16_t)L;
    }
    __syncthreads();
    const PartGeo geo{S.poff, parts};
    cur = combine(S, geo, parts, total, x0, y0, 0);
    const uint32_t h = emit(S, S.pos[cur], (int)S.len[cur][0], x0, y0, p0_idx,
                            [&](int s) {
                                const int p = geo.chain_of(0, s);
                                return (int32_t)A.part_idx[(uint32_t)p * kSP + (uint32_t)(s - S.poff[p])];
                            },
                            A.out);
    __syncthreads();
    publish(A.ds, A.host_ds, tail, m, h, kScanDone);
}

}  // namespace

hipError_t launch_scan_tail(const double2* cand_xy, const uint32_t* cand_idx, const uint16_t* oslot,
                            const uint32_t* ocount, const DevStatus* ds, double2* part_xy,
                            uint32_t* part_idx, uint32_t* part_len, uint32_t* ticket, int32_t* out,
                            DevStatus* host_ds, hipStream_t s) {
    ScanArgs A{};
    A.kept.xy = cand_xy;
    A.kept.idx_u = cand_idx;
    A.kept.oslot = oslot;
    A.ds = ds;
    A.ocount = ocount;
    A.part_xy = part_xy;
    A.part_idx = part_idx;
    A.part_len = part_len;
    A.ticket = ticket;
    A.out = out;
    A.host_ds = host_ds;
    const int grid = (int)ceil_div(2 * (int64_t)kTailCap + 1, kSP);
    hipLaunchKernelGGL(k_scan, dim3(grid), dim3(kSB), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_scan_list(const double2* kept_xy, const int32_t* kept_idx, int64_t m, double x0,
                            double y0, int32_t p0_idx, const DevStatus* ds, double2* part_xy,
                            uint32_t* part_idx, uint32_t* part_len, uint32_t* ticket, int32_t* out,
                            DevStatus* host_ds, hipStream_t s) {
    if (m < 0 || m > (int64_t)kScanMaxParts * kSP) return hipErrorInvalidValue;
    ScanArgs A{};
    A.kept.xy = kept_xy;
    A.kept.idx_i = kept_idx;
    A.m = (uint32_t)m;
    A.x0 = x0;
    A.y0 = y0;
    A.p0_idx = p0_idx;
    A.ds = ds;
    A.part_xy = part_xy;
    A.part_idx = part_idx;
    A.part_len = part_len;
    A.ticket = ticket;
    A.out = out;
    A.host_ds = host_ds;
    const int grid = (int)std::max<int64_t>(1, ceil_div(m, kSP));
    hipLaunchKernelGGL(k_scan, dim3(grid), dim3(kSB), 0, s, A);
    return hipGetLastError();
}

}  // namespace hx
