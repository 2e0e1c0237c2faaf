// hull2d_api.cpp - C ABI of the exact 2D hull library (include/hull2d.h):
// context and workspace management, the per-call pipeline of gfx950 kernels,
// and the final Graham stack scan on the host (Step 8 of gScan, Section 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "exact.hpp"
#include "hull2d.h"
#include "kernels.hpp"

using namespace hx;

// A point of the four-region variant's final stage on the host.
struct HostPt {
    double x, y;
    int32_t i;
};

// The device buffers of one hull2d_compute call, carved out of one block of
// device memory: the context's own allocation (grown on demand), or the
// library's fixed scratch array for the no-allocation entry point.
struct Workspace {
    Cand* partial = nullptr;
    Params* prm = nullptr;
    DevStatus* ds = nullptr;
    uint32_t* hist = nullptr;
    double2* comp_xy = nullptr;
    uint32_t* comp_idx = nullptr;
    uint32_t *keys_a = nullptr, *keys_b = nullptr, *vals_a = nullptr, *vals_b = nullptr;
    uint64_t* stat = nullptr;
    size_t stat_bytes = 0;
    uint32_t* long_list = nullptr;
    uint32_t* huge_list = nullptr;
    uint8_t* keep = nullptr;
    double2* out_xy = nullptr;
    int32_t* out_idx = nullptr;
    double2* cand_xy = nullptr;   // round-2 candidates of the bucketed filter
    uint32_t* cand_idx = nullptr;
    uint32_t* cand_key = nullptr;
    uint32_t* cand_kap = nullptr;
    uint16_t* tail_slot = nullptr;  // the tail's kept slots [2][kTailCap], then two counts
    uint32_t* tail_count = nullptr;
    uint32_t* bmax = nullptr;     // sampled bucket maxima, then those over the candidates
    uint32_t* prefix = nullptr;
    uint32_t* seg_count = nullptr;  // round-1 segments (one per filter block)
    uint32_t* seg_off = nullptr;
    double* blk_d2 = nullptr;
    uint32_t* blk_best = nullptr;
    uint32_t* part_len = nullptr;  // device Step 8: chain length of each part
    ChainTables chain{};           // the four-region variant
    // epoch counter of the look-back words in `stat` (a word is ready only
    // for the epoch that wrote it)
    uint32_t* epoch = nullptr;
};

struct hull2d_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hull2d_options opt{};
    int cu_count = 256;
    Occupancy occ;
    bool broken = false;

    // device workspace (grows on demand)
    int64_t cap_n = -1;
    char* dmem = nullptr;
    Workspace own{};
    uint32_t own_epoch = 0;
    Counters* ctr = nullptr;  // separate allocation, zeroed once, persists

    // pinned host buffers (h_ds holds the two problem statuses; the tail
    // writes them itself through h_ds_dev)
    DevStatus* h_ds = nullptr;
    DevStatus* h_ds_dev = nullptr;
    double2* h_xy = nullptr;
    int32_t* h_idx = nullptr;
    int32_t* h_hull = nullptr;     // the hull written by the device Step 8
    double2* h_xy_dev = nullptr;   // the same buffers as the device addresses them
    int32_t* h_idx_dev = nullptr;
    int32_t* h_hull_dev = nullptr;
    int64_t h_cap = 0;

    uint32_t epoch = 0;
    hipEvent_t ev[HULL2D_NUM_STAGES + 2] = {};  // per stage, then begin and end
    bool have_events = false;

    hipEvent_t ev_sync = nullptr;  // spin-waited: a sleeping wait can add milliseconds
    std::vector<int64_t> stk;      // host scan buffers, reused across calls
    std::vector<int32_t> hull;
    std::vector<uint32_t> huge_host;  // the list of over-long equal-key runs
    // four-region variant: what its last kernel leaves in host memory, the
    // kept lists that did not fit there, the final stage's stack
    ChainHost* h_chain = nullptr;
    ChainHost* h_chain_dev = nullptr;
    std::vector<double2> chain_xy;
    std::vector<int32_t> chain_ix;
    std::vector<HostPt> cstk;
    bool last_chain = false;
    ChainHost last_chain_host{};
    // created with reserve_noalloc: every host buffer above holds
    // HULL2D_NOALLOC_MAX_POINTS points, so hull2d_compute_noalloc grows none
    bool noalloc_ready = false;

    // batched form: workspace over all points of a batch, per-set results
    int64_t bcap_n = -1;
    int32_t bcap_s = -1;
    char* bmem = nullptr;
    double2 *b_sv_xy = nullptr, *b_cd_xy = nullptr;
    uint32_t *b_sv_idx = nullptr, *b_sv_key = nullptr, *b_cd_idx = nullptr, *b_cd_key = nullptr;
    uint32_t *b_ka = nullptr, *b_kb = nullptr, *b_va = nullptr, *b_vb = nullptr;
    uint2* b_gk = nullptr;         // tiled engine: candidates by bucket (key, position)
    uint8_t* b_flag = nullptr;
    int32_t* b_hull = nullptr;
    int64_t* b_offs = nullptr;
    int32_t* b_order = nullptr;
    int32_t* b_meta = nullptr;     // [cursor, count[S], start[S], flags[S]]
    int64_t hb_cap_s = -1;         // pinned host staging
    int64_t* hb_offs = nullptr;
    int32_t* hb_order = nullptr;
    int32_t* hb_meta = nullptr;
    int64_t hb_cap_h = -1;
    int32_t* hb_hull = nullptr;
    WSetIn* hb_win = nullptr;      // tiled engine: per-set layout (hb_cap_s entries)
    int batch_grid = 0;
    // tiled engine: per-set records, tile arrays, bucket tables
    int64_t wcap_s = -1, wcap_nt = -1, wcap_se = -1;
    char* wmem = nullptr;
    WSetIn* w_in = nullptr;
    WSet* w_set = nullptr;
    int32_t* w_tile_set = nullptr;
    Cand* w_tile_ext = nullptr;
    uint32_t* w_tile_flags = nullptr;
    WFar* w_tile_far = nullptr;
    uint32_t* w_tile_cnt = nullptr;
    uint32_t* w_bcnt = nullptr;
    // the batched form's device work captured in a graph, and what it was
    // captured for (replayed while all of it is unchanged)
    hipStream_t cap_stream = nullptr;
    // tiled batch engine: the largest sets run on a second stream beside the
    // others (default priority), joined by events
    hipStream_t side_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipGraphExec_t bgraph = nullptr;
    bool bgraph_off = false;  // capture failed once: plain stream work
    int32_t bg_S = -1;
    int64_t bg_N = -1;
    const double* bg_xy = nullptr;
    const void* bg_ws = nullptr;  // device workspace
    const void* bg_hb = nullptr;  // pinned staging
    int bg_grid = 0;
    int bg_engine = -1;
    int64_t bg_nt = -1, bg_nt_big = -1;
    int32_t bg_big = -1;
    int32_t bg_large[2] = {-1, -1};
    const void* bg_wm = nullptr;  // tiled engine's workspace

    // learned filter: weights (float32 master + bfloat16 inference copies),
    // optimiser state, the per-call proposal, training activations
    bool have_weights = false;
    char* lmem = nullptr;
    float *m_params = nullptr, *m_grad = nullptr, *m_am = nullptr, *m_av = nullptr;
    uint16_t *m_w1 = nullptr, *m_w2 = nullptr, *m_w3 = nullptr;
    LearnOut* learn = nullptr;
    uint32_t* l_hist = nullptr;
    float* l_loss = nullptr;
    double* l_part = nullptr;
    int64_t adam_t = 0;
    int32_t tcap_b = 0;
    char* tmem = nullptr;
    float *t_h1 = nullptr, *t_h2 = nullptr, *t_y = nullptr, *t_d3 = nullptr, *t_d2 = nullptr,
          *t_d1 = nullptr;
    bool last_learned = false;

    // the last compute call, for hull2d_debug_stages
    bool have_last = false;
    Workspace last_ws{};
    bool last_full = false;
    bool last_tail = false;  // the one-workgroup tail finished the last call
    int64_t last_n = 0;
    int last_segs = 0;  // round-1 segments of the last call
    DevStatus last_ds{}, last_ds2{};
};

namespace {

constexpr int kMaxSegs = 8192;  // round-1 blocks (resident blocks of the whole chip) at most
// Step 8 on the device by default from this many kept points on (the host
// scan is faster below; measured on the 20M square and disk)
constexpr int64_t kScanAutoMin = 65536;

constexpr size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
constexpr size_t cdiv(size_t a, size_t b) { return (a + b - 1) / b; }
constexpr size_t smax(size_t a, size_t b) { return a > b ? a : b; }

struct Layout {
    size_t off[29];
    size_t total;
};

// Offsets of the workspace arrays for inputs of up to n points.
constexpr Layout plan(int64_t n) {
    const size_t N = (size_t)(n > 0 ? n : 1);
    size_t stat_words = cdiv(N, kSortTile) * 256;
    stat_words = smax(stat_words, cdiv(N, kF1Tile) + 2);
    stat_words = smax(stat_words, cdiv(N, kR2Tile) + 4);
    stat_words = smax(stat_words, cdiv(N, kCpTile) + 2);
    const size_t sizes[29] = {
        (size_t)kExtGridMax * 4 * sizeof(Cand),      // 0 partial
        sizeof(Params),                              // 1
        2 * sizeof(DevStatus),                       // 2 round-1 problem, candidate problem
        4 * 256 * sizeof(uint32_t),                  // 3 hist
        N * sizeof(double2),                         // 4 comp_xy
        N * sizeof(uint32_t),                        // 5 comp_idx
        N * sizeof(uint32_t),                        // 6 keys_a
        N * sizeof(uint32_t),                        // 7 keys_b
        N * sizeof(uint32_t),                        // 8 vals_a
        N * sizeof(uint32_t),                        // 9 vals_b
        stat_words * sizeof(uint64_t),               // 10 stat
        (size_t)kMaxSegs * sizeof(double),           // 11 blk_d2
        (size_t)kMaxSegs * 2 * sizeof(uint32_t),     // 12 blk_best
        (N / (kRunSmall + 1) + 2) * sizeof(uint32_t),  // 13 long_list
        (N / kRunCap + 2) * 2 * sizeof(uint32_t),    // 14 huge_list
        align_up(N, kCpTile) + kCpTile,              // 15 keep (padded for 16-byte loads)
        N * sizeof(double2),                         // 16 out_xy
        N * sizeof(int32_t),                         // 17 out_idx
        N * sizeof(double2),                         // 18 cand_xy
        N * sizeof(uint32_t),                        // 19 cand_idx
        N * sizeof(uint32_t),                        // 20 cand_key
        2 * kBuckets * sizeof(uint32_t),             // 21 bmax
        2 * kBuckets * sizeof(uint32_t),             // 22 prefix
        (size_t)kMaxSegs * sizeof(uint32_t),         // 23 seg_count
        (size_t)kMaxSegs * sizeof(uint32_t),         // 24 seg_off
        N * sizeof(uint32_t),                        // 25 cand_kap
        2 * (size_t)kTailCap * sizeof(uint16_t) + 2 * sizeof(uint32_t),  // 26 tail slots, counts
        (size_t)kScanMaxParts * sizeof(uint32_t),    // 27 part_len (device Step 8)
        kChainTableBytes};                           // 28 tables of the four-region variant
    Layout L{};
    size_t o = 0;
    for (int i = 0; i < 29; ++i) {
        L.off[i] = o;
        o = align_up(o + sizes[i], 256);
    }
    L.total = o;
    return L;
}

// Points the workspace arrays into `b`, laid out for up to n points.
void carve(char* b, int64_t n, Workspace& w) {
    const Layout L = plan(n);
    w.partial = (Cand*)(b + L.off[0]);
    w.prm = (Params*)(b + L.off[1]);
    w.ds = (DevStatus*)(b + L.off[2]);
    w.hist = (uint32_t*)(b + L.off[3]);
    w.comp_xy = (double2*)(b + L.off[4]);
    w.comp_idx = (uint32_t*)(b + L.off[5]);
    w.keys_a = (uint32_t*)(b + L.off[6]);
    w.keys_b = (uint32_t*)(b + L.off[7]);
    w.vals_a = (uint32_t*)(b + L.off[8]);
    w.vals_b = (uint32_t*)(b + L.off[9]);
    w.stat = (uint64_t*)(b + L.off[10]);
    w.stat_bytes = L.off[11] - L.off[10];
    w.blk_d2 = (double*)(b + L.off[11]);
    w.blk_best = (uint32_t*)(b + L.off[12]);
    w.long_list = (uint32_t*)(b + L.off[13]);
    w.huge_list = (uint32_t*)(b + L.off[14]);
    w.keep = (uint8_t*)(b + L.off[15]);
    w.out_xy = (double2*)(b + L.off[16]);
    w.out_idx = (int32_t*)(b + L.off[17]);
    w.cand_xy = (double2*)(b + L.off[18]);
    w.cand_idx = (uint32_t*)(b + L.off[19]);
    w.cand_key = (uint32_t*)(b + L.off[20]);
    w.bmax = (uint32_t*)(b + L.off[21]);
    w.prefix = (uint32_t*)(b + L.off[22]);
    w.seg_count = (uint32_t*)(b + L.off[23]);
    w.seg_off = (uint32_t*)(b + L.off[24]);
    w.cand_kap = (uint32_t*)(b + L.off[25]);
    w.tail_slot = (uint16_t*)(b + L.off[26]);
    w.tail_count = (uint32_t*)(b + L.off[26] + 2 * (size_t)kTailCap * sizeof(uint16_t));
    w.part_len = (uint32_t*)(b + L.off[27]);
    char* t = b + L.off[28];
    const size_t B4 = 4 * (size_t)kChainBuckets;
    w.chain.bmin = (uint64_t*)t;
    w.chain.prefix = (double*)(t + B4 * 8);
    w.chain.count = (uint32_t*)(t + B4 * 16);
    w.chain.cursor = (uint32_t*)(t + B4 * 20);
    w.chain.offset = (uint32_t*)(t + B4 * 24);
    const size_t tiles = B4 / 1024;
    w.chain.tile_min = (double*)(t + align_up(B4 * 28 + 4, 64));
    w.chain.tile_sum = (uint32_t*)(t + align_up(B4 * 28 + 4, 64) + tiles * 8);
    w.chain.st = (ChainStatus*)(t + align_up(B4 * 28 + 4 + tiles * 12, 64) + 64);
}

hull2d_status ensure_workspace(hull2d_ctx* c, int64_t n) {
    if (n <= c->cap_n) return HULL2D_OK;
    int64_t want = n;
    if (c->cap_n > 0 && want < c->cap_n + c->cap_n / 4) want = c->cap_n + c->cap_n / 4;
    Layout L = plan(want);
    const size_t limit = c->opt.workspace_limit_mib > 0 ? (size_t)c->opt.workspace_limit_mib << 20 : 0;
    if (limit && L.total > limit && want > n) {
        want = n;  // no headroom within the limit
        L = plan(want);
    }
    if (limit && L.total > limit) return HULL2D_ERR_OUT_OF_MEMORY;  // the old workspace stays
    if (c->dmem) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(c->dmem);
        c->dmem = nullptr;
        c->cap_n = -1;
    }
    if (hipMalloc((void**)&c->dmem, L.total) != hipSuccess) {
        (void)hipGetLastError();
        c->dmem = nullptr;
        return HULL2D_ERR_OUT_OF_MEMORY;
    }
    carve(c->dmem, want, c->own);
    c->own.epoch = &c->own_epoch;
    // Look-back words carry the call's epoch; zero means "not ready" for any epoch.
    if (hipMemsetAsync(c->own.stat, 0, c->own.stat_bytes, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        c->broken = true;
        return HULL2D_ERR_DEVICE;
    }
    c->cap_n = want;
    return HULL2D_OK;
}

// ---- the no-allocation entry point's fixed device workspace --------------
// One array per device (each device that loads the library holds its own
// copy until the process ends), laid out by plan() for the largest input the
// entry point accepts.  Its host-side name is not a device address: host code
// uses only the address hipGetSymbolAddress returns for the current device.
constexpr int64_t kNoAllocMax = HULL2D_NOALLOC_MAX_POINTS;
constexpr size_t kScratchBytes = plan(kNoAllocMax).total;
static_assert(kScratchBytes <= (size_t)32 << 20, "scratch stays modest");
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
// look-back epochs of each device's scratch, shared by all contexts on it
uint32_t g_scratch_epoch[kMaxDevices] = {};

// Looks up the scratch array's address on `device` (which must be current)
// once, at context creation.  False if the runtime refused.
bool init_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return false;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return true;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return false;
    }
    g_scratch_ptr[device] = p;
    return true;
}

void* scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

// The next look-back epoch of workspace w.  A look-back word keeps 30 bits
// of the epoch that wrote it; when the counter comes round to a multiple of
// 2^30 the words are cleared first (by a kernel), so that a word left by an
// earlier launch never looks ready.
uint32_t next_epoch(hull2d_ctx* c, Workspace& w) {
    uint32_t e = __atomic_add_fetch(w.epoch, 1u, __ATOMIC_RELAXED);
    if ((e & 0x3FFFFFFFu) == 0u) {
        if (launch_clear_words(w.stat, w.stat_bytes / sizeof(uint64_t), c->stream) != hipSuccess) {
            (void)hipGetLastError();
            c->broken = true;
        }
        e = __atomic_add_fetch(w.epoch, 1u, __ATOMIC_RELAXED);
    }
    return e;
}

hull2d_status ensure_host(hull2d_ctx* c, int64_t m) {
    if (m <= c->h_cap) return HULL2D_OK;
    int64_t want = std::max<int64_t>(m, 4096);
    if (c->h_xy) (void)hipHostFree(c->h_xy);
    if (c->h_idx) (void)hipHostFree(c->h_idx);
    if (c->h_hull) (void)hipHostFree(c->h_hull);
    c->h_xy = nullptr;
    c->h_idx = nullptr;
    c->h_hull = nullptr;
    c->h_cap = 0;
    // mapped and coherent: the device writes the kept points or the hull
    // here directly, saving a copy and a wait
    const unsigned fl = hipHostMallocMapped | hipHostMallocCoherent;
    if (hipHostMalloc((void**)&c->h_xy, (size_t)want * sizeof(double2), fl) != hipSuccess ||
        hipHostMalloc((void**)&c->h_idx, (size_t)want * sizeof(int32_t), fl) != hipSuccess ||
        hipHostMalloc((void**)&c->h_hull, (size_t)(want + 1) * sizeof(int32_t), fl) != hipSuccess ||
        hipHostGetDevicePointer((void**)&c->h_xy_dev, c->h_xy, 0) != hipSuccess ||
        hipHostGetDevicePointer((void**)&c->h_idx_dev, c->h_idx, 0) != hipSuccess ||
        hipHostGetDevicePointer((void**)&c->h_hull_dev, c->h_hull, 0) != hipSuccess) {
        (void)hipGetLastError();
        return HULL2D_ERR_OUT_OF_MEMORY;
    }
    c->h_cap = want;
    return HULL2D_OK;
}

// ensure_host, except that a no-allocation call never grows the buffers
// (they were reserved for the largest input it accepts).
hull2d_status host_buffers(hull2d_ctx* c, int64_t m, bool noalloc) {
    if (noalloc) return m <= c->h_cap ? HULL2D_OK : HULL2D_ERR_TOO_LARGE;
    return ensure_host(c, m);
}

// Batched form: device arrays over all N points of a batch (survivors,
// candidates, radix ping-pong, keep flags, hull indices) and S-sized per-set
// arrays, plus pinned staging for the offsets, the order and the results.
hull2d_status ensure_batch(hull2d_ctx* c, int64_t N, int32_t S) {
    if ((N > c->bcap_n || S > c->bcap_s || S > c->hb_cap_s) && c->bgraph) {
        // the captured work names the buffers replaced below
        (void)hipStreamSynchronize(c->stream);
        (void)hipGraphExecDestroy(c->bgraph);
        c->bgraph = nullptr;
    }
    if (N > c->bcap_n || S > c->bcap_s) {
        const int64_t wn = std::max<int64_t>(std::max<int64_t>(N, c->bcap_n), 1);
        const int64_t ws = std::max<int64_t>(std::max<int64_t>(S, c->bcap_s), 1);
        if (c->bmem) {
            (void)hipStreamSynchronize(c->stream);
            (void)hipFree(c->bmem);
            c->bmem = nullptr;
            c->bcap_n = -1;
            c->bcap_s = -1;
        }
        const size_t sizes[16] = {
            (size_t)wn * sizeof(double2), (size_t)wn * 4, (size_t)wn * 4,   // survivors
            (size_t)wn * sizeof(double2), (size_t)wn * 4, (size_t)wn * 4,   // candidates
            (size_t)wn * 4, (size_t)wn * 4, (size_t)wn * 4, (size_t)wn * 4,  // ka kb va vb
            (size_t)wn,                                                      // flags
            (size_t)wn * 4,                                                  // hull
            (size_t)(ws + 1) * 8, (size_t)ws * 4,                            // offsets, order
            (size_t)(3 * ws + 1) * 4,                                        // meta
            (size_t)wn * sizeof(uint2)};                                     // grouped candidates
        size_t off[16], o = 0;
        for (int i = 0; i < 16; ++i) {
            off[i] = o;
            o = align_up(o + sizes[i], 256);
        }
        if (hipMalloc((void**)&c->bmem, o) != hipSuccess) {
            (void)hipGetLastError();
            c->bmem = nullptr;
            return HULL2D_ERR_OUT_OF_MEMORY;
        }
        char* b = c->bmem;
        c->b_sv_xy = (double2*)(b + off[0]);
        c->b_sv_idx = (uint32_t*)(b + off[1]);
        c->b_sv_key = (uint32_t*)(b + off[2]);
        c->b_cd_xy = (double2*)(b + off[3]);
        c->b_cd_idx = (uint32_t*)(b + off[4]);
        c->b_cd_key = (uint32_t*)(b + off[5]);
        c->b_ka = (uint32_t*)(b + off[6]);
        c->b_kb = (uint32_t*)(b + off[7]);
        c->b_va = (uint32_t*)(b + off[8]);
        c->b_vb = (uint32_t*)(b + off[9]);
        c->b_gk = (uint2*)(b + off[15]);
        c->b_flag = (uint8_t*)(b + off[10]);
        c->b_hull = (int32_t*)(b + off[11]);
        c->b_offs = (int64_t*)(b + off[12]);
        c->b_order = (int32_t*)(b + off[13]);
        c->b_meta = (int32_t*)(b + off[14]);
        c->bcap_n = wn;
        c->bcap_s = (int32_t)ws;
    }
    if (S > c->hb_cap_s) {
        if (c->hb_offs) (void)hipHostFree(c->hb_offs);
        if (c->hb_order) (void)hipHostFree(c->hb_order);
        if (c->hb_meta) (void)hipHostFree(c->hb_meta);
        if (c->hb_win) (void)hipHostFree(c->hb_win);
        c->hb_offs = nullptr;
        c->hb_order = nullptr;
        c->hb_meta = nullptr;
        c->hb_win = nullptr;
        c->hb_cap_s = -1;
        const int64_t ws = std::max<int64_t>(S, 1);
        if (hipHostMalloc((void**)&c->hb_offs, (size_t)(ws + 1) * 8, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&c->hb_order, (size_t)ws * 4, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&c->hb_meta, (size_t)(3 * ws + 1) * 4, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&c->hb_win, (size_t)ws * sizeof(WSetIn), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return HULL2D_ERR_OUT_OF_MEMORY;
        }
        c->hb_cap_s = ws;
    }
    return HULL2D_OK;
}

// The tiled engine's device workspace for S sets, NT tiles and SE entries
// of the sort-bucket table.
hull2d_status ensure_wide(hull2d_ctx* c, int64_t S, int64_t NT, int64_t SE) {
    if (S <= c->wcap_s && NT <= c->wcap_nt && SE <= c->wcap_se) return HULL2D_OK;
    if (c->bgraph) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipGraphExecDestroy(c->bgraph);
        c->bgraph = nullptr;
    }
    const int64_t ws = std::max<int64_t>(std::max<int64_t>(S, c->wcap_s), 1);
    const int64_t wt = std::max<int64_t>(std::max<int64_t>(NT, c->wcap_nt), 1);
    const int64_t wse = std::max<int64_t>(std::max<int64_t>(SE, c->wcap_se), 1);
    if (c->wmem) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(c->wmem);
        c->wmem = nullptr;
        c->wcap_s = c->wcap_nt = c->wcap_se = -1;
    }
    const size_t sizes[8] = {(size_t)ws * sizeof(WSetIn), (size_t)ws * sizeof(WSet),
                             (size_t)wt * 4, (size_t)wt * 4 * sizeof(Cand), (size_t)wt * 4,
                             (size_t)wt * sizeof(WFar), (size_t)wt * 4, (size_t)wse * 4};
    size_t off[8], o = 0;
    for (int i = 0; i < 8; ++i) {
        off[i] = o;
        o = align_up(o + sizes[i], 256);
    }
    if (hipMalloc((void**)&c->wmem, o) != hipSuccess) {
        (void)hipGetLastError();
        c->wmem = nullptr;
        return HULL2D_ERR_OUT_OF_MEMORY;
    }
    char* b = c->wmem;
    c->w_in = (WSetIn*)(b + off[0]);
    c->w_set = (WSet*)(b + off[1]);
    c->w_tile_set = (int32_t*)(b + off[2]);
    c->w_tile_ext = (Cand*)(b + off[3]);
    c->w_tile_flags = (uint32_t*)(b + off[4]);
    c->w_tile_far = (WFar*)(b + off[5]);
    c->w_tile_cnt = (uint32_t*)(b + off[6]);
    c->w_bcnt = (uint32_t*)(b + off[7]);
    c->wcap_s = ws;
    c->wcap_nt = wt;
    c->wcap_se = wse;
    return HULL2D_OK;
}

hull2d_status ensure_batch_hull(hull2d_ctx* c, int64_t h) {
    if (h <= c->hb_cap_h) return HULL2D_OK;
    const int64_t want = std::max<int64_t>(h, 1 << 16);
    if (c->hb_hull) (void)hipHostFree(c->hb_hull);
    c->hb_hull = nullptr;
    c->hb_cap_h = -1;
    if (hipHostMalloc((void**)&c->hb_hull, (size_t)want * 4, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return HULL2D_ERR_OUT_OF_MEMORY;
    }
    c->hb_cap_h = want;
    return HULL2D_OK;
}

// Parameter layout (one float32 vector): W1 [256][1024], b1, W2 [256][256],
// b2, W3 [32][256], b3.
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + (int64_t)kMlpHidden * kMlpIn;
constexpr int64_t kOffW2 = kOffB1 + kMlpHidden;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kMlpHidden * kMlpHidden;
constexpr int64_t kOffW3 = kOffB2 + kMlpHidden;
constexpr int64_t kOffB3 = kOffW3 + (int64_t)kMlpOut * kMlpHidden;
static_assert(kOffB3 + kMlpOut == kMlpParams, "parameter layout");
static_assert(kMlpParams == HULL2D_MLP_PARAMS, "header constant");

hull2d_status ensure_learned(hull2d_ctx* c) {
    if (c->lmem) return HULL2D_OK;
    const size_t P = (size_t)kMlpParams;
    const size_t sizes[11] = {P * 4, P * 4, P * 4, P * 4,
                              (size_t)kMlpIn * kMlpHidden * 2, (size_t)kMlpHidden * kMlpHidden * 2,
                              (size_t)kMlpHidden * kMlpOut * 2, sizeof(LearnOut), (size_t)kMlpIn * 4,
                              16, (size_t)4 * 8 * c->cu_count};
    size_t off[11], o = 0;
    for (int i = 0; i < 11; ++i) {
        off[i] = o;
        o = align_up(o + sizes[i], 256);
    }
    if (hipMalloc((void**)&c->lmem, o) != hipSuccess) {
        (void)hipGetLastError();
        c->lmem = nullptr;
        return HULL2D_ERR_OUT_OF_MEMORY;
    }
    char* b = c->lmem;
    c->m_params = (float*)(b + off[0]);
    c->m_grad = (float*)(b + off[1]);
    c->m_am = (float*)(b + off[2]);
    c->m_av = (float*)(b + off[3]);
    c->m_w1 = (uint16_t*)(b + off[4]);
    c->m_w2 = (uint16_t*)(b + off[5]);
    c->m_w3 = (uint16_t*)(b + off[6]);
    c->learn = (LearnOut*)(b + off[7]);
    c->l_hist = (uint32_t*)(b + off[8]);
    c->l_loss = (float*)(b + off[9]);
    c->l_part = (double*)(b + off[10]);
    return HULL2D_OK;
}

MlpDev mlp_dev(const hull2d_ctx* c) {
    MlpDev W;
    W.w1 = c->m_w1;
    W.w2 = c->m_w2;
    W.w3 = c->m_w3;
    W.b1 = c->m_params + kOffB1;
    W.b2 = c->m_params + kOffB2;
    W.b3 = c->m_params + kOffB3;
    return W;
}

hipError_t refresh_inference(hull2d_ctx* c) {
    hipError_t e = launch_to_bf16(c->m_params + kOffW1, (int64_t)kMlpHidden * kMlpIn, c->m_w1, c->stream);
    if (e == hipSuccess)
        e = launch_to_bf16(c->m_params + kOffW2, (int64_t)kMlpHidden * kMlpHidden, c->m_w2, c->stream);
    if (e == hipSuccess)
        e = launch_to_bf16(c->m_params + kOffW3, (int64_t)kMlpOut * kMlpHidden, c->m_w3, c->stream);
    return e;
}

hull2d_status ensure_train(hull2d_ctx* c, int32_t B) {
    if (B <= c->tcap_b) return HULL2D_OK;
    if (c->tmem) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(c->tmem);
        c->tmem = nullptr;
        c->tcap_b = 0;
    }
    const size_t b = (size_t)B;
    const size_t sizes[6] = {b * kMlpHidden * 4, b * kMlpHidden * 4, b * kMlpOut * 4,
                             b * kMlpOut * 4, b * kMlpHidden * 4, b * kMlpHidden * 4};
    size_t off[6], o = 0;
    for (int i = 0; i < 6; ++i) {
        off[i] = o;
        o = align_up(o + sizes[i], 256);
    }
    if (hipMalloc((void**)&c->tmem, o) != hipSuccess) {
        (void)hipGetLastError();
        c->tmem = nullptr;
        return HULL2D_ERR_OUT_OF_MEMORY;
    }
    c->t_h1 = (float*)(c->tmem + off[0]);
    c->t_h2 = (float*)(c->tmem + off[1]);
    c->t_y = (float*)(c->tmem + off[2]);
    c->t_d3 = (float*)(c->tmem + off[3]);
    c->t_d2 = (float*)(c->tmem + off[4]);
    c->t_d1 = (float*)(c->tmem + off[5]);
    c->tcap_b = B;
    return HULL2D_OK;
}

#define HX_TRY(call)                      \
    do {                                  \
        if ((call) != hipSuccess) {       \
            (void)hipGetLastError();      \
            c->broken = true;             \
            return HULL2D_ERR_DEVICE;     \
        }                                 \
    } while (0)

// Step 8 (Section 3): Graham stack scan of the kept points, already in
// angular order with the pivot first.  A non-left turn pops (collinear points
// are dropped), a repeat of the top point is skipped (the first copy has the
// smallest index).  The result is rotated to start at the lexicographically
// smallest vertex.
int64_t graham_scan(double x0, double y0, int32_t i0, const double2* pts, const int32_t* idx,
                    int64_t m, std::vector<int64_t>& st, std::vector<int32_t>& out) {
    st.clear();
    auto X = [&](int64_t k) { return k < 0 ? x0 : pts[k].x; };
    auto Y = [&](int64_t k) { return k < 0 ? y0 : pts[k].y; };
    st.push_back(-1);  // the pivot
    for (int64_t k = 0; k < m; ++k) {
        const double px = pts[k].x, py = pts[k].y;
        int64_t t = st.back();
        if (X(t) == px && Y(t) == py) continue;
        while (st.size() >= 2) {
            int64_t a = st[st.size() - 2], b = st.back();
            if (orient(X(a), Y(a), X(b), Y(b), px, py) > 0) break;
            st.pop_back();
        }
        st.push_back(k);
    }
    const size_t h = st.size();
    size_t start = 0;
    for (size_t k = 1; k < h; ++k) {
        double x = X(st[k]), y = Y(st[k]);
        double bx = X(st[start]), by = Y(st[start]);
        if (x < bx || (x == bx && y < by)) start = k;
    }
    out.resize(h);
    for (size_t k = 0; k < h; ++k) {
        int64_t s = st[(start + k) % h];
        out[k] = s < 0 ? i0 : idx[s];
    }
    return (int64_t)h;
}

// Waits for the stream by polling an event: a blocking wait may put the
// thread to sleep and wake it up long after the work has finished.
hipError_t spin_sync(hull2d_ctx* c) {
    if (!c->ev_sync) return hipStreamSynchronize(c->stream);
    hipError_t e = hipEventRecord(c->ev_sync, c->stream);
    if (e != hipSuccess) return e;
    for (;;) {
        e = hipEventQuery(c->ev_sync);
        if (e != hipErrorNotReady) return e;
    }
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Argument checks and the start of a compute call (both entry points).
// Returns OK with n == 0 handled (nothing more to do), or an error.
hull2d_status begin_compute(hull2d_ctx* c, const double* d_xy, int64_t n, int32_t* h_out,
                            int64_t cap, int64_t* n_out, hull2d_stats* stats) {
    if (!c || !n_out || n < 0 || cap < 0 || (n > 0 && !d_xy) || (cap > 0 && !h_out))
        return HULL2D_ERR_INVALID_ARG;
    if (n > (int64_t)INT32_MAX) return HULL2D_ERR_INVALID_ARG;
    if (c->broken) return HULL2D_ERR_DEVICE;
    *n_out = 0;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->n = n;
    }
    c->have_last = false;
    c->last_learned = false;
    c->last_chain = false;
    if (c->opt.method != 0 && c->opt.method != 1) return HULL2D_ERR_INVALID_ARG;
    if (c->opt.scan < 0 || c->opt.scan > 2 || c->opt.workspace_limit_mib < 0) return HULL2D_ERR_INVALID_ARG;
    if (c->opt.method == 0 && c->opt.filter == 1 && !c->have_weights) return HULL2D_ERR_WEIGHTS;
    if (n == 0) return HULL2D_OK;
    if (hipSetDevice(c->device) != hipSuccess) return HULL2D_ERR_DEVICE;
    return HULL2D_OK;
}

// Steps 1-8 for one hull, on workspace w (large enough for n points).  With
// noalloc the host buffers must already be large enough for n points (the
// context was created with reserve_noalloc) and nothing is allocated.
hull2d_status compute_impl(hull2d_ctx* c, Workspace& w, bool noalloc, const double* d_xy,
                           int64_t n, int32_t* h_out, int64_t cap, int64_t* n_out,
                           hull2d_stats* stats, std::chrono::steady_clock::time_point t_start) {
    const bool learned = c->opt.filter == 1;
    hull2d_status st = HULL2D_OK;

    const bool prof = c->opt.profile && c->have_events;
    const bool prof_all = prof && c->opt.profile == 1;  // 2: Steps 1 and 2-3 only
    hipStream_t s = c->stream;
    int marks[2 * HULL2D_NUM_STAGES];
    int n_marks = 0;
    auto mark = [&](int i) {
        const bool want = prof_all || (prof && (i == HULL2D_STAGE_EXTREMES || i == HULL2D_STAGE_FILTER1));
        if (want && n_marks < 2 * HULL2D_NUM_STAGES) {
            (void)hipEventRecord(c->ev[i], s);
            marks[n_marks++] = i;
        }
    };
    hipEvent_t ev_begin = c->ev[HULL2D_NUM_STAGES];
    hipEvent_t ev_end = c->ev[HULL2D_NUM_STAGES + 1];
    if (c->have_events) HX_TRY(hipEventRecord(ev_begin, s));

    // Step 1 and Steps 2-3
    const int segs = std::min(
        filter1_blocks(n, c->cu_count, learned ? c->occ.filter1_poly : c->occ.filter1),
        learned ? std::min(kMaxSegs, kExtGridMax) : kMaxSegs);
    if (learned) {
        // The learned filter: first the proposal (sample histogram, network,
        // the sample's farthest point along each direction and the hull of
        // those points; one workgroup), then one pass over the input takes
        // Step 1's extremes and drops the points strictly inside that hull
        // (the final polygon contains it), the end of Step 1 builds the final
        // polygon, and Steps 2-3 read only the points the pass kept.  The
        // pre-filtered points sit in out_xy / out_idx (not yet in use), their
        // per-block counts in seg_off (Step 5 writes it later).
        HX_TRY(launch_front(d_xy, n, mlp_dev(c), c->learn, s));
        mark(HULL2D_STAGE_LEARNED);
        uint32_t* pre_idx = reinterpret_cast<uint32_t*>(w.out_idx);
        HX_TRY(launch_pre(d_xy, n, segs, c->learn, w.partial, w.out_xy, pre_idx, w.seg_off, s));
        HX_TRY(launch_extremes_final(w.partial, segs, w.prm, w.ds, c->learn, s));
        mark(HULL2D_STAGE_EXTREMES);
        HX_TRY(launch_filter1_pre(w.out_xy, pre_idx, w.seg_off, n, segs, w.prm, &c->learn->poly, w.comp_xy,
                                  w.comp_idx, w.keys_a, w.seg_count, w.blk_d2, w.blk_best, w.ds, s));
        mark(HULL2D_STAGE_FILTER1);
    } else {
        const int grid_ext = extremes_grid(n, c->cu_count, c->occ.extremes);
        HX_TRY(launch_extremes(d_xy, n, w.partial, grid_ext, w.prm, w.ds, nullptr, s));
        mark(HULL2D_STAGE_EXTREMES);
        HX_TRY(launch_filter1(d_xy, n, segs, w.prm, nullptr, w.comp_xy, w.comp_idx, w.keys_a,
                              w.seg_count, w.blk_d2, w.blk_best, w.ds, s));
        mark(HULL2D_STAGE_FILTER1);
    }
    // Step 5 (needs every survivor's distance; the sort does not)
    const bool full = c->opt.round2_chunk != 0 || c->opt.full_sort != 0;
    HX_TRY(launch_longest(segs, w.blk_d2, w.blk_best, w.seg_count, w.seg_off, w.comp_xy, w.keys_a,
                          w.prm, w.ds, full ? nullptr : w.bmax, s));
    mark(HULL2D_STAGE_LONGEST);
    // The sorting problem: every round-1 survivor (Step 4 as printed, and the
    // paper's subsets), or only the candidates of the bucketed filter.
    DevStatus* pds = w.ds;
    const double2* pxy = w.comp_xy;
    const uint32_t* pidx = w.comp_idx;
    const uint32_t* pkeys = w.cand_key;   // dense keys of the full problem
    const uint32_t* pvals = w.cand_idx;   // and their slots in the segments
    if (!full) {
        DevStatus* ds2 = w.ds + 1;
        HX_TRY(launch_bucket_max(n, segs, w.seg_count, w.comp_xy, w.keys_a, w.prm, w.bmax,
                                 std::max(1, c->cu_count), s));
        HX_TRY(launch_bucket_scan(w.bmax, w.prefix, ds2, s));
        HX_TRY(launch_prefilter(n, segs, w.seg_count, w.comp_xy, w.comp_idx, w.keys_a, w.prm,
                                w.ds, w.prefix, w.cand_xy, w.cand_idx, w.cand_key, w.cand_kap,
                                w.bmax, ds2, s));
        pds = ds2;
        pxy = w.cand_xy;
        pidx = w.cand_idx;
        pkeys = w.cand_key;
        pvals = nullptr;
    } else {
        HX_TRY(launch_densify(n, segs, w.seg_count, w.seg_off, w.keys_a, w.cand_key, w.cand_idx, s));
    }
    mark(HULL2D_STAGE_BUCKETS);

    // Step 4 and Steps 6-7 with the stable removal, by the multi-kernel path
    // (any size), followed by the status read-back.
    auto sort_path = [&]() -> hull2d_status {
        HX_TRY(launch_histogram(pkeys, pds, w.hist,
                                (int)std::min<int64_t>(kHistGridMax, std::max<int64_t>(1, ceil_div(n, 4096))), s));
        mark(HULL2D_STAGE_HISTOGRAM);
        const uint32_t* kin = pkeys;
        const uint32_t* vin = pvals;
        uint32_t* kout = w.keys_b;
        uint32_t* vout = w.vals_b;
        for (int pass = 0; pass < 4; ++pass) {
            const uint32_t e = next_epoch(c, w);
            HX_TRY(launch_sort_pass(n, pass, kin, vin, kout, vout, w.hist, pds, w.stat, c->ctr, e,
                                    c->cu_count, s));
            mark(HULL2D_STAGE_SORT0 + pass);
            kin = kout;
            vin = vout;
            kout = (kout == w.keys_b) ? w.keys_a : w.keys_b;
            vout = (vout == w.vals_b) ? w.vals_a : w.vals_b;
        }
        // after four passes the result is in keys_a / vals_a
        HX_TRY(launch_ties(n, w.keys_a, w.vals_a, pxy, pidx, w.prm, pds, w.long_list, s));
        mark(HULL2D_STAGE_TIES);
        HX_TRY(launch_ties_long(w.keys_a, w.vals_a, pxy, pidx, w.prm, pds, w.long_list,
                                w.huge_list, c->cu_count, s));
        mark(HULL2D_STAGE_TIES_LONG);
        return HULL2D_OK;
    };
    uint32_t* slots = w.vals_a;
    auto round2 = [&]() -> hull2d_status {
        if (c->opt.round2_chunk == 0) {
            const uint32_t e = next_epoch(c, w);
            HX_TRY(launch_round2_scan(n, slots, pxy, w.prm, pds, w.keep, w.stat, c->ctr, e,
                                      c->cu_count, s));
        } else {
            HX_TRY(launch_round2_chunks(n, c->opt.round2_chunk, slots, pxy, w.prm, pds, w.keep, s));
        }
        mark(HULL2D_STAGE_ROUND2);
        const uint32_t e = next_epoch(c, w);
        HX_TRY(launch_compact(n, w.keep, slots, pxy, pidx, w.out_xy, w.out_idx, pds, w.stat,
                              c->ctr, e, c->cu_count, s));
        mark(HULL2D_STAGE_COMPACT);
        return HULL2D_OK;
    };
    auto read_status = [&]() -> hull2d_status {
        HX_TRY(hipMemcpyAsync(c->h_ds, w.ds, 2 * sizeof(DevStatus), hipMemcpyDeviceToHost, s));
        HX_TRY(spin_sync(c));
        return HULL2D_OK;
    };
    bool tail_done = false;
    bool scanned = false;  // Step 8 ran on the device: the hull is in c->h_hull
    uint32_t* scan_ticket = &c->ctr->ticket[kTicketScan * 16];
    // Step 8 on the device for the tail's kept points only when asked: at
    // the tail's sizes (at most 2 kTailCap + 1 kept points) the host scan
    // of the kept points is faster
    const bool scan_tail = c->opt.scan == 1;
    if (!full) {
        // small candidate sets: one workgroup per region does Steps 4 and
        // 6-7; the kept points (or, with the device scan, the hull) and both
        // statuses go straight to host memory (at most kTailCap kept points
        // per region and P_l)
        st = host_buffers(c, 2 * (int64_t)kTailCap + 1, noalloc);
        if (st != HULL2D_OK) return st;
        c->h_ds[1].tail_state = kTailUnset;  // the kernels overwrite these
        c->h_ds[1].scan_state = kScanUnset;
        if (scan_tail) {
            HX_TRY(launch_tail(w.cand_xy, w.cand_idx, w.cand_key, w.cand_kap, w.bmax, w.prm,
                               w.ds, w.tail_slot, w.tail_count, nullptr, nullptr, nullptr, s));
            mark(HULL2D_STAGE_TAIL);
            HX_TRY(launch_scan_tail(w.cand_xy, w.cand_idx, w.tail_slot, w.tail_count, w.ds, w.out_xy,
                                    w.keys_b, w.part_len, scan_ticket, c->h_hull_dev, c->h_ds_dev, s));
            mark(HULL2D_STAGE_SCAN);
        } else {
            HX_TRY(launch_tail(w.cand_xy, w.cand_idx, w.cand_key, w.cand_kap, w.bmax, w.prm,
                               w.ds, w.tail_slot, w.tail_count, c->h_xy_dev, c->h_idx_dev,
                               c->h_ds_dev, s));
            mark(HULL2D_STAGE_TAIL);
        }
        // one wait ends the call unless the candidates did not fit
        if (c->have_events) HX_TRY(hipEventRecord(ev_end, s));
        HX_TRY(spin_sync(c));
        if (c->h_ds[1].tail_state == kTailUnset) {
            // not written: read the statuses the usual way
            st = read_status();
            if (st != HULL2D_OK) return st;
        }
        tail_done = c->h_ds[1].tail_state == kTailDone;
        scanned = scan_tail && tail_done && c->h_ds[1].scan_state == kScanDone;
        // the scan did nothing: its event is recorded again if the list
        // form runs later (one event per stage)
        if (!tail_done && n_marks > 0 && marks[n_marks - 1] == HULL2D_STAGE_SCAN) --n_marks;
        if (scan_tail && tail_done && !scanned) {
            // the parts' chains were too many for one workgroup: the kept
            // points go to host memory for the host scan
            HX_TRY(launch_tail_out(w.cand_xy, w.cand_idx, w.ds, w.tail_slot, w.tail_count, c->h_xy_dev,
                                   c->h_idx_dev, c->h_ds_dev, s));
            mark(HULL2D_STAGE_D2H);
            if (c->have_events) HX_TRY(hipEventRecord(ev_end, s));
            HX_TRY(spin_sync(c));
        }
    }
    if (!tail_done) {
        st = sort_path();
        if (st != HULL2D_OK) return st;
        st = round2();
        if (st != HULL2D_OK) return st;
        st = read_status();
        if (st != HULL2D_OK) return st;
    }
    DevStatus D = c->h_ds[0];
    DevStatus DP = full ? c->h_ds[0] : c->h_ds[1];
    if (D.flags & kFlagNonfinite) return HULL2D_ERR_NONFINITE;
    if (D.flags & kFlagRange) return HULL2D_ERR_RANGE;
    if (!tail_done && DP.huge_runs > 0) {
        // Runs of equal keys longer than one workgroup sorts: merge them, then
        // run the second round again on the corrected order.
        std::vector<uint32_t>& hl = c->huge_host;
        if (noalloc && 2 * (size_t)DP.huge_runs > hl.capacity()) return HULL2D_ERR_TOO_LARGE;
        hl.resize(2 * (size_t)DP.huge_runs);
        HX_TRY(hipMemcpyAsync(hl.data(), w.huge_list, hl.size() * sizeof(uint32_t),
                              hipMemcpyDeviceToHost, s));
        HX_TRY(spin_sync(c));
        for (uint32_t r = 0; r < DP.huge_runs; ++r)
            HX_TRY(launch_huge_run(slots, w.vals_b, hl[2 * r], hl[2 * r + 1], pxy, pidx, w.prm, pds, s));
        st = round2();
        if (st != HULL2D_OK) return st;
        st = read_status();
        if (st != HULL2D_OK) return st;
        D = c->h_ds[0];
        DP = full ? c->h_ds[0] : c->h_ds[1];
    }
    const DevStatus DS = DP;
    const int64_t m = (int64_t)DS.n_kept;
    st = host_buffers(c, m + 1, noalloc);
    if (st != HULL2D_OK) return st;
    const bool scan_list = c->opt.scan == 1 || (c->opt.scan == 0 && m >= kScanAutoMin);
    if (!tail_done && scan_list && m <= (int64_t)kScanMaxParts * kScanPart) {
        // Step 8 on the device over the compacted kept points; the parts'
        // chains go to arrays that are dead by now
        double2* part_xy = pxy == w.cand_xy ? w.comp_xy : w.cand_xy;
        c->h_ds[1].scan_state = kScanUnset;
        HX_TRY(launch_scan_list(w.out_xy, w.out_idx, m, D.x0, D.y0, D.p0_idx, w.ds, part_xy, w.keys_b,
                                w.part_len, scan_ticket, c->h_hull_dev, c->h_ds_dev, s));
        mark(HULL2D_STAGE_SCAN);
        if (c->have_events) HX_TRY(hipEventRecord(ev_end, s));
        HX_TRY(spin_sync(c));
        scanned = c->h_ds[1].scan_state == kScanDone;
    }
    auto t_d2h = std::chrono::steady_clock::now();
    if (!tail_done && !scanned) {
        if (m > 0) {
            HX_TRY(hipMemcpyAsync(c->h_xy, w.out_xy, (size_t)m * sizeof(double2),
                                  hipMemcpyDeviceToHost, s));
            HX_TRY(hipMemcpyAsync(c->h_idx, w.out_idx, (size_t)m * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, s));
        }
        mark(HULL2D_STAGE_D2H);
        if (c->have_events) HX_TRY(hipEventRecord(ev_end, s));
        HX_TRY(spin_sync(c));
    }
    const double ms_d2h_wall = tail_done || scanned ? 0.0 : ms_since(t_d2h);

    // Step 8 on the host when the device scan did not finish the hull
    auto t_scan = std::chrono::steady_clock::now();
    int64_t h = 0;
    const int32_t* hull_out = c->h_hull;
    if (scanned) {
        h = (int64_t)c->h_ds[1].n_hull;
    } else {
        std::vector<int64_t>& stk = c->stk;
        std::vector<int32_t>& hull = c->hull;
        stk.reserve((size_t)m + 1);
        h = graham_scan(D.x0, D.y0, D.p0_idx, c->h_xy, c->h_idx, m, stk, hull);
        hull_out = hull.data();
    }
    const double ms_scan = scanned ? 0.0 : ms_since(t_scan);

    c->have_last = true;
    c->last_learned = learned;
    c->last_full = full;
    c->last_n = n;
    c->last_segs = segs;
    c->last_ws = w;
    c->last_tail = tail_done;
    c->last_ds = D;
    c->last_ds2 = DS;

    *n_out = h;
    if (stats) {
        stats->n_round1 = (int64_t)D.n_sorted + (int64_t)D.n_p0;
        stats->n_sorted = D.n_sorted;
        stats->n_round2 = m + 1;
        stats->n_hull = h;
        stats->n_candidates = DS.n_sorted;
        if (c->have_events) {
            float f = 0.f;
            if (hipEventElapsedTime(&f, ev_begin, ev_end) == hipSuccess)
                stats->ms_device = f;
        }
        if (prof) {
            // each recorded stage ends at its event and starts at the previous
            // recorded one; Step 1's two kernels are reported under EXTREMES
            hipEvent_t prev = ev_begin;
            for (int k = 0; k < n_marks; ++k) {
                float f = 0.f;
                if (hipEventElapsedTime(&f, prev, c->ev[marks[k]]) == hipSuccess && f > 0.f)
                    stats->ms_stage[marks[k]] += f;
                prev = c->ev[marks[k]];
            }
        }
        stats->ms_stage[HULL2D_STAGE_HOST_SCAN] = ms_scan;
        if (!prof) stats->ms_stage[HULL2D_STAGE_D2H] = ms_d2h_wall;
    }
    if (h > cap) {
        if (stats) stats->ms_total = ms_since(t_start);
        return HULL2D_ERR_CAPACITY;
    }
    std::memcpy(h_out, hull_out, (size_t)h * sizeof(int32_t));
    if (stats) stats->ms_total = ms_since(t_start);
    return HULL2D_OK;
}

// The four-region variant (options.method = 1; Section 5.1, Table 8): Steps
// 1-2 as gScan, then the regions, their candidates, the exact sort and the
// walk per region on the device (launch_chain), and the variant's second
// stage on the host: per region one stack scan from corner k over the kept
// points to corner k+1 (a non-left turn pops, a repeat of the top is
// skipped), the chains joined without their last points, the result rotated
// to the lexicographically smallest vertex.
hull2d_status compute_chain(hull2d_ctx* c, Workspace& w, bool noalloc, const double* d_xy, int64_t n,
                            int32_t* h_out, int64_t cap, int64_t* n_out, hull2d_stats* stats,
                            std::chrono::steady_clock::time_point t_start) {
    hipStream_t s = c->stream;
    hull2d_status st = host_buffers(c, 4 * (int64_t)kChainHostCap, noalloc);
    if (st != HULL2D_OK) return st;
    hipEvent_t ev_begin = c->ev[HULL2D_NUM_STAGES];
    hipEvent_t ev_end = c->ev[HULL2D_NUM_STAGES + 1];
    if (c->have_events) HX_TRY(hipEventRecord(ev_begin, s));
    const int grid_ext = extremes_grid(n, c->cu_count, c->occ.extremes);
    HX_TRY(launch_extremes(d_xy, n, w.partial, grid_ext, w.prm, w.ds, nullptr, s));
    HX_TRY(launch_chain(d_xy, n, w.prm, w.ds, w.chain, w.cand_xy, w.cand_idx, w.cand_key, w.comp_xy,
                        w.comp_idx, w.out_xy, w.out_idx, c->h_chain_dev, c->h_xy_dev, c->h_idx_dev,
                        c->cu_count * 8, s));
    if (c->have_events) HX_TRY(hipEventRecord(ev_end, s));
    HX_TRY(spin_sync(c));
    const ChainHost H = *c->h_chain;
    if (H.ds0.flags & kFlagNonfinite) return HULL2D_ERR_NONFINITE;
    if (H.ds0.flags & kFlagRange) return HULL2D_ERR_RANGE;
    for (int r = 0; r < 4; ++r)
        if (H.overflow[r]) return HULL2D_ERR_UNIMPLEMENTED;

    // the kept lists: in the host buffers, or copied from the device
    const double2* kxy[4];
    const int32_t* kix[4];
    size_t off_host = 0;
    for (int r = 0; r < 4; ++r)
        if (!H.on_host[r]) off_host += H.n_kept[r];
    if (off_host > 0) {
        if (noalloc && off_host > c->chain_xy.capacity()) return HULL2D_ERR_TOO_LARGE;
        c->chain_xy.resize(off_host);
        c->chain_ix.resize(off_host);
    }
    size_t at = 0;
    for (int r = 0; r < 4; ++r) {
        if (H.on_host[r]) {
            kxy[r] = c->h_xy + (size_t)r * kChainHostCap;
            kix[r] = c->h_idx + (size_t)r * kChainHostCap;
            continue;
        }
        kxy[r] = c->chain_xy.data() + at;
        kix[r] = c->chain_ix.data() + at;
        if (H.n_kept[r] > 0) {
            HX_TRY(hipMemcpyAsync(c->chain_xy.data() + at, w.out_xy + H.kept_at[r],
                                  (size_t)H.n_kept[r] * sizeof(double2), hipMemcpyDeviceToHost, s));
            HX_TRY(hipMemcpyAsync(c->chain_ix.data() + at, w.out_idx + H.kept_at[r],
                                  (size_t)H.n_kept[r] * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        }
        at += H.n_kept[r];
    }
    if (off_host > 0) HX_TRY(spin_sync(c));

    auto t_scan = std::chrono::steady_clock::now();
    std::vector<HostPt>& stk = c->cstk;
    stk.clear();
    size_t need = 8;
    for (int r = 0; r < 4; ++r) need += H.n_kept[r];
    if (noalloc && need > stk.capacity()) return HULL2D_ERR_TOO_LARGE;
    stk.reserve(need);
    for (int k = 0; k < 4; ++k) {
        const size_t beg = stk.size();
        auto push = [&](double x, double y, int32_t i) {
            if (stk.size() > beg && stk.back().x == x && stk.back().y == y) return;
            while (stk.size() - beg >= 2) {
                const HostPt& a = stk[stk.size() - 2];
                const HostPt& b = stk.back();
                if (orient(a.x, a.y, b.x, b.y, x, y) > 0) break;
                stk.pop_back();
            }
            stk.push_back(HostPt{x, y, i});
        };
        push(H.cx[k], H.cy[k], H.ci[k]);
        for (uint32_t j = 0; j < H.n_kept[k]; ++j) push(kxy[k][j].x, kxy[k][j].y, kix[k][j]);
        push(H.cx[(k + 1) & 3], H.cy[(k + 1) & 3], H.ci[(k + 1) & 3]);
        stk.pop_back();  // corner k+1 starts the next chain
    }
    if (stk.empty()) stk.push_back(HostPt{H.cx[0], H.cy[0], H.ci[0]});
    const int64_t h = (int64_t)stk.size();
    size_t start = 0;
    for (size_t k = 1; k < stk.size(); ++k)
        if (stk[k].x < stk[start].x || (stk[k].x == stk[start].x && stk[k].y < stk[start].y)) start = k;
    const double ms_scan = ms_since(t_scan);

    int distinct = 0;
    for (int k = 0; k < 4; ++k) {
        bool dup = false;
        for (int j = 0; j < k; ++j) dup |= (H.cx[j] == H.cx[k] && H.cy[j] == H.cy[k]);
        distinct += dup ? 0 : 1;
    }
    c->have_last = true;
    c->last_learned = false;
    c->last_chain = true;
    c->last_chain_host = H;
    c->last_n = n;
    c->last_ws = w;
    c->last_ds = H.ds0;
    *n_out = h;
    if (stats) {
        int64_t kept = 0, cand = 0, inreg = 0;
        for (int r = 0; r < 4; ++r) {
            kept += H.n_kept[r];
            cand += H.n_cand[r];
            inreg += H.n_region[r];
        }
        stats->n_round1 = H.m1;
        stats->n_sorted = inreg;
        stats->n_candidates = cand;
        stats->n_round2 = kept + distinct;
        stats->n_hull = h;
        if (c->have_events) {
            float f = 0.f;
            if (hipEventElapsedTime(&f, ev_begin, ev_end) == hipSuccess) stats->ms_device = f;
        }
        stats->ms_stage[HULL2D_STAGE_HOST_SCAN] = ms_scan;
    }
    if (h > cap) {
        if (stats) stats->ms_total = ms_since(t_start);
        return HULL2D_ERR_CAPACITY;
    }
    for (int64_t k = 0; k < h; ++k) h_out[k] = stk[(start + (size_t)k) % (size_t)h].i;
    if (stats) stats->ms_total = ms_since(t_start);
    return HULL2D_OK;
}

}  // namespace

extern "C" {

const char* hull2d_status_string(hull2d_status s) {
    switch (s) {
        case HULL2D_OK: return "ok";
        case HULL2D_ERR_INVALID_ARG: return "invalid argument";
        case HULL2D_ERR_NONFINITE: return "non-finite coordinate";
        case HULL2D_ERR_RANGE: return "coordinate magnitude outside [2^-300, 2^300]";
        case HULL2D_ERR_CAPACITY: return "output capacity too small";
        case HULL2D_ERR_OUT_OF_MEMORY: return "out of memory";
        case HULL2D_ERR_DEVICE: return "device error";
        case HULL2D_ERR_WEIGHTS: return "learned-filter weights missing or corrupt";
        case HULL2D_ERR_UNIMPLEMENTED: return "not implemented";
        case HULL2D_ERR_TOO_LARGE: return "input larger than HULL2D_NOALLOC_MAX_POINTS";
    }
    return "unknown status";
}

hull2d_status hull2d_create(hull2d_ctx** out, int device, void* hip_stream,
                            const hull2d_options* opt) {
    if (!out) return HULL2D_ERR_INVALID_ARG;
    *out = nullptr;
    if (opt && opt->struct_size < sizeof(uint32_t) + sizeof(int32_t)) return HULL2D_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return ndev > 0 ? HULL2D_ERR_INVALID_ARG : HULL2D_ERR_DEVICE;
    }
    hull2d_ctx* c = new (std::nothrow) hull2d_ctx();
    if (!c) return HULL2D_ERR_OUT_OF_MEMORY;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->opt.struct_size = sizeof(hull2d_options);
    c->opt.round2_chunk = 0;
    if (opt) {
        size_t n = std::min<size_t>(opt->struct_size, sizeof(hull2d_options));
        std::memcpy(&c->opt, opt, n);
        c->opt.struct_size = sizeof(hull2d_options);
    }
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return HULL2D_ERR_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->cu_count = prop.multiProcessorCount;
    c->occ = query_occupancy();
    if (hipMalloc((void**)&c->ctr, sizeof(Counters)) != hipSuccess ||
        hipMemset(c->ctr, 0, sizeof(Counters)) != hipSuccess ||
        hipHostMalloc((void**)&c->h_ds, 2 * sizeof(DevStatus),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void**)&c->h_ds_dev, c->h_ds, 0) != hipSuccess ||
        hipHostMalloc((void**)&c->h_chain, sizeof(ChainHost),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void**)&c->h_chain_dev, c->h_chain, 0) != hipSuccess) {
        (void)hipGetLastError();
        hull2d_destroy(c);
        return HULL2D_ERR_OUT_OF_MEMORY;
    }
    // the no-allocation entry point: the fixed device workspace of this
    // device, and (on request) host buffers for its largest input
    const bool have_scratch = init_scratch(device);
    if (c->opt.reserve_noalloc) {
        if (!have_scratch) {
            hull2d_destroy(c);
            return HULL2D_ERR_DEVICE;
        }
        if (ensure_host(c, kNoAllocMax + 1) != HULL2D_OK) {
            hull2d_destroy(c);
            return HULL2D_ERR_OUT_OF_MEMORY;
        }
        try {
            c->stk.reserve((size_t)kNoAllocMax + 1);
            c->hull.reserve((size_t)kNoAllocMax + 1);
            c->huge_host.reserve(2 * ((size_t)kNoAllocMax / kRunCap + 2));
            c->chain_xy.reserve((size_t)kNoAllocMax);
            c->chain_ix.reserve((size_t)kNoAllocMax);
            c->cstk.reserve((size_t)kNoAllocMax + 8);
        } catch (...) {
            hull2d_destroy(c);
            return HULL2D_ERR_OUT_OF_MEMORY;
        }
        c->noalloc_ready = true;
    }
    // Stage events only time the stream (the host waits on ev_sync): without
    // the system-scope fence a record does not write back and invalidate the
    // caches, which otherwise idles the device for several microseconds.
    bool ev_ok = true;
    for (int i = 0; i < HULL2D_NUM_STAGES + 2; ++i)
        ev_ok = ev_ok && hipEventCreateWithFlags(&c->ev[i], hipEventDisableSystemFence) == hipSuccess;
    c->have_events = ev_ok;
    if (hipEventCreateWithFlags(&c->ev_sync, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        c->ev_sync = nullptr;
    }
    *out = c;
    return HULL2D_OK;
}

void hull2d_destroy(hull2d_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream || c->dmem) (void)hipStreamSynchronize(c->stream);
    if (c->dmem) (void)hipFree(c->dmem);
    if (c->ctr) (void)hipFree(c->ctr);
    if (c->bgraph) (void)hipGraphExecDestroy(c->bgraph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->side_stream) (void)hipStreamDestroy(c->side_stream);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->h_ds) (void)hipHostFree(c->h_ds);
    if (c->h_chain) (void)hipHostFree(c->h_chain);
    if (c->h_xy) (void)hipHostFree(c->h_xy);
    if (c->h_idx) (void)hipHostFree(c->h_idx);
    if (c->h_hull) (void)hipHostFree(c->h_hull);
    if (c->bmem) (void)hipFree(c->bmem);
    if (c->lmem) (void)hipFree(c->lmem);
    if (c->tmem) (void)hipFree(c->tmem);
    if (c->hb_offs) (void)hipHostFree(c->hb_offs);
    if (c->hb_order) (void)hipHostFree(c->hb_order);
    if (c->hb_meta) (void)hipHostFree(c->hb_meta);
    if (c->hb_hull) (void)hipHostFree(c->hb_hull);
    if (c->hb_win) (void)hipHostFree(c->hb_win);
    if (c->wmem) (void)hipFree(c->wmem);
    for (int i = 0; i < HULL2D_NUM_STAGES + 2; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    if (c->ev_sync) (void)hipEventDestroy(c->ev_sync);
    delete c;
}

hull2d_status hull2d_compute(hull2d_ctx* c, const double* d_xy, int64_t n, int32_t* h_out,
                             int64_t cap, int64_t* n_out, hull2d_stats* stats) {
    auto t_start = std::chrono::steady_clock::now();
    hull2d_status st = begin_compute(c, d_xy, n, h_out, cap, n_out, stats);
    if (st != HULL2D_OK || n == 0) return st;
    st = ensure_workspace(c, n);
    if (st != HULL2D_OK) return st;
    if (c->opt.method == 1) return compute_chain(c, c->own, false, d_xy, n, h_out, cap, n_out, stats, t_start);
    return compute_impl(c, c->own, false, d_xy, n, h_out, cap, n_out, stats, t_start);
}

hull2d_status hull2d_compute_noalloc(hull2d_ctx* c, const double* d_xy, int64_t n, int32_t* h_out,
                                     int64_t cap, int64_t* n_out, hull2d_stats* stats) {
    auto t_start = std::chrono::steady_clock::now();
    if (c && n > kNoAllocMax) return HULL2D_ERR_TOO_LARGE;
    if (c && !c->noalloc_ready) return HULL2D_ERR_INVALID_ARG;
    hull2d_status st = begin_compute(c, d_xy, n, h_out, cap, n_out, stats);
    if (st != HULL2D_OK || n == 0) return st;
    void* base = scratch_address(c->device);
    if (!base) return HULL2D_ERR_DEVICE;
    Workspace w;
    carve((char*)base, kNoAllocMax, w);
    w.epoch = &g_scratch_epoch[c->device];
    if (c->opt.method == 1) return compute_chain(c, w, true, d_xy, n, h_out, cap, n_out, stats, t_start);
    return compute_impl(c, w, true, d_xy, n, h_out, cap, n_out, stats, t_start);
}

hull2d_status hull2d_batch(hull2d_ctx* c, const double* d_xy, const int64_t* h_offsets, int32_t S,
                           int32_t* h_out, int64_t cap, int64_t* h_out_offsets,
                           hull2d_stats* stats) {
    auto t_start = std::chrono::steady_clock::now();
    if (!c || S < 0 || !h_offsets || !h_out_offsets || cap < 0 || (cap > 0 && !h_out))
        return HULL2D_ERR_INVALID_ARG;
    if (h_offsets[0] != 0) return HULL2D_ERR_INVALID_ARG;
    for (int32_t s = 0; s < S; ++s)
        if (h_offsets[s + 1] < h_offsets[s] || h_offsets[s + 1] - h_offsets[s] > (int64_t)INT32_MAX)
            return HULL2D_ERR_INVALID_ARG;
    if (h_offsets[S] > 0 && !d_xy) return HULL2D_ERR_INVALID_ARG;
    if (c->opt.batch_engine < 0 || c->opt.batch_engine > 1) return HULL2D_ERR_INVALID_ARG;
    {
        // the tiled engine's schedule (0: default)
        const int32_t t = c->opt.batch_tile;
        if (t != 0 && (t < (int32_t)kWideTileMin || t > (int32_t)kWideTileMax || (t & (t - 1)) != 0))
            return HULL2D_ERR_INVALID_ARG;
        const int32_t fb = c->opt.batch_filter_bits, sb = c->opt.batch_sort_bits, ss = c->opt.batch_side_sets;
        if (fb != 0 && (fb < 4 || fb > kWideFilterBits)) return HULL2D_ERR_INVALID_ARG;
        if (sb != 0 && (sb < 4 || sb > kWideSortBits)) return HULL2D_ERR_INVALID_ARG;
        if (ss < -1 || ss > 4096) return HULL2D_ERR_INVALID_ARG;
        const int32_t it = c->opt.batch_items;
        if (it != 0 && it != 2 && it != 4 && it != 8) return HULL2D_ERR_INVALID_ARG;
    }
    if (c->broken) return HULL2D_ERR_DEVICE;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->n = h_offsets[S];
    }
    h_out_offsets[0] = 0;
    if (S == 0) return HULL2D_OK;
    if (hipSetDevice(c->device) != hipSuccess) return HULL2D_ERR_DEVICE;
    const int64_t N = h_offsets[S];
    hull2d_status st = ensure_batch(c, N, S);
    if (st != HULL2D_OK) return st;
    {
        const int fit = std::max(1, batch_blocks_per_cu());
        const int want = c->opt.batch_blocks_per_cu > 0 ? std::min(c->opt.batch_blocks_per_cu, fit) : fit;
        c->batch_grid = c->cu_count * want;
    }
    hipStream_t s = c->stream;

    // the order in which workgroups take the sets
    std::memcpy(c->hb_offs, h_offsets, (size_t)(S + 1) * sizeof(int64_t));
    auto size_of = [&](int32_t i) { return h_offsets[i + 1] - h_offsets[i]; };
    if (c->opt.batch_order == 2) {
        for (int32_t i = 0; i < S; ++i) c->hb_order[i] = i;
    } else if (c->opt.batch_order == 1) {
        for (int32_t i = 0; i < S; ++i) c->hb_order[i] = i;
        std::stable_sort(c->hb_order, c->hb_order + S,
                         [&](int32_t a, int32_t b) { return size_of(a) > size_of(b); });
    } else {
        // largest size class (power of two) first: counting sort, stable
        int32_t cnt[64] = {0};
        auto cls = [&](int32_t i) {
            const int64_t n = size_of(i);
            return 63 - (n > 0 ? __builtin_clzll((unsigned long long)n) : 63);
        };
        for (int32_t i = 0; i < S; ++i) ++cnt[cls(i)];
        int32_t pos[64];
        int32_t acc = 0;
        for (int k = 63; k >= 0; --k) {
            pos[k] = acc;
            acc += cnt[k];
        }
        for (int32_t i = 0; i < S; ++i) c->hb_order[pos[cls(i)]++] = i;
    }
    // the tiled engine's layout: each set's tiles and bucket counts (2^bf
    // buckets per region for the bucket maxima, about a quarter of the set's
    // size, 16 to 16,384; 2^bs sort buckets, at most 4,096)
    const int engine = c->opt.batch_engine;
    int64_t NT = 0, SE = 0, NT_big = 0;
    int32_t S_big = 0;  // the largest sets, run beside the others on a second stream
    int32_t L_big = 0, L_rest = 0;  // sets with the large Steps 6-7 table leading each launch
    if (engine == 0) {
        // the tiled engine takes its sets by exact size, largest first,
        // whatever the persistent engine's order option says: the sets that
        // need the large Steps 6-7 table are then a prefix of each launch
        for (int32_t i = 0; i < S; ++i) c->hb_order[i] = i;
        std::stable_sort(c->hb_order, c->hb_order + S,
                         [&](int32_t a, int32_t b) { return size_of(a) > size_of(b); });
        const uint32_t tile = c->opt.batch_tile > 0 ? (uint32_t)c->opt.batch_tile : kWideTile;
        const uint32_t fbits =
            c->opt.batch_filter_bits > 0 ? (uint32_t)c->opt.batch_filter_bits : (uint32_t)kWideFilterBits;
        const uint32_t sbits = c->opt.batch_sort_bits > 0 ? (uint32_t)c->opt.batch_sort_bits : (uint32_t)kWideSortBits;
        const int32_t side = c->opt.batch_side_sets == 0 ? kWideBigSets : std::max(0, c->opt.batch_side_sets);
        while (S_big < std::min<int32_t>(S - 1, side) && size_of(c->hb_order[S_big]) >= kWideBigMin) ++S_big;
        for (int32_t r = 0; r < S; ++r) {
            // tiles numbered in this order: the big sets' tiles come first
            const int32_t i = c->hb_order[r];
            const int64_t n = size_of(i);
            WSetIn& w = c->hb_win[i];
            uint32_t bf = 0;
            if (n > 0) {
                bf = 4;
                while (bf < fbits && ((int64_t)1 << bf) < (n + 3) / 4) ++bf;
                bf = std::min(bf, fbits);
            }
            w.o = h_offsets[i];
            w.n = (uint32_t)n;
            w.t0 = (uint32_t)NT;
            w.nt = (uint32_t)((n + tile - 1) / tile);
            w.bf = bf;
            w.bs = std::min(bf, sbits);
            w.soff = (uint32_t)SE;
            w.tile = tile;
            NT += w.nt;
            if (r < S_big) NT_big = NT;
            SE += n > 0 ? ((int64_t)2 << w.bs) : 0;
            if (NT > (int64_t)UINT32_MAX || SE > (int64_t)UINT32_MAX) return HULL2D_ERR_OUT_OF_MEMORY;
        }
        if (S_big > 0 && !c->side_stream) {
            if (hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                return HULL2D_ERR_DEVICE;
            }
        }
        st = ensure_wide(c, S, NT, SE);
        if (st != HULL2D_OK) return st;
        // the leading sets of each launch (the side stream's, or the only
        // one, then the others) that need the large Steps 6-7 table
        auto n_large = [&](int32_t first, int32_t count) {
            int32_t k = 0;
            while (k < count && c->hb_win[c->hb_order[first + k]].bf > (uint32_t)kWideSmallBits) ++k;
            return k;
        };
        L_big = S_big > 0 ? n_large(0, S_big) : n_large(0, S);
        L_rest = S_big > 0 ? n_large(S_big, S - S_big) : 0;
    }
    int32_t* d_count = c->b_meta + 1;
    int32_t* d_start = d_count + S;
    uint32_t* d_flags = (uint32_t*)(d_start + S);
    // the device work of one call: uploads of the offsets and the order, the
    // counter reset, the persistent launch, the download of the per-set
    // counts, starts and flags
    auto device_work = [&](hipStream_t q) -> hipError_t {
        if (engine == 0) {
            hipError_t e = hipMemcpyAsync(c->w_in, c->hb_win, (size_t)S * sizeof(WSetIn), hipMemcpyHostToDevice, q);
            if (e == hipSuccess)
                e = hipMemcpyAsync(c->b_order, c->hb_order, (size_t)S * 4, hipMemcpyHostToDevice, q);
            if (e == hipSuccess) e = launch_batch_clear((uint32_t*)c->b_meta, q);
            if (e == hipSuccess) {
                WideArgs a;
                a.xy = reinterpret_cast<const double2*>(d_xy);
                a.in = c->w_in;
                a.ws = c->w_set;
                a.order = c->b_order;
                a.S = S;
                a.S_large = 0;
                a.items = c->opt.batch_items > 0 ? c->opt.batch_items : 4;
                a.t_base = 0;
                a.NT = (uint32_t)NT;
                a.tile_set = c->w_tile_set;
                a.tile_ext = c->w_tile_ext;
                a.tile_flags = c->w_tile_flags;
                a.tile_far = c->w_tile_far;
                a.tile_cnt = c->w_tile_cnt;
                a.bcnt = c->w_bcnt;
                a.sv_xy = c->b_sv_xy;
                a.sv_idx = c->b_sv_idx;
                a.sv_key = c->b_sv_key;
                a.cd_xy = c->b_cd_xy;
                a.cd_idx = c->b_cd_idx;
                a.cd_key = c->b_cd_key;
                a.ka = c->b_ka;
                a.kb = c->b_kb;
                a.va = c->b_va;
                a.vb = c->b_vb;
                a.gk = c->b_gk;
                a.flag = c->b_flag;
                a.hull = c->b_hull;
                a.hull_cursor = (uint32_t*)c->b_meta;
                a.h_count = d_count;
                a.h_start = d_start;
                a.h_flags = d_flags;
                if (S_big == 0) {
                    a.S_large = L_big;
                    e = launch_wide(a, q);
                } else {
                    // the big sets on the side stream, the others on q
                    WideArgs big = a, rest = a;
                    big.S = S_big;
                    big.S_large = L_big;
                    big.NT = (uint32_t)NT_big;
                    rest.order = c->b_order + S_big;
                    rest.S = S - S_big;
                    rest.S_large = L_rest;
                    rest.t_base = (uint32_t)NT_big;
                    rest.NT = (uint32_t)(NT - NT_big);
                    e = hipEventRecord(c->ev_fork, q);
                    if (e == hipSuccess) e = hipStreamWaitEvent(c->side_stream, c->ev_fork, 0);
                    if (e == hipSuccess) e = launch_wide(big, c->side_stream);
                    if (e == hipSuccess) e = launch_wide(rest, q);
                    if (e == hipSuccess) e = hipEventRecord(c->ev_join, c->side_stream);
                    if (e == hipSuccess) e = hipStreamWaitEvent(q, c->ev_join, 0);
                }
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(c->hb_meta, c->b_meta, (size_t)(3 * S + 1) * 4, hipMemcpyDeviceToHost, q);
            return e;
        }
        hipError_t e = hipMemcpyAsync(c->b_offs, c->hb_offs, (size_t)(S + 1) * 8, hipMemcpyHostToDevice, q);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->b_order, c->hb_order, (size_t)S * 4, hipMemcpyHostToDevice, q);
        if (e == hipSuccess) e = launch_batch_clear((uint32_t*)c->b_meta, q);
        if (e == hipSuccess)
            e = launch_batch(reinterpret_cast<const double2*>(d_xy), c->b_offs, c->b_order, S, c->b_sv_xy,
                             c->b_sv_idx, c->b_sv_key, c->b_cd_xy, c->b_cd_idx, c->b_cd_key, c->b_ka,
                             c->b_kb, c->b_va, c->b_vb, c->b_flag, c->b_hull, (uint32_t*)c->b_meta,
                             d_count, d_start, d_flags, c->ctr, c->batch_grid, q);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->hb_meta, c->b_meta, (size_t)(3 * S + 1) * 4, hipMemcpyDeviceToHost, q);
        return e;
    };
    if (c->have_events) HX_TRY(hipEventRecord(c->ev[HULL2D_NUM_STAGES], s));
    bool replayed = false;
    if (c->opt.batch_graph && !c->bgraph_off) {
        const bool same = c->bgraph && c->bg_S == S && c->bg_N == N && c->bg_xy == d_xy &&
                          c->bg_ws == (const void*)c->b_sv_xy && c->bg_hb == (const void*)c->hb_offs &&
                          c->bg_grid == c->batch_grid && c->bg_engine == engine && c->bg_nt == NT &&
                          c->bg_wm == (const void*)c->wmem && c->bg_big == S_big && c->bg_nt_big == NT_big &&
                          c->bg_large[0] == L_big && c->bg_large[1] == L_rest;
        if (!same) {
            if (c->bgraph) {
                (void)hipGraphExecDestroy(c->bgraph);
                c->bgraph = nullptr;
            }
            // captured on a stream of its own (the caller's stream may be the
            // null stream, which cannot be captured), replayed on the caller's
            if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
                (void)hipGetLastError();
                c->cap_stream = nullptr;
            }
            hipGraph_t g = nullptr;
            bool ok = c->cap_stream &&
                      hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                const hipError_t we = device_work(c->cap_stream);
                ok = hipStreamEndCapture(c->cap_stream, &g) == hipSuccess && we == hipSuccess && g;
            }
            if (ok) ok = hipGraphInstantiate(&c->bgraph, g, nullptr, nullptr, 0) == hipSuccess;
            if (g) (void)hipGraphDestroy(g);
            if (!ok) {
                (void)hipGetLastError();
                if (c->bgraph) (void)hipGraphExecDestroy(c->bgraph);
                c->bgraph = nullptr;
                c->bgraph_off = true;
            } else {
                c->bg_S = S;
                c->bg_N = N;
                c->bg_xy = d_xy;
                c->bg_ws = (const void*)c->b_sv_xy;
                c->bg_hb = (const void*)c->hb_offs;
                c->bg_grid = c->batch_grid;
                c->bg_engine = engine;
                c->bg_nt = NT;
                c->bg_big = S_big;
                c->bg_nt_big = NT_big;
                c->bg_large[0] = L_big;
                c->bg_large[1] = L_rest;
                c->bg_wm = (const void*)c->wmem;
            }
        }
        if (c->bgraph) {
            HX_TRY(hipGraphLaunch(c->bgraph, s));
            replayed = true;
        }
    }
    if (!replayed) HX_TRY(device_work(s));
    HX_TRY(spin_sync(c));
    const int32_t* cnt = c->hb_meta + 1;
    const int32_t* start = cnt + S;
    const uint32_t* flags = (const uint32_t*)(start + S);
    uint32_t any = 0;
    for (int32_t i = 0; i < S; ++i) any |= flags[i];
    if (any & kFlagNonfinite) return HULL2D_ERR_NONFINITE;
    if (any & kFlagRange) return HULL2D_ERR_RANGE;
    const int64_t total = (int64_t)(uint32_t)c->hb_meta[0];
    st = ensure_batch_hull(c, total);
    if (st != HULL2D_OK) return st;
    if (total > 0) {
        HX_TRY(hipMemcpyAsync(c->hb_hull, c->b_hull, (size_t)total * 4, hipMemcpyDeviceToHost, s));
    }
    if (c->have_events) HX_TRY(hipEventRecord(c->ev[HULL2D_NUM_STAGES + 1], s));
    HX_TRY(spin_sync(c));
    float ms_dev = 0.f;
    if (c->have_events) (void)hipEventElapsedTime(&ms_dev, c->ev[HULL2D_NUM_STAGES], c->ev[HULL2D_NUM_STAGES + 1]);

    // sets the workgroups left to the single-hull path
    std::vector<std::pair<int32_t, std::vector<int32_t>>> side;
    if (any & kBatchFallback) {
        for (int32_t i = 0; i < S; ++i) {
            if (!(flags[i] & kBatchFallback)) continue;
            const int64_t n = h_offsets[i + 1] - h_offsets[i];
            std::vector<int32_t> hv((size_t)std::max<int64_t>(n, 1));
            int64_t h = 0;
            st = hull2d_compute(c, d_xy + 2 * h_offsets[i], n, hv.data(), (int64_t)hv.size(), &h,
                                nullptr);
            if (st != HULL2D_OK) return st;
            hv.resize((size_t)h);
            side.emplace_back(i, std::move(hv));
        }
    }
    size_t si = 0;
    int64_t need = 0;
    for (int32_t i = 0; i < S; ++i) {
        int64_t h = cnt[i];
        if (si < side.size() && side[si].first == i) h = (int64_t)side[si++].second.size();
        need += h;
        h_out_offsets[i + 1] = need;
    }
    if (need > cap) {
        if (stats) stats->ms_total = ms_since(t_start);
        return HULL2D_ERR_CAPACITY;
    }
    si = 0;
    for (int32_t i = 0; i < S; ++i) {
        int32_t* dst = h_out + h_out_offsets[i];
        if (si < side.size() && side[si].first == i) {
            const std::vector<int32_t>& hv = side[si++].second;
            if (!hv.empty()) std::memcpy(dst, hv.data(), hv.size() * 4);
        } else if (cnt[i] > 0) {
            std::memcpy(dst, c->hb_hull + start[i], (size_t)cnt[i] * 4);
        }
    }
    if (stats) {
        stats->n_hull = need;
        stats->n_candidates = (int64_t)side.size();  // sets finished on the host
        stats->ms_device = ms_dev;
        stats->ms_total = ms_since(t_start);
    }
    return HULL2D_OK;
}

hull2d_status hull2d_set_weights(hull2d_ctx* c, const float* h_params, int64_t count) {
    if (!c || !h_params || count != kMlpParams) return HULL2D_ERR_INVALID_ARG;
    if (c->broken) return HULL2D_ERR_DEVICE;
    for (int64_t i = 0; i < count; ++i)
        if (!(std::fabs(h_params[i]) <= 3.4e38f)) return HULL2D_ERR_WEIGHTS;
    if (hipSetDevice(c->device) != hipSuccess) return HULL2D_ERR_DEVICE;
    hull2d_status st = ensure_learned(c);
    if (st != HULL2D_OK) return st;
    HX_TRY(hipMemcpyAsync(c->m_params, h_params, (size_t)count * 4, hipMemcpyHostToDevice, c->stream));
    HX_TRY(hipMemsetAsync(c->m_am, 0, (size_t)count * 4, c->stream));
    HX_TRY(hipMemsetAsync(c->m_av, 0, (size_t)count * 4, c->stream));
    HX_TRY(refresh_inference(c));
    HX_TRY(hipStreamSynchronize(c->stream));
    c->adam_t = 0;
    c->have_weights = true;
    return HULL2D_OK;
}

hull2d_status hull2d_load_weights(hull2d_ctx* c, const char* path) {
    if (!c || !path) return HULL2D_ERR_INVALID_ARG;
    FILE* f = std::fopen(path, "rb");
    if (!f) return HULL2D_ERR_WEIGHTS;
    std::vector<float> w((size_t)kMlpParams);
    const size_t got = std::fread(w.data(), 4, w.size(), f);
    const bool extra = std::fgetc(f) != EOF;
    std::fclose(f);
    if (got != w.size() || extra) return HULL2D_ERR_WEIGHTS;
    return hull2d_set_weights(c, w.data(), kMlpParams);
}

hull2d_status hull2d_get_weights(hull2d_ctx* c, float* h_params, int64_t count) {
    if (!c || !h_params || count != kMlpParams) return HULL2D_ERR_INVALID_ARG;
    if (!c->have_weights) return HULL2D_ERR_WEIGHTS;
    if (hipSetDevice(c->device) != hipSuccess) return HULL2D_ERR_DEVICE;
    HX_TRY(hipMemcpyAsync(h_params, c->m_params, (size_t)count * 4, hipMemcpyDeviceToHost, c->stream));
    HX_TRY(hipStreamSynchronize(c->stream));
    return HULL2D_OK;
}

hull2d_status hull2d_histogram(hull2d_ctx* c, const double* d_xy, int64_t n, float* d_x) {
    if (!c || n < 0 || !d_x || (n > 0 && !d_xy)) return HULL2D_ERR_INVALID_ARG;
    if (c->broken) return HULL2D_ERR_DEVICE;
    if (hipSetDevice(c->device) != hipSuccess) return HULL2D_ERR_DEVICE;
    hull2d_status st = ensure_learned(c);
    if (st != HULL2D_OK) return st;
    HX_TRY(launch_histogram_sample(d_xy, n, c->l_part, learned_grid(n, c->cu_count), c->l_hist, c->stream));
    HX_TRY(launch_hist_to_x(c->l_hist, n, d_x, c->stream));
    HX_TRY(hipStreamSynchronize(c->stream));
    return HULL2D_OK;
}

hull2d_status hull2d_mlp_infer(hull2d_ctx* c, const float* d_x, int32_t rows, float* d_y) {
    if (!c || rows < 0 || (rows > 0 && (!d_x || !d_y))) return HULL2D_ERR_INVALID_ARG;
    if (!c->have_weights) return HULL2D_ERR_WEIGHTS;
    if (rows == 0) return HULL2D_OK;
    if (rows > 65535) return HULL2D_ERR_INVALID_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return HULL2D_ERR_DEVICE;
    hull2d_status st = ensure_train(c, rows);
    if (st != HULL2D_OK) return st;
    HX_TRY(launch_mlp_infer(d_x, rows, mlp_dev(c), c->t_h1, c->t_h2, d_y, c->stream));
    HX_TRY(hipStreamSynchronize(c->stream));
    return HULL2D_OK;
}

hull2d_status hull2d_train_step(hull2d_ctx* c, const float* d_x, const float* d_t, int32_t B,
                                float lr, int32_t apply, float* h_loss, float* h_grad) {
    if (!c || !d_x || !d_t || B < 1 || B > 4096) return HULL2D_ERR_INVALID_ARG;
    if (!c->have_weights) return HULL2D_ERR_WEIGHTS;
    if (c->broken) return HULL2D_ERR_DEVICE;
    if (hipSetDevice(c->device) != hipSuccess) return HULL2D_ERR_DEVICE;
    hull2d_status st = ensure_train(c, B);
    if (st != HULL2D_OK) return st;
    hipStream_t s = c->stream;
    const float* p = c->m_params;
    float* g = c->m_grad;
    const int H = kMlpHidden, I = kMlpIn, O = kMlpOut;
    // forward
    HX_TRY(launch_gemm(B, H, I, d_x, I, 0, p + kOffW1, I, 1, p + kOffB1, 1, nullptr, c->t_h1, H, s));
    HX_TRY(launch_gemm(B, H, H, c->t_h1, H, 0, p + kOffW2, H, 1, p + kOffB2, 1, nullptr, c->t_h2, H, s));
    HX_TRY(launch_gemm(B, O, H, c->t_h2, H, 0, p + kOffW3, H, 1, p + kOffB3, 0, nullptr, c->t_y, O, s));
    HX_TRY(launch_mse(c->t_y, d_t, B * O, c->t_d3, c->l_loss, s));
    // backward
    HX_TRY(launch_gemm(O, H, B, c->t_d3, O, 1, c->t_h2, H, 0, nullptr, 0, nullptr, g + kOffW3, H, s));
    HX_TRY(launch_colsum(c->t_d3, B, O, g + kOffB3, s));
    HX_TRY(launch_gemm(B, H, O, c->t_d3, O, 0, p + kOffW3, H, 0, nullptr, 0, c->t_h2, c->t_d2, H, s));
    HX_TRY(launch_gemm(H, H, B, c->t_d2, H, 1, c->t_h1, H, 0, nullptr, 0, nullptr, g + kOffW2, H, s));
    HX_TRY(launch_colsum(c->t_d2, B, H, g + kOffB2, s));
    HX_TRY(launch_gemm(B, H, H, c->t_d2, H, 0, p + kOffW2, H, 0, nullptr, 0, c->t_h1, c->t_d1, H, s));
    HX_TRY(launch_gemm(H, I, B, c->t_d1, H, 1, d_x, I, 0, nullptr, 0, nullptr, g + kOffW1, I, s));
    HX_TRY(launch_colsum(c->t_d1, B, H, g + kOffB1, s));
    float loss = 0.f;
    HX_TRY(hipMemcpyAsync(&loss, c->l_loss, 4, hipMemcpyDeviceToHost, s));
    if (h_grad) HX_TRY(hipMemcpyAsync(h_grad, g, (size_t)kMlpParams * 4, hipMemcpyDeviceToHost, s));
    if (apply) {
        const float b1 = 0.9f, b2 = 0.999f;
        c->adam_t += 1;
        const float c1 = 1.f - std::pow(b1, (float)c->adam_t);
        const float c2 = 1.f - std::pow(b2, (float)c->adam_t);
        HX_TRY(launch_adam(c->m_params, g, c->m_am, c->m_av, kMlpParams, lr, b1, b2, 1e-8f, c1, c2, s));
        HX_TRY(refresh_inference(c));
    }
    HX_TRY(hipStreamSynchronize(s));
    if (h_loss) *h_loss = loss;
    return HULL2D_OK;
}

hull2d_status hull2d_debug_learned(hull2d_ctx* c, double* dirs, int32_t* cand, float* y, int32_t* nv) {
    if (!c) return HULL2D_ERR_INVALID_ARG;
    if (!c->have_last || !c->last_learned) return HULL2D_ERR_INVALID_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return HULL2D_ERR_DEVICE;
    LearnOut L;
    HX_TRY(hipMemcpyAsync(&L, c->learn, sizeof(LearnOut), hipMemcpyDeviceToHost, c->stream));
    HX_TRY(hipStreamSynchronize(c->stream));
    if (dirs) std::memcpy(dirs, L.dirs, sizeof(L.dirs));
    if (cand) std::memcpy(cand, L.cand, sizeof(L.cand));
    if (y) std::memcpy(y, L.y, sizeof(L.y));
    if (nv) *nv = L.poly.nv;
    return HULL2D_OK;
}

hull2d_status hull2d_debug_orient(hull2d_ctx* c, const double* d_abc, int64_t count, int32_t* d_out) {
    if (!c || count < 0 || (count > 0 && (!d_abc || !d_out))) return HULL2D_ERR_INVALID_ARG;
    if (c->broken) return HULL2D_ERR_DEVICE;
    if (hipSetDevice(c->device) != hipSuccess) return HULL2D_ERR_DEVICE;
    HX_TRY(launch_debug_orient(d_abc, count, d_out, c->stream));
    HX_TRY(hipStreamSynchronize(c->stream));
    return HULL2D_OK;
}

hull2d_status hull2d_debug_angle_key(hull2d_ctx* c, const double* d_xy, int64_t count, double x0,
                                     double y0, uint32_t* d_out) {
    if (!c || count < 0 || (count > 0 && (!d_xy || !d_out))) return HULL2D_ERR_INVALID_ARG;
    if (c->broken) return HULL2D_ERR_DEVICE;
    if (hipSetDevice(c->device) != hipSuccess) return HULL2D_ERR_DEVICE;
    HX_TRY(launch_debug_key(d_xy, count, x0, y0, d_out, c->stream));
    HX_TRY(hipStreamSynchronize(c->stream));
    return HULL2D_OK;
}

hull2d_status hull2d_debug_stages(hull2d_ctx* c, int32_t* extremes, int32_t* sorted, int32_t* round2,
                                  int64_t cap, int64_t* counts) {
    if (!c || cap < 0) return HULL2D_ERR_INVALID_ARG;
    if (!c->have_last || c->last_chain) return HULL2D_ERR_INVALID_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return HULL2D_ERR_DEVICE;
    const DevStatus& D = c->last_ds;
    const DevStatus& DS = c->last_ds2;
    const int64_t ms = D.n_sorted, m2 = (int64_t)DS.n_kept + 1;
    int64_t l = 0;
    if (ms > 0) l = c->last_full ? (int64_t)D.l_pos + 1 : (int64_t)D.n_right + 1;
    if (counts) {
        counts[0] = ms;
        counts[1] = l;
        counts[2] = m2;
        counts[3] = D.l_idx;
        counts[4] = c->last_full ? 1 : 0;
        counts[5] = DS.n_sorted;
    }
    if (extremes)
        for (int k = 0; k < 4; ++k) extremes[k] = D.ext[k];
    if ((sorted && c->last_full && cap < ms) || (round2 && cap < m2)) return HULL2D_ERR_CAPACITY;
    if (sorted && c->last_full && ms > 0) {
        // the sorted slots sit in vals_a after four passes
        std::vector<uint32_t> sl((size_t)ms), ix((size_t)c->last_n);
        HX_TRY(hipMemcpy(sl.data(), c->last_ws.vals_a, (size_t)ms * sizeof(uint32_t), hipMemcpyDeviceToHost));
        HX_TRY(hipMemcpy(ix.data(), c->last_ws.comp_idx, (size_t)c->last_n * sizeof(uint32_t),
                         hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < ms; ++i) sorted[i] = (int32_t)ix[sl[i]];
    }
    if (round2) {
        // the kept points in angular order, read back from the device: the
        // tail's kept slots into the candidates (right region, P_l, left
        // region), or the compacted list of the multi-kernel path
        const Workspace& w = c->last_ws;
        round2[0] = D.p0_idx;
        const int64_t m = m2 - 1;
        if (m > 0 && c->last_tail) {
            uint32_t cnt[2];
            std::vector<uint16_t> sl(2 * (size_t)kTailCap);
            std::vector<uint32_t> ix((size_t)DS.n_sorted);
            HX_TRY(hipMemcpy(cnt, w.tail_count, sizeof(cnt), hipMemcpyDeviceToHost));
            HX_TRY(hipMemcpy(sl.data(), w.tail_slot, sl.size() * sizeof(uint16_t), hipMemcpyDeviceToHost));
            HX_TRY(hipMemcpy(ix.data(), w.cand_idx, ix.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
            if ((int64_t)cnt[0] + 1 + (int64_t)cnt[1] != m) return HULL2D_ERR_DEVICE;
            int64_t o = 1;
            for (uint32_t k = 0; k < cnt[0]; ++k) round2[o++] = (int32_t)ix[sl[k]];
            round2[o++] = (int32_t)ix[DS.l_slot];
            for (uint32_t k = 0; k < cnt[1]; ++k) round2[o++] = (int32_t)ix[sl[kTailCap + k]];
        } else if (m > 0) {
            HX_TRY(hipMemcpy(round2 + 1, w.out_idx, (size_t)m * sizeof(int32_t), hipMemcpyDeviceToHost));
        }
    }
    return HULL2D_OK;
}

hull2d_status hull2d_debug_chain(hull2d_ctx* c, int64_t* counts, int32_t* kept, int64_t cap) {
    if (!c || cap < 0) return HULL2D_ERR_INVALID_ARG;
    if (!c->have_last || !c->last_chain) return HULL2D_ERR_INVALID_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return HULL2D_ERR_DEVICE;
    const ChainHost& H = c->last_chain_host;
    int64_t total = 0;
    for (int r = 0; r < 4; ++r) total += H.n_kept[r];
    if (counts) {
        int distinct = 0;
        for (int k = 0; k < 4; ++k) {
            bool dup = false;
            for (int j = 0; j < k; ++j) dup |= (H.cx[j] == H.cx[k] && H.cy[j] == H.cy[k]);
            distinct += dup ? 0 : 1;
        }
        counts[0] = H.m1;
        for (int r = 0; r < 4; ++r) {
            counts[1 + r] = H.n_region[r];
            counts[5 + r] = H.n_cand[r];
            counts[9 + r] = H.n_kept[r];
        }
        counts[13] = total + distinct;
    }
    if (kept) {
        if (cap < total) return HULL2D_ERR_CAPACITY;
        int64_t o = 0;
        for (int r = 0; r < 4; ++r) {
            if (H.n_kept[r] > 0)
                HX_TRY(hipMemcpy(kept + o, c->last_ws.out_idx + H.kept_at[r], (size_t)H.n_kept[r] * sizeof(int32_t),
                                 hipMemcpyDeviceToHost));
            o += H.n_kept[r];
        }
    }
    return HULL2D_OK;
}

hull2d_status hull2d_debug_round1(hull2d_ctx* c, int32_t* idx, int64_t cap, int64_t* n_out) {
    if (!c || !n_out || cap < 0 || (cap > 0 && !idx)) return HULL2D_ERR_INVALID_ARG;
    if (!c->have_last || c->last_chain) return HULL2D_ERR_INVALID_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return HULL2D_ERR_DEVICE;
    const int64_t ms = c->last_ds.n_sorted;
    *n_out = ms;
    if (cap < ms) return HULL2D_ERR_CAPACITY;
    if (ms == 0) return HULL2D_OK;
    // segment b holds its survivors in input order at [b * chunk, + seg_count[b])
    const int segs = c->last_segs;
    const int64_t chunk = filter1_chunk(c->last_n, segs);
    std::vector<uint32_t> cnt((size_t)segs), ix((size_t)c->last_n);
    HX_TRY(hipMemcpy(cnt.data(), c->last_ws.seg_count, (size_t)segs * sizeof(uint32_t), hipMemcpyDeviceToHost));
    HX_TRY(hipMemcpy(ix.data(), c->last_ws.comp_idx, (size_t)c->last_n * sizeof(uint32_t), hipMemcpyDeviceToHost));
    int64_t o = 0;
    for (int b = 0; b < segs; ++b)
        for (uint32_t k = 0; k < cnt[(size_t)b] && o < ms; ++k) idx[o++] = (int32_t)ix[(size_t)(b * chunk + k)];
    if (o != ms) return HULL2D_ERR_DEVICE;
    return HULL2D_OK;
}

}  // extern "C"
