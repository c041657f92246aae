// api.cpp -- host side of the C ABI declared in include/epic.h: context and
// workspace management, host-side validation, per-pair descriptors, and the
// launch sequence of the interpolation (Algorithm 1 of the paper):
//   clear -> seed -> geodesic transform -> graph emit -> CSR scan ->
//   CSR scatter -> K-NN + fit -> assignment
// Every stage is one launch for all pairs of a call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "epic.h"
#include "epic_dev.h"

using namespace epic;

namespace {

constexpr int kMaxPairs = 1024;      // pairs per call
constexpr int kAutoPassesStart = 16;    // automatic budget before any call finished
constexpr int kAutoPassesHistory = 8;   // recent needs the automatic budget covers
constexpr int kAutoPassesMin = 4;
constexpr int kRing = 4;             // descriptor upload slots
constexpr size_t kAlign = 256;
constexpr int kMaxK = 256;
constexpr int kStages = 8;
constexpr int kProfRing = 64;
const char* const kStageNames[kStages] = {"clear", "seed", "geodesic", "graph_emit",
                                          "csr_scan", "csr_scatter", "knn_fit", "assign"};

thread_local std::string g_last_error;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

int next_pow2(long long v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

int hash_cap_for(int N) { return next_pow2(std::max(1024LL, 16LL * N)); }

struct Tiling {
    int tw, th;
};

Tiling tiling_from(const epic_options& o) {
    if (o.tile_h == 32) return {32, 32};
    if (o.tile_h == 64) return {32, 64};
    return {32, 16};
}

size_t pair_bytes(int H, int W, int N, int precision) {
    const size_t HW = (size_t)H * W;
    const size_t cap = (size_t)hash_cap_for(N);
    size_t b = 0;
    if (precision == 1) {
        b += align_up(4 * HW);            // labels
        b += align_up(8 * cap);           // hval64
        b += align_up(8 * (size_t)N);     // minin64
        b += align_up(8 * cap);           // adjw64
        b += align_up(8 * cap);           // nbmin64
        b += align_up(48 * (size_t)N);    // params64
    }
    b += align_up(8 * HW);            // keys
    b += align_up(4 * (size_t)N);     // seed_pix
    b += align_up(8 * cap);           // hkey
    b += align_up(4 * cap);           // hval
    b += 3 * align_up(4 * (size_t)N); // deg, fill, minin
    b += align_up(4 * ((size_t)N + 1));
    b += align_up(16 * cap);          // adjacency records
    b += align_up(4 * (size_t)N);     // K-NN overflow list share
    b += align_up(24 * (size_t)N);    // params
    b += align_up(4 * C_NCOUNTERS);
    b += align_up(16 * (size_t)N);    // kept matches (consistency check)
    b += align_up(4 * (size_t)N);     // their original indices
    return b;
}

size_t tiles_of(int H, int W, Tiling t) {
    return (size_t)((W + t.tw - 1) / t.tw) * ((H + t.th - 1) / t.th);
}

constexpr size_t kFixed = 4096 + (size_t)kRing * kMaxPairs * sizeof(PairDev);
static_assert(kFixed % 256 == 0, "the carved arrays start 256-byte aligned (16-byte vector accesses rely on it)");
// per-tile arrays of a call: two dirty-flag arrays and three dirty-tile lists
constexpr size_t kTileArrays = 5;

}  // namespace

struct epic_ctx {
    int device = 0;
    epic_options opt{};
    char* ws = nullptr;
    size_t ws_bytes = 0;
    PairDev* h_desc = nullptr;          // pinned, kRing * kMaxPairs
    hipEvent_t ring_ev[kRing]{};
    bool ring_used[kRing]{};
    int ring_next = 0;
    // last call
    hipStream_t last_stream = nullptr;
    int last_npairs = 0;
    int* last_counters[kMaxPairs]{};    // per pair of the last call (fixed: calls allocate nothing)
    int* g_any = nullptr;
    int* g_error = nullptr;
    int passes = 16;                    // geodesic passes launched per call (fixed budget)
    bool auto_passes = true;            // budget from the passes the last call needed
    // pinned, 4 ints written by the transform's finisher(s): slots 0-1 the
    // transform of a call (FP64: its two phases), 2-3 the first transform
    // of a call with the consistency check, whose seeds differ
    int* h_passes_used = nullptr;
    int used_hist[4][kAutoPassesHistory]{};  // needs seen at the last calls, per slot (0: none yet)
    int used_next[4]{};
    // stage timing
    bool prof = false;
    hipEvent_t prof_ev[kProfRing][kStages + 1]{};
    bool prof_ok[kProfRing]{};
    int prof_next = 0;
    int prof_count = 0;
    bool last_pruned = false;           // the last call ran the consistency check
    PairDev* last_desc = nullptr;       // device descriptor table of the last call
    size_t last_used = 0;               // workspace bytes the last call carved (from its start)
    bool last_pass_visits = false;      // the last call counted its transform's visits per pass
};

extern "C" {

const char* epic_strerror(int s) {
    switch (s) {
        case EPIC_OK: return "ok";
        case EPIC_ERR_ARG: return "invalid argument";
        case EPIC_ERR_WORKSPACE: return "workspace too small for this call";
        case EPIC_ERR_NO_MATCHES: return "no match lies in the image";
        case EPIC_ERR_HIP: return "HIP runtime error";
        case EPIC_ERR_BUDGET: return "request exceeds its memory budget";
        case EPIC_ERR_CAPACITY: return "fixed-capacity device structure overflowed";
        case EPIC_ERR_CONVERGENCE: return "geodesic transform did not converge within its bound";
        case EPIC_ERR_COST: return "cost map holds a value that is not finite and > 0";
        case EPIC_ERR_INVARIANT: return "a debug_validate check of the transform or the graph failed";
        default: return "unknown status";
    }
}

const char* epic_last_error(void) { return g_last_error.c_str(); }

int epic_validate(const float* cost, int H, int W, const float* matches, int N, int K, float a, int mode,
                  const float* flow) {
    if (!cost || !matches || !flow) return EPIC_ERR_ARG;
    // vector loads and stores: matches rows are read as float4, flow as float2
    if (((uintptr_t)cost & 3) || ((uintptr_t)matches & 15) || ((uintptr_t)flow & 7)) return EPIC_ERR_ARG;
    if (H < 1 || W < 1 || N < 1 || K < 1 || K > kMaxK) return EPIC_ERR_ARG;
    if ((long long)H * W >= (1LL << 31) || N >= (1 << 30)) return EPIC_ERR_ARG;
    if (!std::isfinite(a) || a < 0.0f) return EPIC_ERR_ARG;
    if (mode != EPIC_NW && mode != EPIC_LA) return EPIC_ERR_ARG;
    return EPIC_OK;
}

size_t epic_workspace_bytes(int H, int W, int N, int K, int mode, int precision) {
    if (H < 1 || W < 1 || N < 1 || K < 1 || K > kMaxK || (mode != 0 && mode != 1) ||
        (precision != 0 && precision != 1) || (long long)H * W >= (1LL << 31))
        return 0;
    // the smallest tiling gives the largest tile-state array and queue ring
    const size_t t = tiles_of(H, W, Tiling{32, 16});       // the smallest tile
    return kFixed + kTileArrays * align_up(4 * t) + pair_bytes(H, W, N, precision);
}

epic_ctx* epic_create(int device, size_t workspace_bytes, const epic_options* opts) {
    g_last_error.clear();
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        g_last_error = "no such HIP device";
        return nullptr;
    }
    epic_ctx* c = new epic_ctx();
    c->device = device;
    epic_options o{};
    o.connectivity = 8;
    o.la_weight_power = 2;
    o.precision = 0;
    o.fp64_route = 1e-3f;
    o.degenerate_tau = 1e-9;
    o.tile_w = 32;
    o.tile_h = 16;
    o.geo_passes = 0;
    o.geo_threads = 0;
    o.debug_validate = 0;
    o.prune_px = 0.0f;
    if (opts) {
        o = *opts;
        if (o.connectivity != 4) o.connectivity = 8;
        if (o.la_weight_power != 1) o.la_weight_power = 2;
        if (o.precision != 1) o.precision = 0;
        if (!(o.fp64_route > 0.0f)) o.fp64_route = 1e-3f;
        if (!(o.degenerate_tau > 0.0)) o.degenerate_tau = 1e-9;
        const Tiling t = tiling_from(o);
        o.tile_w = t.tw;
        o.tile_h = t.th;
        if (o.geo_passes < 0) o.geo_passes = 0;
        if (o.geo_passes > kMaxPasses - 1) o.geo_passes = kMaxPasses - 1;
        if (o.debug_validate != 1 && o.debug_validate != 2) o.debug_validate = 0;
        if (!(o.tile_h == 16 && (o.geo_threads == 128 || o.geo_threads == 256))) o.geo_threads = 0;
        if (!(o.prune_px > 0.0f)) o.prune_px = 0.0f;     // off (also for NaN)
    }
    c->auto_passes = o.geo_passes == 0;
    c->passes = c->auto_passes ? kAutoPassesStart : o.geo_passes;
    c->opt = o;
    auto fail = [&](const char* what) {
        g_last_error = what;
        epic_destroy(c);
        return (epic_ctx*)nullptr;
    };
    if (hipSetDevice(device) != hipSuccess) return fail("hipSetDevice failed");
    c->ws_bytes = std::max(workspace_bytes, kFixed + 4096);
    if (hipMalloc((void**)&c->ws, c->ws_bytes) != hipSuccess) return fail("workspace allocation failed");
    if (hipHostMalloc((void**)&c->h_desc, sizeof(PairDev) * kRing * kMaxPairs, hipHostMallocDefault) !=
        hipSuccess)
        return fail("pinned descriptor allocation failed");
    for (int i = 0; i < kRing; ++i)
        if (hipEventCreateWithFlags(&c->ring_ev[i], hipEventDisableTiming) != hipSuccess)
            return fail("event creation failed");
    if (hipHostMalloc((void**)&c->h_passes_used, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess)
        return fail("pinned counter allocation failed");
    for (int i = 0; i < 4; ++i) c->h_passes_used[i] = 0;
    c->g_error = reinterpret_cast<int*>(c->ws);
    c->g_any = reinterpret_cast<int*>(c->ws) + 256;         // kMaxPasses ints
    return c;
}

void epic_destroy(epic_ctx* c) {
    if (!c) return;
    hipSetDevice(c->device);
    for (int i = 0; i < kRing; ++i)
        if (c->ring_ev[i]) {
            if (c->ring_used[i]) hipEventSynchronize(c->ring_ev[i]);
            hipEventDestroy(c->ring_ev[i]);
        }
    for (int r = 0; r < kProfRing; ++r)
        for (int i = 0; i <= kStages; ++i)
            if (c->prof_ev[r][i]) hipEventDestroy(c->prof_ev[r][i]);
    if (c->h_desc) hipHostFree(c->h_desc);
    if (c->h_passes_used) hipHostFree(c->h_passes_used);
    if (c->ws) hipFree(c->ws);
    delete c;
}

}  // extern "C"

namespace {

struct DebugOut {
    float* D = nullptr;
    int* L = nullptr;
    int* em = nullptr;
    int* en = nullptr;
    float* ew = nullptr;
    int max_edges = 0;
    int* n_edges = nullptr;
    int* knn_idx = nullptr;
    float* knn_d = nullptr;
    float* params = nullptr;
    // consistency check only (epic_prune): stop after it, write the kept
    // original indices and their count
    bool prune_only = false;
    float prune_px = 0.0f;
    int* kept = nullptr;
    int* n_kept = nullptr;
    // partial sequences (the exact per-pixel interpolation): 1 = stop after
    // the seeding, 2 = after the transform; geo_passes > 0 overrides the
    // pass budget
    int stop_after = 0;
    int geo_passes = 0;
    // the exact interpolation's single-source transforms: per-pixel bound
    // on the distances worth keeping (32 x 16 tiles)
    const float* ubound = nullptr;
    const int4* clear_boxes = nullptr;   // per pair: what its keys' clearing must reset
};

// Where a call's descriptor table lives: the context's upload ring (default)
// or buffers owned by a captured graph.
struct DescTarget {
    PairDev* host;      // pinned
    PairDev* dev;
};

int run_pairs(epic_ctx* c, const epic_request* reqs, int n, hipStream_t stream, const DebugOut* dbg,
              const DescTarget* tgt = nullptr, size_t reserve_tail = 0) {
    if (!c || !reqs || n < 1 || n > kMaxPairs) return EPIC_ERR_ARG;
    for (int i = 0; i < n; ++i) {
        const epic_request& r = reqs[i];
        const float* flow_chk = (dbg && !r.flow) ? r.cost : r.flow;   // debug may omit the flow
        const int v = epic_validate(r.cost, r.H, r.W, r.matches, r.N, r.K, r.a, r.mode, flow_chk);
        if (v != EPIC_OK) return v;
    }
    // the FP64 transform runs on 32 x 16 tiles
    const bool bounded = dbg && dbg->ubound;
    const Tiling tl = c->opt.precision == 1 || bounded ? Tiling{32, 16} : Tiling{c->opt.tile_w, c->opt.tile_h};
    // ---- carve the workspace
    size_t total_tiles = 0, need = kFixed;
    for (int i = 0; i < n; ++i) total_tiles += tiles_of(reqs[i].H, reqs[i].W, tl);
    need += kTileArrays * align_up(4 * total_tiles);
    for (int i = 0; i < n; ++i) need += pair_bytes(reqs[i].H, reqs[i].W, reqs[i].N, c->opt.precision);
    if (need + reserve_tail > c->ws_bytes) return EPIC_ERR_WORKSPACE;
    if (hipSetDevice(c->device) != hipSuccess) return EPIC_ERR_HIP;

    int slot = -1;
    PairDev* hd = nullptr;
    PairDev* dd = nullptr;
    if (tgt) {
        hd = tgt->host;
        dd = tgt->dev;
    } else {
        slot = c->ring_next;
        c->ring_next = (c->ring_next + 1) % kRing;
        if (c->ring_used[slot] && hipEventSynchronize(c->ring_ev[slot]) != hipSuccess) return EPIC_ERR_HIP;
        hd = c->h_desc + (size_t)slot * kMaxPairs;
        dd = reinterpret_cast<PairDev*>(c->ws + 4096) + (size_t)slot * kMaxPairs;
    }

    char* cur = c->ws + kFixed;
    auto take = [&](size_t bytes) {
        char* p = cur;
        cur += align_up(bytes);
        return p;
    };
    u32* dirty0 = reinterpret_cast<u32*>(take(4 * total_tiles));
    u32* dirty1 = reinterpret_cast<u32*>(take(4 * total_tiles));
    u32* wl[3];
    for (int k = 0; k < 3; ++k) wl[k] = reinterpret_cast<u32*>(take(4 * total_tiles));
    long long total_n = 0;
    for (int i = 0; i < n; ++i) total_n += reqs[i].N;
    int* ovf_list = reinterpret_cast<int*>(take(4 * (size_t)total_n));
    c->last_used = need;
    long long total_px = 0;
    int tile_base = 0, pix_blocks = 0, seed_blocks = 0, src_blocks = 0, slot_blocks = 0, init_blocks = 0;
    int emit_blocks = 0;
    int kmax = 1, nmax = 1;
    for (int i = 0; i < n; ++i) c->last_counters[i] = nullptr;
    for (int i = 0; i < n; ++i) {
        const epic_request& r = reqs[i];
        PairDev& P = hd[i];
        std::memset(&P, 0, sizeof(P));
        P.cost = r.cost;
        P.matches = r.matches;
        P.flow = r.flow;
        P.H = r.H;
        P.W = r.W;
        P.N = r.N;
        P.K = r.K;
        P.a = r.a;
        P.mode = r.mode;
        kmax = std::max(kmax, r.K);
        nmax = std::max(nmax, r.N);
        P.tiles_x = (r.W + tl.tw - 1) / tl.tw;
        P.tiles_y = (r.H + tl.th - 1) / tl.th;
        P.tile_base = tile_base;
        tile_base += P.tiles_x * P.tiles_y;
        const long long HW = (long long)r.H * r.W;
        // each pair's pixel blocks come in groups of ASSIGN_PPT, one block of
        // the assignment's grid per group (the other pixel kernels check
        // their pixel index against H * W)
        total_px += HW;
        P.pix_block_base = pix_blocks;
        pix_blocks += (int)((HW + PIX_BLOCK * ASSIGN_PPT - 1) / (PIX_BLOCK * ASSIGN_PPT)) * ASSIGN_PPT;
        P.emit_block_base = emit_blocks;
        emit_blocks += ((r.W + EMIT_TW - 1) / EMIT_TW) * ((r.H + EMIT_TH - 1) / EMIT_TH);
        P.seed_block_base = seed_blocks;
        seed_blocks += (r.N + PIX_BLOCK - 1) / PIX_BLOCK;
        P.src_block_base = src_blocks;
        src_blocks += r.N;
        P.hash_cap = hash_cap_for(r.N);
        int lg = 0;
        while ((1 << lg) < P.hash_cap) ++lg;
        P.hash_shift = 64 - lg;
        P.slot_block_base = slot_blocks;
        slot_blocks += P.hash_cap / SLOT_BLOCK;
        P.init_block_base = init_blocks;
        P.init_blocks = (int)std::min<long long>(1024, std::max<long long>(1, (std::max<long long>(HW, P.hash_cap) + 1023) / 1024));
        // bounded single-source runs come 1024 to a call: a few blocks per
        // pair (each striding over its pair) keep the grid small
        if (bounded) P.init_blocks = std::min(P.init_blocks, 16);
        init_blocks += P.init_blocks;
        const size_t cap = (size_t)P.hash_cap;
        P.keys = reinterpret_cast<u64*>(take(8 * (size_t)HW));
        P.seed_pix = reinterpret_cast<int*>(take(4 * (size_t)r.N));
        P.hkey = reinterpret_cast<u64*>(take(8 * cap));
        P.hval = reinterpret_cast<u32*>(take(4 * cap));
        P.deg = reinterpret_cast<u32*>(take(4 * (size_t)r.N));
        P.fill = reinterpret_cast<u32*>(take(4 * (size_t)r.N));
        P.minin = reinterpret_cast<u32*>(take(4 * (size_t)r.N));
        P.row_ptr = reinterpret_cast<u32*>(take(4 * ((size_t)r.N + 1)));
        P.adj = reinterpret_cast<uint4*>(take(16 * cap));
        P.params = reinterpret_cast<float*>(take(24 * (size_t)r.N));
        P.counters = reinterpret_cast<int*>(take(4 * C_NCOUNTERS));
        P.matches_kept = reinterpret_cast<float*>(take(16 * (size_t)r.N));
        P.kept_idx = reinterpret_cast<int*>(take(4 * (size_t)r.N));
        if (c->opt.precision == 1) {
            P.labels = reinterpret_cast<u32*>(take(4 * (size_t)HW));
            P.hval64 = reinterpret_cast<u64*>(take(8 * cap));
            P.minin64 = reinterpret_cast<u64*>(take(8 * (size_t)r.N));
            P.adjw64 = reinterpret_cast<double*>(take(8 * cap));
            P.nbmin64 = reinterpret_cast<u64*>(take(8 * cap));
            P.params64 = reinterpret_cast<double*>(take(48 * (size_t)r.N));
        }
        c->last_counters[i] = P.counters;
        if (bounded) {
            P.ubound = dbg->ubound;
            if (dbg->clear_boxes) P.clear_box = dbg->clear_boxes + i;
        }
        if (dbg && i == 0) {
            P.dbg_knn_idx = dbg->knn_idx;
            P.dbg_knn_d = dbg->knn_d;
            if (dbg->knn_idx && !dbg->knn_d) P.dbg_knn_d = nullptr;
            P.dbg_em = (dbg->em && dbg->en && dbg->ew && dbg->n_edges) ? dbg->em : nullptr;
            P.dbg_en = dbg->en;
            P.dbg_ew = dbg->ew;
            P.dbg_max_edges = dbg->max_edges;
            P.dbg_n_edges = dbg->n_edges;
            P.dbg_kept = dbg->kept;
            P.dbg_n_kept = dbg->n_kept;
        }
    }
    if ((size_t)(cur - c->ws) > c->ws_bytes) return EPIC_ERR_WORKSPACE;
    if (dbg && dbg->knn_idx && !dbg->knn_d) return EPIC_ERR_ARG;

    RunDev run{};
    for (int k = 0; k < 3; ++k) run.wl[k] = wl[k];
    run.wl_cnt = c->g_error + 12;
    run.dirty[0] = dirty0;
    run.dirty[1] = dirty1;
    run.any = c->g_any;
    run.any2 = c->g_any + kMaxPasses;
    run.pass_visits = c->prof && c->opt.precision == 0 ? c->g_any + 2 * kMaxPasses : nullptr;
    c->last_pass_visits = run.pass_visits != nullptr;
    run.error = c->g_error;
    run.passes_used = c->h_passes_used;
    run.ovf_list = ovf_list;
    run.ovf_count = c->g_error + 8;
    run.total_tiles = tile_base;
    run.npairs = n;
    run.conn = c->opt.connectivity;
    run.bounded = bounded ? 1 : 0;
    run.tile_w = tl.tw;
    run.tile_h = tl.th;
    run.la_wpow = c->opt.la_weight_power;
    run.precision = c->opt.precision;
    run.fp64_route = c->opt.fp64_route;
    run.deg_tau = c->opt.degenerate_tau;

    // small tables travel in the first kernel's arguments (no upload copy)
    const bool inline_desc = n <= kInlinePairs;
    hipError_t e = hipSuccess;
    if (!inline_desc) {
        e = hipMemcpyAsync(dd, hd, sizeof(PairDev) * n, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess && slot >= 0) e = hipEventRecord(c->ring_ev[slot], stream);
        if (e != hipSuccess) return EPIC_ERR_HIP;
        if (slot >= 0) c->ring_used[slot] = true;
    }

    hipEvent_t* ev = nullptr;
    if (c->prof && !tgt && !(dbg && (dbg->prune_only || dbg->stop_after))) {
        const int r = c->prof_next;
        c->prof_next = (c->prof_next + 1) % kProfRing;
        ev = c->prof_ev[r];
        c->prof_ok[r] = false;
        for (int i = 0; i <= kStages && e == hipSuccess; ++i)
            if (!ev[i]) e = hipEventCreate(&ev[i]);
        if (e == hipSuccess) e = hipEventRecord(ev[0], stream);
        if (e == hipSuccess) {
            c->prof_ok[r] = true;
            c->prof_count = std::min(kProfRing, c->prof_count + 1);
        }
    }
    auto mark = [&](int stage) {
        if (ev && e == hipSuccess) e = hipEventRecord(ev[stage + 1], stream);
    };
    // Automatic budget: the largest number of passes the recently finished
    // transforms needed (read when each call is issued; the value may come
    // from an older call while the last one is still running), plus one when
    // those needs varied; the FP64 path keeps one history per phase.  Any
    // budget gives the same result: the finisher completes a transform the
    // launched passes did not.
    auto budget = [&](int phase) {
        int passes = c->passes;
        if (!c->auto_passes) return passes;
        const int used = reinterpret_cast<volatile int*>(c->h_passes_used)[phase];
        if (used <= 0) return passes;
        int* hist = c->used_hist[phase];
        hist[c->used_next[phase]] = used;
        c->used_next[phase] = (c->used_next[phase] + 1) % kAutoPassesHistory;
        int hi = 0, lo = 1 << 30;
        for (int k = 0; k < kAutoPassesHistory; ++k)
            if (hist[k] > 0) {
                hi = std::max(hi, hist[k]);
                lo = std::min(lo, hist[k]);
            }
        // FP64: when the needs vary, never fewer than the starting budget (its
        // single-workgroup finisher costs far more than idle passes)
        const int floor_ = (c->opt.precision == 1 && hi != lo) ? kAutoPassesStart : kAutoPassesMin;
        return std::min(kMaxPasses - 1, std::max(floor_, hi + (hi == lo ? 0 : 1)));
    };
    // With the consistency check (Sec. 5.1) the sequence runs twice: first
    // with NW fits and no assignment, then k_prune compacts the kept matches
    // and points each pair's descriptor at them, and the second pass
    // interpolates those.  Stage timing marks the second pass (its "clear"
    // stage then spans the whole first pass).
    const float prune_px = dbg && dbg->prune_only ? dbg->prune_px : c->opt.prune_px;
    const bool two_pass = prune_px > 0.0f;
    bool any_flow = false;
    for (int i = 0; i < n; ++i) any_flow |= reqs[i].flow != nullptr;
    for (int pass = two_pass ? 0 : 1; pass < 2 && e == hipSuccess; ++pass) {
        const bool first = pass == 0;
        const bool last = pass == 1;
        run.force_nw = first ? 1 : 0;
        run.keep_prune_counters = two_pass && last ? 1 : 0;
        run.prune_px = first ? prune_px : 0.0f;
        // each transform of the call keeps its own pass history
        const int slot0 = first ? 2 : 0;
        run.passes_used = c->h_passes_used ? c->h_passes_used + slot0 : nullptr;
        // the descriptor table travels inline only with the first launch of
        // the call (the second pass reads the table k_prune rewrote)
        const bool inl = inline_desc && (first || !two_pass);
        if (e == hipSuccess) e = launch_clear(dd, run, init_blocks, inl ? hd : nullptr, inl ? n : 0, stream);
        if (last) mark(0);
        // a pair whose cost map fails the check is not seeded (it then takes
        // the path of a pair without usable matches)
        if (e == hipSuccess && c->opt.debug_validate) e = launch_check_cost(dd, run, pix_blocks, stream);
        if (e == hipSuccess) e = launch_seed(dd, run, seed_blocks, stream);
        if (last) mark(1);
        if (dbg && dbg->stop_after == 1) break;
        const int pb0 = dbg && dbg->geo_passes > 0 ? dbg->geo_passes : budget(slot0);
        if (e == hipSuccess)
            e = c->opt.precision == 1
                    ? launch_geodesic64(dd, run, pb0, dbg && dbg->geo_passes > 0 ? pb0 : budget(slot0 + 1), stream)
                    : launch_geodesic(dd, run, tl.tw, tl.th, c->opt.geo_threads, pb0, stream);
        if (last) mark(2);
        if (dbg && dbg->stop_after == 2) break;
        if (e == hipSuccess && c->opt.debug_validate)
            e = launch_check_transform(dd, run, pix_blocks, c->opt.debug_validate == 2, stream);
        if (e == hipSuccess) e = launch_graph_emit(dd, run, emit_blocks, total_px, stream);
        if (last) mark(3);
        if (e == hipSuccess) e = launch_csr_scan(dd, run, stream);
        if (last) mark(4);
        if (e == hipSuccess) e = launch_csr_scatter(dd, run, slot_blocks, stream);
        if (e == hipSuccess && c->opt.debug_validate) e = launch_check_graph(dd, run, slot_blocks, stream);
        if (last) mark(5);
        if (e == hipSuccess) e = launch_knn_fit(dd, run, src_blocks, kmax, nmax, stream);
        if (last) mark(6);
        if (first) {
            if (e == hipSuccess) e = launch_prune(dd, run, stream);
            if (dbg && dbg->prune_only) break;
            continue;
        }
        if (e == hipSuccess && any_flow) e = launch_assign(dd, run, pix_blocks, total_px, stream);
        mark(7);
    }
    c->last_pruned = two_pass && !(dbg && dbg->prune_only);
    c->last_desc = dd;
    if (e == hipSuccess && dbg && (dbg->D || dbg->L)) e = launch_unpack(dd, run, pix_blocks, dbg->D, dbg->L, stream);
    if (e == hipSuccess && dbg && dbg->params)
        e = hipMemcpyAsync(dbg->params, hd[0].params, 24 * (size_t)reqs[0].N, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return EPIC_ERR_HIP;
    c->last_stream = stream;
    c->last_npairs = n;
    return EPIC_OK;
}

}  // namespace

extern "C" {

int epic_interp(epic_ctx* ctx, const float* cost, int H, int W, const float* matches, int N, int K, float a,
                int mode, float* flow, void* stream) {
    const int v = epic_validate(cost, H, W, matches, N, K, a, mode, flow);
    if (v != EPIC_OK) return v;
    if (!ctx) return EPIC_ERR_ARG;
    epic_request r{cost, H, W, matches, N, K, a, mode, flow};
    return run_pairs(ctx, &r, 1, (hipStream_t)stream, nullptr);
}

int epic_interp_batch(epic_ctx* ctx, const epic_request* reqs, int n, void* stream) {
    if (!ctx || !reqs || n < 1) return EPIC_ERR_ARG;
    return run_pairs(ctx, reqs, n, (hipStream_t)stream, nullptr);
}

int epic_debug_stages(epic_ctx* ctx, const float* cost, int H, int W, const float* matches, int N, int K,
                      float a, int mode, float* D, int* L, int* edge_m, int* edge_n, float* edge_w,
                      int max_edges, int* n_edges, int* knn_idx, float* knn_d, float* params, float* flow,
                      void* stream) {
    if (!ctx) return EPIC_ERR_ARG;
    DebugOut d;
    d.D = D;
    d.L = L;
    d.em = edge_m;
    d.en = edge_n;
    d.ew = edge_w;
    d.max_edges = max_edges;
    d.n_edges = n_edges;
    d.knn_idx = knn_idx;
    d.knn_d = knn_d;
    d.params = params;
    epic_request r{cost, H, W, matches, N, K, a, mode, flow};
    return run_pairs(ctx, &r, 1, (hipStream_t)stream, &d);
}

int epic_prune(epic_ctx* ctx, const float* cost, int H, int W, const float* matches, int N, int K, float a,
               float prune_px, int* kept, int* n_kept, void* stream) {
    if (!ctx || !kept || !n_kept || !(prune_px > 0.0f) || !std::isfinite(prune_px)) return EPIC_ERR_ARG;
    DebugOut d;
    d.prune_only = true;
    d.prune_px = prune_px;
    d.kept = kept;
    d.n_kept = n_kept;
    epic_request r{cost, H, W, matches, N, K, a, EPIC_NW, nullptr};
    // no flow: the debug path validates the request against its cost pointer
    return run_pairs(ctx, &r, 1, (hipStream_t)stream, &d);
}

int epic_image_cost(const epic_image* imgs, int n, float eps, void* stream) {
    if (!imgs || n < 1 || !std::isfinite(eps) || !(eps > 0.0f)) return EPIC_ERR_ARG;
    for (int i = 0; i < n; ++i) {
        const epic_image& m = imgs[i];
        if (!m.image || !m.cost || ((uintptr_t)m.image & 3) || ((uintptr_t)m.cost & 3)) return EPIC_ERR_ARG;
        if (m.H < 1 || m.W < 1 || (long long)m.H * m.W >= (1LL << 31) || m.channels < 1 || m.channels > 4)
            return EPIC_ERR_ARG;
    }
    // one launch per run of up to kImagesPerLaunch images with the same
    // channel count
    for (int i = 0; i < n;) {
        ImageCostArgs args{};
        args.eps = eps;
        const int ch = imgs[i].channels;
        int blocks = 0;
        while (i < n && args.n < kImagesPerLaunch && imgs[i].channels == ch) {
            ImageDesc& d = args.img[args.n++];
            d.image = imgs[i].image;
            d.cost = imgs[i].cost;
            d.H = imgs[i].H;
            d.W = imgs[i].W;
            d.block_base = blocks;
            blocks += image_cost_blocks(d.H, d.W);
            ++i;
        }
        if (launch_image_cost(args, ch, blocks, (hipStream_t)stream) != hipSuccess) return EPIC_ERR_HIP;
    }
    return EPIC_OK;
}

int epic_interp_image(epic_ctx* ctx, const float* image, int H, int W, int channels, float eps,
                      const float* matches, int N, int K, float a, int mode, float* flow, void* stream) {
    if (!ctx) return EPIC_ERR_ARG;
    if (!image || channels < 1 || channels > 4 || !std::isfinite(eps) || !(eps > 0.0f)) return EPIC_ERR_ARG;
    if (H < 1 || W < 1 || (long long)H * W >= (1LL << 31)) return EPIC_ERR_ARG;
    // the cost map lives at the end of the workspace, after what the call needs
    const size_t tail = align_up(4 * (size_t)H * W);
    if (tail > ctx->ws_bytes) return EPIC_ERR_WORKSPACE;
    float* cost = reinterpret_cast<float*>(ctx->ws + ((ctx->ws_bytes - tail) & ~(kAlign - 1)));
    const int v = epic_validate(cost, H, W, matches, N, K, a, mode, flow);
    if (v != EPIC_OK) return v;
    // check the workspace before anything is enqueued
    epic_request r{cost, H, W, matches, N, K, a, mode, flow};
    const size_t need = kFixed + kTileArrays * align_up(4 * tiles_of(H, W, Tiling{ctx->opt.tile_w, ctx->opt.tile_h})) +
                        pair_bytes(H, W, N, ctx->opt.precision);
    if (need + tail + kAlign > ctx->ws_bytes) return EPIC_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return EPIC_ERR_HIP;
    epic_image im{image, H, W, channels, cost};
    const int rc = epic_image_cost(&im, 1, eps, stream);
    if (rc != EPIC_OK) return rc;
    return run_pairs(ctx, &r, 1, (hipStream_t)stream, nullptr, nullptr, tail + kAlign);
}

int epic_interp_exact(epic_ctx* ctx, const float* cost, int H, int W, const float* matches, int N, int K,
                      float a, int mode, float* flow, void* stream) {
    const int v = epic_validate(cost, H, W, matches, N, K, a, mode, flow);
    if (v != EPIC_OK) return v;
    if (!ctx || K > 128) return EPIC_ERR_ARG;
    if (ctx->opt.precision != 0) return EPIC_ERR_ARG;
    const hipStream_t st = (hipStream_t)stream;
    const long long HW = (long long)H * W;
    // at the end of the workspace: the pixels' lists, the owner flags, the
    // per-pixel distance bounds and the approximate K-NN lists they come from
    const size_t lists_b = align_up(8 * (size_t)K * HW), owner_b = align_up((size_t)N);
    const size_t ub_b = align_up(4 * (size_t)HW), knn_b = align_up(4 * (size_t)N * K);
    const size_t box_b = align_up(16 * (size_t)kExactChunk);
    const size_t tail = lists_b + owner_b + ub_b + 2 * knn_b + 2 * box_b + kAlign;
    if (tail >= ctx->ws_bytes) return EPIC_ERR_WORKSPACE;
    char* tail_p = ctx->ws + ((ctx->ws_bytes - (tail - kAlign)) & ~(kAlign - 1));
    ExactArgs A{};
    A.matches = matches;
    A.N = N;
    A.K = K;
    A.H = H;
    A.W = W;
    A.HW = HW;
    A.lists = reinterpret_cast<u64*>(tail_p);
    A.owner = reinterpret_cast<unsigned char*>(tail_p + lists_b);
    A.ubound = reinterpret_cast<float*>(tail_p + lists_b + owner_b);
    A.knn_idx = reinterpret_cast<int*>(tail_p + lists_b + owner_b + ub_b);
    A.knn_d = reinterpret_cast<float*>(tail_p + lists_b + owner_b + ub_b + knn_b);
    A.boxes = reinterpret_cast<int4*>(tail_p + lists_b + owner_b + ub_b + 2 * knn_b);
    A.clear_boxes = reinterpret_cast<int4*>(tail_p + lists_b + owner_b + ub_b + 2 * knn_b + box_b);
    A.flow = flow;
    A.a = a;
    A.mode = mode;
    A.wpow = ctx->opt.la_weight_power;
    A.fp64_route = ctx->opt.fp64_route;
    A.deg_tau = ctx->opt.degenerate_tau;
    // 1. the approximated interpolation (Sec. 3.4) of the whole set: which
    //    matches hold their pixel, and each match's K nearest in the graph,
    //    whose K-th distance plus D(p) bounds the distance of every pixel's
    //    K-th nearest match (each approximated distance is the length of a
    //    path of the pixel graph)
    DebugOut approx;
    approx.knn_idx = A.knn_idx;
    approx.knn_d = A.knn_d;
    epic_request full{cost, H, W, matches, N, K, a, mode, flow};
    int rc = run_pairs(ctx, &full, 1, st, &approx, nullptr, tail);
    if (rc != EPIC_OK) return rc;
    if (launch_exact_owner(ctx->last_desc, A, st) != hipSuccess) return EPIC_ERR_HIP;
    if (launch_exact_bound(ctx->last_desc, A, st) != hipSuccess) return EPIC_ERR_HIP;
    // 2. single-source transforms bounded by those distances, one match per
    //    pair, in chunks that fit
    const Tiling tl{32, 16};
    const size_t per = pair_bytes(H, W, 1, 0) + kTileArrays * align_up(4 * tiles_of(H, W, tl)) + kAlign;
    if (ctx->ws_bytes < kFixed + tail + per) return EPIC_ERR_WORKSPACE;
    const int chunk = (int)std::min<size_t>(std::min(kMaxPairs, kExactChunk), (ctx->ws_bytes - kFixed - tail) / per);
    // generous budget: a single source's distances may cross the whole image
    const int tx = (W + tl.tw - 1) / tl.tw, ty = (H + tl.th - 1) / tl.th;
    DebugOut transform_only;
    transform_only.stop_after = 2;
    transform_only.geo_passes = std::min(kMaxPasses - 1, 2 * (tx + ty) + 8);
    transform_only.ubound = A.ubound;
    std::vector<epic_request> reqs;
    int prev_n = 0;
    for (int s0 = 0; s0 < N; s0 += chunk) {
        const int n = std::min(chunk, N - s0);
        // a chunk of the previous one's size reuses its workspace layout, so
        // only the boxes those transforms reached need clearing
        transform_only.clear_boxes = n == prev_n ? A.clear_boxes : nullptr;
        prev_n = n;
        reqs.assign(n, epic_request{});
        for (int j = 0; j < n; ++j)
            reqs[j] = epic_request{cost, H, W, matches + 4LL * (s0 + j), 1, 1, a, mode, flow};
        rc = run_pairs(ctx, reqs.data(), n, st, &transform_only, nullptr, tail);
        if (rc != EPIC_OK) return rc;
        // 3. fold the chunk into every pixel's K nearest
        if (launch_exact_select(ctx->last_desc, n, s0, s0 == 0, s0 + n == N, A, st) != hipSuccess)
            return EPIC_ERR_HIP;
        if (s0 == 0 && chunk < N && ctx->h_passes_used) {
            // the later chunks launch the passes the first one needed, and a
            // few more (their sources are alike; the finisher completes any
            // transform that needs more, so the budget never changes results)
            if (hipStreamSynchronize(st) != hipSuccess) return EPIC_ERR_HIP;
            const int used = reinterpret_cast<volatile int*>(ctx->h_passes_used)[0];
            if (used > 0) transform_only.geo_passes = std::min(transform_only.geo_passes, used + used / 2 + 4);
        }
    }
    // 4. one fit per pixel
    if (launch_exact_fit(A, st) != hipSuccess) return EPIC_ERR_HIP;
    ctx->last_npairs = 0;          // no per-call statistics
    return EPIC_OK;
}

void epic_refine_defaults(epic_refine_params* p) {
    if (!p) return;
    p->lam = 0.1f;
    p->delta = 0.1f;
    p->gamma = 0.7f;
    p->kappa = 5.0f;
    p->eps = 1e-3f;
    p->zeta = 0.1f;
    p->omega = 1.6f;
    p->fixed_point = 5;
    p->sor = 30;
}

size_t epic_refine_bytes(int H, int W, int channels) {
    if (H < 1 || W < 1 || channels < 1 || channels > 4) return 0;
    const size_t HW = (size_t)H * W;
    return align_up(4 * HW * channels) + kVarPlanes * align_up(4 * HW) + kAlign;
}

int epic_refine(epic_ctx* ctx, const float* I1, const float* I2, int H, int W, int channels,
                const float* flow_in, float* flow_out, const epic_refine_params* params, void* stream) {
    if (!ctx || !I1 || !I2 || !flow_in || !flow_out) return EPIC_ERR_ARG;
    if (H < 1 || W < 1 || (long long)H * W >= (1LL << 31) || channels < 1 || channels > 4) return EPIC_ERR_ARG;
    for (const void* q : {(const void*)I1, (const void*)I2, (const void*)flow_in, (const void*)flow_out})
        if ((uintptr_t)q & 3) return EPIC_ERR_ARG;
    const long long HW = (long long)H * W;
    // the output may be the input itself, but not a shifted view of it
    const char *fi = (const char*)flow_in, *fo = (const char*)flow_out;
    if (fi != fo && fo < fi + 8 * HW && fi < fo + 8 * HW) return EPIC_ERR_ARG;
    epic_refine_params p;
    if (params) p = *params; else epic_refine_defaults(&p);
    const float fs[] = {p.lam, p.delta, p.gamma, p.kappa, p.eps, p.zeta, p.omega};
    for (float f : fs)
        if (!std::isfinite(f) || f < 0.0f) return EPIC_ERR_ARG;
    if (!(p.eps > 0.0f) || !(p.zeta > 0.0f) || !(p.omega > 0.0f) || !(p.omega < 2.0f)) return EPIC_ERR_ARG;
    if (p.fixed_point < 0 || p.fixed_point > 100 || p.sor < 0 || p.sor > 10000) return EPIC_ERR_ARG;
    // the refinement's planes sit at the end of the workspace, behind the
    // descriptor ring; the last interpolation's statistics stay readable
    // when its part of the workspace lies before them
    const size_t need = epic_refine_bytes(H, W, channels);
    if (kFixed + need > ctx->ws_bytes) return EPIC_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return EPIC_ERR_HIP;
    const size_t start = (ctx->ws_bytes - need + kAlign - 1) & ~(kAlign - 1);
    char* w = ctx->ws + start;
    VarArgs A{};
    A.I1 = I1;
    A.I2 = I2;
    A.u0 = flow_in;
    A.flow = flow_out;
    A.I2w = reinterpret_cast<float*>(w);
    w += align_up(4 * (size_t)HW * channels);
    float* planes[kVarPlanes];
    for (int k = 0; k < kVarPlanes; ++k, w += align_up(4 * (size_t)HW)) planes[k] = reinterpret_cast<float*>(w);
    A.coef = planes[0];            // 13 consecutive planes
    A.sys = planes[13];            // 9
    A.du[0] = planes[22];
    A.du[1] = planes[23];
    A.dv[0] = planes[24];
    A.dv[1] = planes[25];
    A.H = H;
    A.W = W;
    A.C = channels;
    A.HW = HW;
    A.lam = p.lam;
    A.delta = p.delta;
    A.gamma = p.gamma;
    A.kappa = p.kappa;
    A.eps = p.eps;
    A.zeta = p.zeta;
    A.omega = p.omega;
    A.fixed_point = p.fixed_point;
    A.sor = p.sor;
    if (start < ctx->last_used) ctx->last_npairs = 0;
    if (launch_variational(A, (hipStream_t)stream) != hipSuccess) return EPIC_ERR_HIP;
    return EPIC_OK;
}

struct epic_graph {
    epic_ctx* ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    PairDev* h_desc = nullptr;
    PairDev* d_desc = nullptr;
    int n = 0;
    std::vector<int*> counters;
};

void epic_graph_destroy(epic_graph* g) {
    if (!g) return;
    if (g->ctx) hipSetDevice(g->ctx->device);
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    if (g->d_desc) hipFree(g->d_desc);
    if (g->h_desc) hipHostFree(g->h_desc);
    delete g;
}

epic_graph* epic_graph_capture(epic_ctx* ctx, const epic_request* reqs, int n) {
    if (!ctx || !reqs || n < 1 || n > kMaxPairs) return nullptr;
    if (hipSetDevice(ctx->device) != hipSuccess) return nullptr;
    epic_graph* g = new epic_graph();
    g->ctx = ctx;
    g->n = n;
    hipStream_t s = nullptr;
    bool ok = hipHostMalloc((void**)&g->h_desc, sizeof(PairDev) * n, hipHostMallocDefault) == hipSuccess &&
              hipMalloc((void**)&g->d_desc, sizeof(PairDev) * n) == hipSuccess &&
              hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    if (ok) ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        DescTarget tgt{g->h_desc, g->d_desc};
        const int rc = run_pairs(ctx, reqs, n, s, nullptr, &tgt);
        const hipError_t e = hipStreamEndCapture(s, &g->graph);
        ok = rc == EPIC_OK && e == hipSuccess && g->graph;
    }
    if (ok) ok = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) == hipSuccess;
    if (s) hipStreamDestroy(s);
    if (!ok) {
        epic_graph_destroy(g);
        return nullptr;
    }
    g->counters.assign(ctx->last_counters, ctx->last_counters + n);
    return g;
}

int epic_graph_launch(epic_graph* g, void* stream) {
    if (!g || !g->exec) return EPIC_ERR_ARG;
    epic_ctx* c = g->ctx;
    if (hipSetDevice(c->device) != hipSuccess) return EPIC_ERR_HIP;
    if (hipGraphLaunch(g->exec, (hipStream_t)stream) != hipSuccess) return EPIC_ERR_HIP;
    std::copy(g->counters.begin(), g->counters.end(), c->last_counters);
    c->last_npairs = g->n;
    c->last_stream = (hipStream_t)stream;
    return EPIC_OK;
}

int epic_profile(epic_ctx* ctx, int enable) {
    if (!ctx) return EPIC_ERR_ARG;
    ctx->prof = enable != 0;
    if (!ctx->prof) {
        ctx->prof_count = 0;
        for (int r = 0; r < kProfRing; ++r) ctx->prof_ok[r] = false;
    }
    return EPIC_OK;
}

int epic_stage_times(epic_ctx* ctx, float* ms, int n_stages, int calls) {
    if (!ctx || !ms || n_stages < 1 || calls < 1) return EPIC_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return EPIC_ERR_HIP;
    const int n = std::min(n_stages, kStages);
    const int use = std::min(calls, ctx->prof_count);
    for (int i = 0; i < n; ++i) ms[i] = 0.0f;
    if (use == 0) return n;
    int got = 0;
    for (int k = 1; k <= kProfRing && got < use; ++k) {
        const int r = (ctx->prof_next - k + kProfRing) % kProfRing;
        if (!ctx->prof_ok[r]) continue;
        if (hipEventSynchronize(ctx->prof_ev[r][kStages]) != hipSuccess) return EPIC_ERR_HIP;
        for (int i = 0; i < n; ++i) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, ctx->prof_ev[r][i], ctx->prof_ev[r][i + 1]) != hipSuccess)
                return EPIC_ERR_HIP;
            ms[i] += t;
        }
        ++got;
    }
    for (int i = 0; i < n; ++i) ms[i] /= (float)got;
    return n;
}

const char* epic_stage_name(int i) { return (i >= 0 && i < kStages) ? kStageNames[i] : ""; }

int epic_pass_visits(epic_ctx* ctx, int* visits, int n) {
    if (!ctx || !visits || n < 1) return EPIC_ERR_ARG;
    const int m = std::min(n, kMaxPasses);
    for (int i = 0; i < m; ++i) visits[i] = 0;
    if (!ctx->last_pass_visits) return 0;
    if (hipSetDevice(ctx->device) != hipSuccess) return EPIC_ERR_HIP;
    if (hipStreamSynchronize(ctx->last_stream) != hipSuccess) return EPIC_ERR_HIP;
    if (hipMemcpy(visits, ctx->g_any + 2 * kMaxPasses, sizeof(int) * m, hipMemcpyDeviceToHost) != hipSuccess)
        return EPIC_ERR_HIP;
    int used = 0;
    for (int i = 0; i < m; ++i)
        if (visits[i] > 0) used = i + 1;
    return used;
}

int epic_get_stats(epic_ctx* ctx, int pair, epic_stats* out) {
    if (!ctx || !out || pair < 0 || pair >= ctx->last_npairs) return EPIC_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return EPIC_ERR_HIP;
    if (hipStreamSynchronize(ctx->last_stream) != hipSuccess) return EPIC_ERR_HIP;
    int cnt[C_NCOUNTERS];
    int gerr = 0;
    if (hipMemcpy(cnt, ctx->last_counters[pair], sizeof(cnt), hipMemcpyDeviceToHost) != hipSuccess)
        return EPIC_ERR_HIP;
    if (hipMemcpy(&gerr, ctx->g_error, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return EPIC_ERR_HIP;
    out->status = cnt[C_STATUS];
    if (ctx->last_pruned && out->status == 0) out->status = cnt[C_STATUS0];
    // found after the CSR scan wrote the status: a K-NN visited set that
    // outgrew even the retry's table (that match's model is zero), or the
    // transform finisher's pass bound
    if ((cnt[C_OVERFLOW] & 2) && out->status == 0) out->status = EPIC_ERR_CAPACITY;
    if ((gerr & 1) && out->status == 0) out->status = EPIC_ERR_CONVERGENCE;
    if (cnt[C_INVARIANT] && out->status == 0) out->status = EPIC_ERR_INVARIANT;
    out->n_used = cnt[C_USED];
    // with the consistency check, drops are those of the original matches
    out->n_outside = ctx->last_pruned ? cnt[C_OUTSIDE0] : cnt[C_OUTSIDE];
    out->n_duplicate = ctx->last_pruned ? cnt[C_DUP0] : cnt[C_DUPLICATE];
    out->n_pruned = ctx->last_pruned ? cnt[C_PRUNED] : 0;
    out->n_edges = cnt[C_EDGES];
    out->n_degenerate = cnt[C_DEGENERATE];
    out->n_fp64_fits = cnt[C_FP64];
    out->tile_visits = cnt[C_TILE_VISITS];
    out->n_bad_cost = cnt[C_BADCOST];
    out->n_invariant = cnt[C_INVARIANT];
    return EPIC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free entry point.  Its workspace is a device array of the
// library, one copy per GPU for the life of the process; its host state is a
// static context per device; descriptors travel in the first kernel's
// arguments; the pass budget is fixed (the transform's finisher completes
// any remainder, so results are those of epic_interp).
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = 64ull << 20;     // 64 MiB per GPU
constexpr int kNoAllocPasses = 8;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

struct NoAllocState {
    std::once_flag once;
    int init_status = EPIC_ERR_HIP;
    char* ptr = nullptr;          // this device's copy of `scratch`
    epic_ctx ctx;                 // host state (no pinned memory, no events)
};
NoAllocState g_noalloc[kMaxDevices];

}  // namespace

extern "C" int epic_interp_noalloc(const float* cost, int H, int W, const float* matches, int N, int K,
                                   float a, int mode, float* flow, void* stream) {
    const int v = epic_validate(cost, H, W, matches, N, K, a, mode, flow);
    if (v != EPIC_OK) return v;
    // sizes beyond the array are refused before any device call
    if (epic_workspace_bytes(H, W, N, K, mode, 0) > kScratchBytes) return EPIC_ERR_WORKSPACE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return EPIC_ERR_HIP;
    NoAllocState& st = g_noalloc[dev];
    std::call_once(st.once, [&] {
        // the array's name is a host-side stand-in: its device address comes
        // from the runtime, once per device, with that device current
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return;
        st.ptr = static_cast<char*>(p);
        epic_ctx& c = st.ctx;
        c.device = dev;
        c.opt.connectivity = 8;
        c.opt.la_weight_power = 2;
        c.opt.precision = 0;
        c.opt.fp64_route = 1e-3f;
        c.opt.degenerate_tau = 1e-9;
        c.opt.tile_w = 32;
        c.opt.tile_h = 16;
        c.opt.geo_passes = kNoAllocPasses;
        c.auto_passes = false;
        c.passes = kNoAllocPasses;
        c.ws = st.ptr;
        c.ws_bytes = kScratchBytes;
        c.g_error = reinterpret_cast<int*>(st.ptr);
        c.g_any = reinterpret_cast<int*>(st.ptr) + 256;
        st.init_status = EPIC_OK;
    });
    if (st.init_status != EPIC_OK) return st.init_status;
    PairDev host_desc[1];
    DescTarget tgt{host_desc, reinterpret_cast<PairDev*>(st.ptr + 4096)};
    epic_request r{cost, H, W, matches, N, K, a, mode, flow};
    return run_pairs(&st.ctx, &r, 1, (hipStream_t)stream, nullptr, &tgt);
}
