// Host orchestrator and C-ABI of the S^5 library (declared in include/s5.h).
//
// One call runs the recursion of string sample sort (Section 3.1) level by
// level: every pass distributes all segments larger than the base threshold
// at once; the device plans the next pass (appending work items with atomic
// counters) and the host reads back one small counter block per pass to size
// the next launches.  Buckets at or below the base threshold collect in one
// list that the LDS base-case sorter finishes after the last pass, and a final
// kernel completes the LCPs at bucket boundaries.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/s5.h"
#include "../../include/s5_profile.h"
#include "../../include/s5_learned.h"
#include "../../include/s5_debug.h"
#include "s5_internal.h"

#include "s5_launch.h"

using namespace s5;

namespace {

// learned splitters: samples per segment, Adam steps and learning rate
constexpr uint32_t kLearnSamples = kLearnM, kLearnSteps = 64;
constexpr float kLearnRate = 0.03f;

struct Cfg {
    uint32_t dmax, alpha, unroll, tile_min, T, mode, classifier;
    uint32_t alphabet;  // S5_ALPHABET_*
    uint32_t b;         // bits per character of this sort's keys (8: bytes; set per call)
    uint32_t T_caps, tile_caps;  // smallest T and tile of any set: storage capacities
    float beta;
    uint32_t graph_levels;
    uint32_t distribution;  // S5_DISTRIBUTE_*
    uint64_t seed;
};

// distribution levels a batched sort captures in its graph by default
constexpr uint32_t kGraphLevels = 12, kGraphLevelsMax = 64;

int resolve_cfg(const s5_config* c, Cfg* o) {
    memset(o, 0, sizeof *o);  // Cfg is compared byte-wise as part of graph keys
    s5_config z;
    memset(&z, 0, sizeof z);
    if (!c) c = &z;
    uint32_t v = c->splitters ? c->splitters : 255u;
    uint32_t d = 0;
    while (((1u << (d + 1)) - 1) <= v && d < 31) ++d;  // largest d with 2^d - 1 <= v
    if (v < 7 || v > 1023 || ((1u << d) - 1) != v) return S5_ERR_INVALID;
    o->dmax = d;
    o->alpha = c->oversample ? c->oversample : 2u;
    if (o->alpha < 1 || o->alpha > 4) return S5_ERR_INVALID;
    o->unroll = c->unroll ? c->unroll : 4u;
    if (o->unroll != 1 && o->unroll != 2 && o->unroll != 4 && o->unroll != 8) return S5_ERR_INVALID;
    o->tile_min = c->tile ? c->tile : 2048u;
    if (o->tile_min % 64 || o->tile_min > (1u << 20)) return S5_ERR_INVALID;
    o->T = c->base_threshold ? c->base_threshold : 1024u;
    if (o->T < 64 || o->T > 2048) return S5_ERR_INVALID;
    o->T_caps = o->T;
    o->tile_caps = o->tile_min;
    o->mode = c->splitter_mode;
    if (o->mode != S5_SPLIT_SAMPLED && o->mode != S5_SPLIT_LEARNED) return S5_ERR_INVALID;
    o->beta = c->imbalance_bound > 0 ? c->imbalance_bound : 4.0f;
    o->graph_levels = c->graph_levels ? c->graph_levels : kGraphLevels;
    if (o->graph_levels > kGraphLevelsMax) return S5_ERR_INVALID;
    o->seed = c->seed;
    o->classifier = c->classifier;
    o->alphabet = c->alphabet;
    o->b = 8;
    if (o->alphabet != S5_ALPHABET_BYTES && o->alphabet != S5_ALPHABET_AUTO) return S5_ERR_INVALID;
    o->distribution = c->distribution;
    if (o->distribution != S5_DISTRIBUTE_ONE_PASS && o->distribution != S5_DISTRIBUTE_TWO_PASS)
        return S5_ERR_INVALID;
    if (o->classifier != S5_CLASSIFY_UNROLL && o->classifier != S5_CLASSIFY_EQUAL &&
        o->classifier != S5_CLASSIFY_JUMP)
        return S5_ERR_INVALID;
    return S5_OK;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// test-only limits of device capacities (0 = none), s5_debug_limit_capacity
uint32_t g_cap_limit[5];

uint32_t limited(uint32_t cap, uint32_t which) {
    return g_cap_limit[which] ? std::min(cap, g_cap_limit[which]) : cap;
}

// Workspace regions (byte offsets into one device allocation).
struct Layout {
    size_t key[2], key2[2], key3, idx[2], bid, bid2, lseg[2], tile_tab, chunk_tab, tree_lo, tree_in, tree_lcp, jump, cm, cs,
        bstart, base_list, learn, learn_seg, set_tune, code_tab, alpha_bits, counters[2], glob,
        total;
    uint32_t learn_cap, tune_sets;
    bool has_jump;
    Caps caps;
};

Layout make_layout(uint64_t n, const Cfg& c, uint32_t tune_sets) {
    Layout L;
    const uint64_t kmax = (2ull << c.dmax) - 1;
    Caps cp;
    uint64_t large = n / (c.T_caps + 1) + 2;
    // tiles of a segment: ceil(|S| / tile_len) with tile_len >= tile_min
    uint64_t tiles = n / c.tile_caps + large + 1;
    uint64_t chunks = tiles / kChunkRows + large + 1;
    // sum over segments of 2^d < 4 |S| / T (plus the d >= 1 floor)
    uint64_t tree = 4 * n / c.T_caps + 2 * large + 2;
    cp.large = (uint32_t)large;
    cp.tiles = (uint32_t)std::min<uint64_t>(tiles, 0xFFFFFFFFull);
    cp.chunks = (uint32_t)chunks;
    cp.tree = (uint32_t)tree;
    cp.bstart = (uint32_t)(2 * tree + large + 2);
    // every base item holds >= 2 strings, and > 64 / > 512 in the larger classes
    cp.base[0] = (uint32_t)(n / 2 + 2);
    cp.base[1] = (uint32_t)(n / (kBaseWave + 1) + 2);
    cp.base[2] = (uint32_t)(n / (kBaseSmall + 1) + 2);
    cp.base[3] = (uint32_t)(n / (kBaseMid + 1) + 2);
    cp.large = limited(cp.large, S5_CAP_LARGE);
    for (int q = 0; q < kBaseClasses; ++q) cp.base[q] = limited(cp.base[q], S5_CAP_BASE0 + q);
    // sum over segments of tiles x k: tiles_s <= |S|/tile_min + 1 and
    // k_s <= max(3, min(kmax, 8 |S| / T))
    const uint64_t ksum = 3 * large + 8 * n / c.T_caps + kmax;
    cp.cm = (unsigned long long)(kmax * (n / c.tile_caps + 1) + 4 * ksum);
    cp.cs = (unsigned long long)(cp.cm / kChunkRows + ksum);
    size_t p = 0;
    auto take = [&](size_t bytes) {
        size_t o = p;
        p = align_up(p + bytes);
        return o;
    };
    for (int b = 0; b < 2; ++b) L.key[b] = take(n * 8);
    for (int b = 0; b < 2; ++b) L.key2[b] = take(n * 8);
    L.key3 = take(n * 8);
    for (int b = 0; b < 2; ++b) L.idx[b] = take(n * 4);
    L.bid = take(n * 2);
    // two-pass distribution: the bucket ids travel with the first move
    L.bid2 = take(c.distribution == S5_DISTRIBUTE_TWO_PASS ? n * 2 : 0);
    for (int b = 0; b < 2; ++b) L.lseg[b] = take((size_t)cp.large * sizeof(LSeg));
    L.tile_tab = take((size_t)cp.tiles * 4);
    L.chunk_tab = take((size_t)cp.chunks * 4);
    L.tree_lo = take((size_t)cp.tree * 8);
    L.tree_in = take((size_t)cp.tree * 8);
    L.tree_lcp = take((size_t)cp.tree);
    // jump tables (Jump classification only): kJumpPerTreeSlot entries per tree slot
    L.has_jump = c.classifier == S5_CLASSIFY_JUMP;
    L.jump = take(L.has_jump ? (size_t)cp.tree * kJumpPerTreeSlot * 2 : 0);
    L.cm = take((size_t)cp.cm * 4);
    L.cs = take((size_t)cp.cs * 4);
    L.bstart = take((size_t)cp.bstart * 4);
    size_t base_items = 0;
    for (int q = 0; q < kBaseClasses; ++q) base_items += cp.base[q];
    L.base_list = take(base_items * sizeof(Seg));
    // learned splitters: one slot per segment of >= kLearnMin strings in a pass
    L.learn_cap = c.mode == S5_SPLIT_LEARNED ? (uint32_t)std::min<uint64_t>(large, n / kLearnMin + 1) : 0u;
    L.learn = take(learn_bytes(L.learn_cap, kLearnSamples));
    L.learn_seg = take((size_t)L.learn_cap * 4);
    // packed per-set parameters of a tuned batched sort
    L.tune_sets = tune_sets;
    L.set_tune = take((size_t)tune_sets * 4);
    // alphabet compression: byte -> code table and the sampled byte bitmap
    L.code_tab = take(256);
    L.alpha_bits = take(32);
    // [counters 0 | globals | counters 1] back to back: one copy reads a pass's
    // counters together with the globals
    L.counters[0] = take(sizeof(Counters) + sizeof(Globals) + sizeof(Counters));
    L.glob = L.counters[0] + sizeof(Counters);
    L.counters[1] = L.glob + sizeof(Globals);
    L.total = p;
    L.caps = cp;
    return L;
}

struct DevPool {
    void* ptr = nullptr;
    size_t bytes = 0;
    void* host = nullptr;  // pinned readback block
};

std::mutex g_mu;
std::unordered_map<int, DevPool> g_pools;
struct StreamRecord {
    s5_stats stats;
    int status;
    uint64_t seq;  // order of the sorts that wrote the records
};
std::unordered_map<hipStream_t, StreamRecord> g_last;
uint64_t g_seq = 0;

#define S5_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return S5_ERR_HIP;       \
    } while (0)

void graphs_release();

// Pinned readback block of a device: [raw copy | counters | globals], one slot each.
constexpr size_t kHostSlot = 4096;
static_assert(2 * sizeof(Counters) + sizeof(Globals) <= kHostSlot, "readback slot too small");
// the word of the raw slot that a publish kernel raises once the counters are in
constexpr size_t kFlagOff = kHostSlot - 64;
static_assert(sizeof(Counters) + sizeof(Globals) <= kFlagOff, "readback slot layout");
static_assert((sizeof(Counters) + sizeof(Globals)) % 4 == 0 &&
                  sizeof(Counters) + sizeof(Globals) <= 4096,
              "counters are published in at most 1024 words");

// Get the pool of the current device with at least `bytes`.
int pool_get(size_t bytes, DevPool** out) {
    int dev = 0;
    S5_HIP(hipGetDevice(&dev));
    DevPool& P = g_pools[dev];
    if (!P.host) S5_HIP(hipHostMalloc(&P.host, 3 * kHostSlot, hipHostMallocDefault));
    if (P.bytes < bytes) {
        if (P.ptr) {
            S5_HIP(hipDeviceSynchronize());
            graphs_release();  // captured graphs point into the old pool
            S5_HIP(hipFree(P.ptr));
            P.ptr = nullptr;
            P.bytes = 0;
        }
        if (hipMalloc(&P.ptr, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return S5_ERR_NOMEM;
        }
        P.bytes = bytes;
    }
    *out = &P;
    return S5_OK;
}


// ---- per-kernel event timing (s5_profile.h) --------------------------------
enum KId { K_INIT, K_ROOTS, K_SAMPLE, K_CLASSIFY, K_COLSCAN, K_PLAN, K_SCATTER, K_BASE, K_LCPFIX,
           K_LEARN, K_GRAPH, K_DIGITS, K_COUNT };
const char* const kKName[K_COUNT] = {"init_keys", "plan_roots",      "sample_tree", "classify",
                                     "colscan",   "bucket_plan",     "scatter",     "base_sort",
                                     "lcp_fix",   "learn_splitters", "sort_graph",  "digit_counts"};
// algorithmic bytes per string processed: init reads an offset and 8 key bytes
// and writes key + index; classify reads a key and writes a bucket id; a
// redistribution pass reads and writes (key, index); the base case reads
// (key, index) and writes perm + lcp; the LCP completion reads one lcp word
// (the two-pass distribution's digit counts read a bucket id)
const double kKBytes[K_COUNT] = {28, 0, 0, 10, 0, 0, 24, 20, 4, 0, 0, 2};
struct ProfAcc {
    uint64_t launches = 0, items = 0;
    double ms = 0, bytes = 0;
};
struct Pending {
    int k;
    hipEvent_t a, b;
    uint64_t items;
};
bool g_prof_on = false;
thread_local bool t_quiet = false;  // no events (the sort without allocations)
int g_prof_only = -1;  // time only this kernel (-1: all)
ProfAcc g_prof[K_COUNT];
std::vector<hipEvent_t> g_event_pool;
std::vector<Pending> g_pending;

hipEvent_t prof_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch `fn` on `st`, bracketed by events when profiling is on.
template <class F>
void timed(int k, uint64_t items, hipStream_t st, F&& fn) {
    if (!g_prof_on || t_quiet || (g_prof_only >= 0 && k != g_prof_only)) {
        fn();
        return;
    }
    hipEvent_t a = prof_event(), b = prof_event();
    if (a) (void)hipEventRecord(a, st);
    fn();
    if (b) (void)hipEventRecord(b, st);
    if (a && b) g_pending.push_back({k, a, b, items});
}

// Same for a launcher that takes the two events itself and lets the kernel's
// dispatch stamp them (their interval is the one kernel's execution).
template <class F>
void timed_dispatch(int k, uint64_t items, hipStream_t st, F&& fn) {
    if (!g_prof_on || t_quiet || (g_prof_only >= 0 && k != g_prof_only)) {
        fn(nullptr, nullptr);
        return;
    }
    (void)st;
    hipEvent_t a = prof_event(), b = prof_event();
    if (!a || !b) {
        fn(nullptr, nullptr);
        if (a) g_event_pool.push_back(a);
        if (b) g_event_pool.push_back(b);
        return;
    }
    fn(a, b);
    g_pending.push_back({k, a, b, items});
}

// Fold pending events into totals (each waited for first: a sort's last
// readback need not wait for its whole stream).
void prof_collect() {
    for (auto& p : g_pending) (void)hipEventSynchronize(p.b);
    for (auto& p : g_pending) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            ProfAcc& A = g_prof[p.k];
            A.launches += 1;
            A.items += p.items;
            A.ms += ms;
            A.bytes += kKBytes[p.k] * (double)p.items;
        }
        g_event_pool.push_back(p.a);
        g_event_pool.push_back(p.b);
    }
    g_pending.clear();
}

struct SortArgs {
    const uint8_t* chars;
    uint64_t chars_len;  // 0 = unknown (no device-side argument checks)
    const uint64_t* offsets;
    const uint64_t* set_begin;  // device, or null for a single set
    uint32_t num_sets, n;
    uint32_t* perm;
    uint32_t* lcp;
    const uint32_t* tune_host;  // packed per-set parameters (host), or null
};

// Device views of one workspace.
struct Ptrs {
    uint64_t* key[2];
    uint64_t* key2[2];  // the 8 bytes after key, or kKeyUnknown
    uint64_t* key3;     // the 8 bytes after those, for the first pass only
    uint32_t* idx[2];
    uint16_t* bid;
    uint16_t* bid2;
    LSeg* lseg[2];
    uint32_t *tile_tab, *chunk_tab;
    uint64_t *tree_lo, *tree_in;
    uint8_t* tree_lcp;
    uint16_t* jump;  // jump tables, or null when the classification does not use them
    uint32_t *cm, *cs, *bstart, *learn_seg, *set_tune;
    uint8_t* code_tab;
    uint32_t* alpha_bits;
    LearnCtx lctx;
    Seg* base_list[kBaseClasses];
    Counters* cnt[2];
    Globals* glob;
};

Ptrs make_ptrs(const Layout& L, char* W) {
    Ptrs P;
    for (int b = 0; b < 2; ++b) {
        P.key[b] = (uint64_t*)(W + L.key[b]);
        P.key2[b] = (uint64_t*)(W + L.key2[b]);
        P.key3 = (uint64_t*)(W + L.key3);
        P.idx[b] = (uint32_t*)(W + L.idx[b]);
        P.lseg[b] = (LSeg*)(W + L.lseg[b]);
        P.cnt[b] = (Counters*)(W + L.counters[b]);
    }
    P.bid = (uint16_t*)(W + L.bid);
    P.bid2 = (uint16_t*)(W + L.bid2);
    P.tile_tab = (uint32_t*)(W + L.tile_tab);
    P.chunk_tab = (uint32_t*)(W + L.chunk_tab);
    P.tree_lo = (uint64_t*)(W + L.tree_lo);
    P.tree_in = (uint64_t*)(W + L.tree_in);
    P.tree_lcp = (uint8_t*)(W + L.tree_lcp);
    P.jump = L.has_jump ? (uint16_t*)(W + L.jump) : nullptr;
    P.cm = (uint32_t*)(W + L.cm);
    P.cs = (uint32_t*)(W + L.cs);
    P.bstart = (uint32_t*)(W + L.bstart);
    P.learn_seg = (uint32_t*)(W + L.learn_seg);
    P.set_tune = L.tune_sets ? (uint32_t*)(W + L.set_tune) : nullptr;
    P.code_tab = (uint8_t*)(W + L.code_tab);
    P.alpha_bits = (uint32_t*)(W + L.alpha_bits);
    P.lctx = learn_ctx(W + L.learn, L.learn_cap, kLearnSamples);
    P.base_list[0] = (Seg*)(W + L.base_list);
    for (int q = 1; q < kBaseClasses; ++q) P.base_list[q] = P.base_list[q - 1] + L.caps.base[q - 1];
    P.glob = (Globals*)(W + L.glob);
    return P;
}

// The key codec of a sort: bytes, or packed codes of c.b bits (the table is
// in the workspace; a byte outside the alphabet sets the status word).
KeyCodec codec_of(const Cfg& c, const Ptrs& P) {
    return make_codec(c.b, P.code_tab, &P.glob->status);
}

PlanCtx plan_ctx(const Ptrs& P, const Layout& L, const Cfg& c, const SortArgs& a, int next) {
    PlanCtx x;
    x.set_begin = a.set_begin;
    x.set_tune = P.set_tune;
    x.num_sets = a.num_sets;
    x.lseg = P.lseg[next];
    x.cnt = P.cnt[next];
    for (int q = 0; q < kBaseClasses; ++q) x.base_list[q] = P.base_list[q];
    x.glob = P.glob;
    x.caps = L.caps;
    x.T = c.T;
    x.d_max = c.dmax;
    x.tile_min = c.tile_min;
    x.learn = c.mode == S5_SPLIT_LEARNED ? 1u : 0u;
    x.learn_cap = L.learn_cap;
    x.learn_seg = P.learn_seg;
    x.stats = 0;
    x.kc = codec_of(c, P);
    return x;
}

// Launch shapes of one pass: the host-read counters (host-driven) or the
// capacities and fixed grids (graph mode).
struct PassShape {
    Counters now;                // host-driven: this pass's counters
    uint32_t vmax, kmax;
    Dyn seg, tile, chunk, learn;  // graph mode: device counts
    uint32_t n_learn;            // host-driven: learned segments
};

Dyn dyn_of(const uint32_t* cnt, uint32_t cap, uint32_t gmax) {
    Dyn d;
    d.cnt = cnt;
    d.cap = cap;
    d.grid = std::max<uint32_t>(1u, std::min(cap, gmax));
    return d;
}

// Fixed grids of graph-mode launches (grid-stride over the device counts).
constexpr uint32_t kGraphSegGrid = 4096, kGraphTileGrid = 4096, kGraphLearnGrid = 512,
                   kGraphBaseGrid = 8192;

PassShape graph_shape(const Ptrs& P, const Layout& L, const Cfg& c, int cur) {
    PassShape S;
    memset(&S.now, 0, sizeof S.now);
    S.vmax = (1u << c.dmax) - 1;
    S.kmax = 2 * S.vmax + 1;
    S.seg = dyn_of(&P.cnt[cur]->n_large, L.caps.large, kGraphSegGrid);
    S.tile = dyn_of(&P.cnt[cur]->tiles, L.caps.tiles, kGraphTileGrid);
    S.chunk = dyn_of(&P.cnt[cur]->chunks, L.caps.chunks, kGraphTileGrid);
    S.learn = dyn_of(&P.cnt[cur]->pad0, L.learn_cap, kGraphLearnGrid);
    S.n_learn = 0;
    return S;
}

PassShape host_shape(const Counters& now, const Layout& L) {
    PassShape S;
    S.now = now;
    S.kmax = now.kmax;
    S.vmax = (now.kmax - 1) / 2;
    S.n_learn = std::min(now.pad0, L.learn_cap);
    return S;
}

// Learned proposals (a proposal that fails on its own sample is switched back
// to sampled splitters), sampled trees, classification and column scans.
// redo = 1: the same for the segments the exact learned check rejected.
void pass_front(const SortArgs& a, const Cfg& c, const Layout& L, const Ptrs& P,
                const PassShape& S, int cur, int buf, uint32_t redo, hipStream_t st) {
    const bool graph = S.seg.cnt != nullptr;
    const int nxt = cur ^ 1;
    if (!redo && c.mode == S5_SPLIT_LEARNED && (graph || S.n_learn)) {
        timed(K_LEARN, S.n_learn, st, [&] {
            launch_learn_sort_trees(P.lctx, S.n_learn, P.lseg[cur], P.learn_seg, P.key[buf],
                                    c.seed, kLearnSteps, kLearnRate, c.beta, P.glob, P.tree_lo,
                                    P.tree_in, P.tree_lcp, P.jump, codec_of(c, P), S.learn, st);
        });
    }
    timed(K_SAMPLE, S.now.n_large, st, [&] {
        launch_sample_tree(S.now.n_large, P.lseg[cur], P.key[buf], c.alpha, S.vmax, c.seed,
                           P.tree_lo, P.tree_in, P.tree_lcp, P.jump, P.tile_tab, P.chunk_tab,
                           P.cnt[nxt], P.glob, S.seg, redo, codec_of(c, P), st);
    });
    timed(K_CLASSIFY, S.now.moved, st, [&] {
        launch_classify(S.now.tiles, c.unroll, c.classifier, P.lseg[cur], P.tile_tab, P.key[buf],
                        P.tree_lo, P.tree_in, P.jump, P.bid, P.cm, S.vmax, S.kmax, P.glob, S.tile,
                        redo, st);
    });
    timed(K_COLSCAN, S.now.moved, st, [&] {
        launch_colscan(S.now.chunks, S.kmax, P.lseg[cur], P.chunk_tab, P.cm, P.cs, P.glob,
                       S.chunk, redo, st);
    });
    (void)a;
    (void)L;
}

// Bucket plan of the next pass.
void pass_plan(const SortArgs& a, const Cfg& c, const Layout& L, const Ptrs& P,
               const PassShape& S, int cur, int buf, uint32_t level, hipStream_t st) {
    const int nxt = cur ^ 1;
    PlanCtx x = plan_ctx(P, L, c, a, nxt);
    x.stats = level == 0 ? 1u : 0u;  // the statistics report the first pass only
    timed(K_PLAN, S.now.moved, st, [&] {
        // the buffer the level leaves its strings in
        const int out = c.distribution == S5_DISTRIBUTE_TWO_PASS ? buf : buf ^ 1;
        launch_bucket_plan(S.now.n_large, P.lseg[cur], P.cs, P.bstart, P.tree_in, P.tree_lcp, x,
                           (uint32_t)out, S.kmax, S.seg, st);
    });
}

// The redistribution of the pass: one move from buffer `buf` into the other,
// or (two-pass distribution) a move by the low digit of the bucket ids into
// the other buffer and one by the high digit back into `buf`.  Each move
// first counts its digit per tile, scans the columns and adds the digits'
// starts (the bucket count matrix is used up by the plan by then).
void pass_scatter(const SortArgs& a, const Cfg& c, const Ptrs& P, const PassShape& S, int cur,
                  int buf, uint32_t level, hipStream_t st) {
    const bool two = c.distribution == S5_DISTRIBUTE_TWO_PASS;
    for (uint32_t dig = two ? kDigitLow : 0u; dig <= (two ? kDigitHigh : 0u); ++dig) {
        const int from = dig == kDigitHigh ? buf ^ 1 : buf, to = dig == kDigitHigh ? buf : buf ^ 1;
        const uint16_t* bid = dig == kDigitHigh ? P.bid2 : P.bid;
        if (dig) {
            timed(K_DIGITS, S.now.moved, st, [&] {
                launch_digit_count(S.now.tiles, P.lseg[cur], P.tile_tab, bid, P.cm, dig, st);
                launch_colscan(S.now.chunks, S.kmax, P.lseg[cur], P.chunk_tab, P.cm, P.cs, P.glob,
                               S.chunk, 0u, st, dig);
                launch_digit_starts(S.now.n_large, P.lseg[cur], P.cs, dig, st);
            });
        }
        timed_dispatch(K_SCATTER, S.now.moved, st, [&](hipEvent_t e0, hipEvent_t e1) {
            launch_scatter(S.now.tiles, c.unroll, P.lseg[cur], P.tile_tab, bid, P.key[from],
                           P.key2[from], P.idx[from], P.key[to], P.key2[to], P.idx[to], P.cm,
                           P.cs, P.bstart, P.tree_in, P.tree_lcp, a.chars, a.offsets, a.perm,
                           a.lcp, S.vmax, S.kmax, P.glob, S.tile,
                           level == 0 && dig != kDigitHigh ? P.key3 : nullptr, codec_of(c, P),
                           st, e0, e1, dig, dig == kDigitLow ? P.bid2 : nullptr);
        });
    }
}

// Bucket plan of the next pass, then the redistribution.
void pass_back(const SortArgs& a, const Cfg& c, const Layout& L, const Ptrs& P,
               const PassShape& S, int cur, int buf, uint32_t level, hipStream_t st) {
    pass_plan(a, c, L, P, S, cur, buf, level, st);
    pass_scatter(a, c, P, S, cur, buf, level, st);
}

void clear_counters(const Ptrs& P, hipStream_t st) {
    launch_zero_words(P.cnt[0], 2 * sizeof(Counters) + sizeof(Globals), st);
}

void start_sort(const SortArgs& a, const Cfg& c, const Layout& L, const Ptrs& P, hipStream_t st) {
    clear_counters(P, st);
    timed(K_INIT, a.n, st, [&] {
        launch_init_keys(a.chars, a.chars_len, a.offsets, a.n, P.key[0], P.key2[0], P.key3,
                         P.idx[0], P.glob, codec_of(c, P), st);
    });
    timed(K_ROOTS, a.num_sets, st, [&] {
        launch_plan_roots(a.set_begin, a.num_sets, a.n, a.perm, a.lcp, plan_ctx(P, L, c, a, 0), st);
    });
}

// Host-side state of a sort in progress (pinned readback block).
struct HostView {
    void* host;
    Counters* hc;
    Globals* hg;
    char* dev;  // the block's device address: counters are published into it (null: copied)
};

// Device addresses of the pinned readback blocks, looked up once per block
// (the caller holds g_mu; s5_release clears them with the pools).
std::unordered_map<void*, char*> g_host_dev;

// `mapped`: the block is pinned host memory that kernels can write.
HostView host_view(void* host, bool mapped) {
    HostView v{host, (Counters*)((char*)host + kHostSlot), (Globals*)((char*)host + 2 * kHostSlot),
               nullptr};
    if (!mapped) return v;
    auto it = g_host_dev.find(host);
    if (it != g_host_dev.end()) {
        v.dev = it->second;
        return v;
    }
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, host, 0) == hipSuccess && d) {
        v.dev = (char*)d;
        g_host_dev[host] = v.dev;
    } else {
        (void)hipGetLastError();
    }
    return v;
}

// Return code of a device status word: argument checks first.
// internal: a packed sort met a byte outside its alphabet; sort again with bytes
constexpr int kRetryBytes = -100;

int status_rc(uint32_t status) {
    if (status & kErrArgs) return S5_ERR_INVALID;
    if (status & ~kErrAlphabet) return S5_ERR_DEVICE;
    return status ? kRetryBytes : S5_OK;
}

// Alphabet compression (appendix A): with S5_ALPHABET_AUTO the bytes of a
// sample of the strings are the alphabet; with sigma' <= 7 byte values the
// sort packs order-preserving 3-bit codes, 21 characters per key (code 0 the
// terminator, 1..sigma' the alphabet's bytes in byte order, 0xFF a byte
// outside it) and c.b = 3, else c.b stays 8 (byte keys).
constexpr size_t kAlphaSlot = 3072;  // bitmap readback, inside the raw slot
static_assert(sizeof(Counters) + sizeof(Globals) <= kAlphaSlot, "readback slot layout");

int choose_alphabet(const SortArgs& a, Cfg& c, const Ptrs& P, void* host, hipStream_t st) {
    c.b = 8;
    if (c.alphabet != S5_ALPHABET_AUTO || a.n == 0) return S5_OK;
    const uint32_t samples = std::min<uint32_t>(a.n, 65536u);
    launch_alphabet(a.chars, a.chars_len, a.offsets, a.n, samples, P.alpha_bits, st);
    uint32_t* hb = (uint32_t*)((char*)host + kAlphaSlot);
    S5_HIP(hipMemcpyAsync(hb, P.alpha_bits, 32, hipMemcpyDeviceToHost, st));
    S5_HIP(hipStreamSynchronize(st));
    uint8_t tab[256];
    uint32_t sigma = 0;
    for (uint32_t ch = 0; ch < 256; ++ch) {
        const bool in = ch != 0 && ((hb[ch >> 5] >> (ch & 31)) & 1u);
        tab[ch] = ch == 0 ? 0 : (in ? (uint8_t)(++sigma) : (uint8_t)0xFF);
    }
    if (sigma > 7) return S5_OK;  // byte keys
    S5_HIP(hipMemcpyAsync(P.code_tab, tab, 256, hipMemcpyHostToDevice, st));
    S5_HIP(hipStreamSynchronize(st));  // `tab` lives on this stack
    c.b = kPackBits;
    return S5_OK;
}

// A pass's counters together with the globals (they lie next to each other).
const char* readback_src(const Ptrs& P, int which) {
    return which == 0 ? (const char*)P.cnt[0] : (const char*)P.glob;
}

// Copy them into the host block.
int readback_start(const Ptrs& P, const HostView& H, int which, hipStream_t st) {
    S5_HIP(hipMemcpyAsync(H.host, readback_src(P, which), sizeof(Counters) + sizeof(Globals),
                          hipMemcpyDeviceToHost, st));
    return S5_OK;
}

// Or have a kernel write them into the mapped host block and raise its flag
// to a new sequence number (returned).  Unlike a copy followed by an event,
// this puts no marker between the kernels of the stream.
uint32_t g_publish_seq = 0;
bool g_miss_publish = false;  // test hook: raise a word next to the flag instead
uint32_t publish_start(const Ptrs& P, const HostView& H, int which, hipStream_t st) {
    if (++g_publish_seq == 0) ++g_publish_seq;  // 0 never marks a publication
    launch_publish(readback_src(P, which), sizeof(Counters) + sizeof(Globals), H.dev,
                   (uint32_t*)(H.dev + kFlagOff + (g_miss_publish ? 4 : 0)), g_publish_seq, st);
    return g_publish_seq;
}

// Unpack the host block once the copy has landed.
int readback_parse(const HostView& H, int which) {
    const char* hb = (const char*)H.host;
    memcpy(H.hc, which == 0 ? hb : hb + sizeof(Globals), sizeof(Counters));
    memcpy(H.hg, which == 0 ? hb + sizeof(Counters) : hb, sizeof(Globals));
    return status_rc(H.hg->status);
}

// Copy a pass's counters together with the globals and wait for them.
int readback_copy(const Ptrs& P, const HostView& H, int which, hipStream_t st) {
    int rc = readback_start(P, H, which, st);
    if (rc) return rc;
    S5_HIP(hipStreamSynchronize(st));
    return readback_parse(H, which);
}

// Wait until publication `seq` has landed, then unpack it.  The host polls
// the flag word, yielding its core between polls once the wait has lasted
// 200 us.  From 2 ms on it also asks the stream, at most once a millisecond,
// whether it has drained, and if it has while the flag still holds another
// number, it copies the counters instead, so the wait always ends.  (Not
// sooner or more often: a stream query puts a marker into the stream, and the
// kernel after it starts about 5 us later.)
int publish_wait(const Ptrs& P, const HostView& H, int which, uint32_t seq, hipStream_t st) {
    using clock = std::chrono::steady_clock;
    const volatile uint32_t* flag = (const volatile uint32_t*)((const char*)H.host + kFlagOff);
    const auto t0 = clock::now();
    auto next_query = t0 + std::chrono::milliseconds(2);
    bool yielding = false, queried = false;
    for (uint32_t spin = 1; *flag != seq; ++spin) {
        if (yielding) std::this_thread::yield();
        if (spin % 256) continue;
        const auto now = clock::now();
        yielding = now - t0 >= std::chrono::microseconds(200);
        if (now < next_query) continue;
        next_query = now + std::chrono::milliseconds(1);
        queried = true;
        const hipError_t q = hipStreamQuery(st);
        if (q == hipErrorNotReady) continue;
        (void)hipGetLastError();
        if (q != hipSuccess) return S5_ERR_HIP;
        if (*flag != seq) return readback_copy(P, H, which, st);
    }
    if (queried) (void)hipGetLastError();  // a not-ready answer is no error
    std::atomic_thread_fence(std::memory_order_acquire);
    return readback_parse(H, which);
}

// Read a pass's counters together with the globals and wait for them.
int readback(const Ptrs& P, const HostView& H, int which, hipStream_t st) {
    if (!H.dev) return readback_copy(P, H, which, st);
    const uint32_t seq = publish_start(P, H, which, st);
    S5_HIP(hipGetLastError());
    return publish_wait(P, H, which, seq, st);
}

// Host-driven passes from `level` on (counters of the pass about to run in
// H.hc), then the base case and the boundary LCPs.
int host_passes(const SortArgs& a, const Cfg& c, const Layout& L, const Ptrs& P,
                const HostView& H, uint32_t level, hipStream_t st, s5_stats* stats) {
    int cur = (int)(level & 1u), buf = (int)(level & 1u);
    int rc = S5_OK;
    while (H.hc->n_large > 0) {
        const PassShape S = host_shape(*H.hc, L);
        const int nxt = cur ^ 1;
        pass_front(a, c, L, P, S, cur, buf, 0u, st);
        if (S.n_learn) {
            // learned splitters that leave a range bucket too large are redone sampled
            const uint32_t before = H.hg->late_fallbacks;
            launch_learn_check(S.n_learn, P.lseg[cur], P.learn_seg, P.cs, c.beta, P.glob, Dyn{}, st);
            rc = readback(P, H, cur, st);
            if (rc) return rc;
            if (H.hg->late_fallbacks != before) pass_front(a, c, L, P, S, cur, buf, 1u, st);
        }
        // the plan writes the next pass's counters; they are published to the
        // host while the redistribution runs, and the host waits for them
        // only, so the next pass's launches queue behind the redistribution
        // with no idle gap (the sort without allocations copies them and waits
        // for the whole stream instead)
        pass_plan(a, c, L, P, S, cur, buf, level, st);
        uint32_t seq = 0;
        if (H.dev) {
            seq = publish_start(P, H, nxt, st);
        } else {
            rc = readback_start(P, H, nxt, st);
            if (rc) return rc;
        }
        pass_scatter(a, c, P, S, cur, buf, level, st);
        S5_HIP(hipGetLastError());
        if (seq) {
            rc = publish_wait(P, H, nxt, seq, st);
        } else {
            S5_HIP(hipStreamSynchronize(st));
            rc = readback_parse(H, nxt);
        }
        if (rc) return rc;
        stats->moved_M += S.now.moved;
        stats->segments += S.now.n_large;
        if (level == 0) {
            stats->max_bucket = H.hc->max_bucket;
            stats->entropy_bits = S.now.moved ? H.hc->entropy_sum / (double)S.now.moved : 0.0;
        }
        ++level;
        cur = nxt;
        if (c.distribution != S5_DISTRIBUTE_TWO_PASS) buf ^= 1;
    }
    stats->passes = level;
    uint32_t n_base[kBaseClasses];
    for (int q = 0; q < kBaseClasses; ++q) n_base[q] = H.hg->n_base[q];
    const Dyn none[kBaseClasses];
    timed(K_BASE, H.hg->base_elems, st, [&] {
        launch_base_sort(n_base, P.base_list, P.key[0], P.key[1], P.key2[0], P.key2[1],
                         P.idx[0], P.idx[1], a.chars, a.offsets, a.perm, a.lcp, c.T, P.glob,
                         none, nullptr, codec_of(c, P), st);
    });
    timed(K_LCPFIX, a.n, st, [&] {
        launch_lcp_fix(a.chars, a.offsets, a.set_begin, a.num_sets, a.n, a.perm, a.lcp, nullptr,
                       P.glob, st);
    });
    S5_HIP(hipGetLastError());
    return S5_OK;
}

// The counters of the root level.  A single set of more than T strings is one
// large segment, whose shape the host computes with the planner's own
// seg_shape, so the first level is launched without waiting for the device.
// The status word (the key cache's argument checks) then arrives with the
// first level's counters, before any kernel reads the arena past the three
// words the key cache loaded: the first level advances keys by at most 8
// bytes, from those words.  Sets, and a root that goes straight to the base
// case, read the counters back.
int root_counters(const SortArgs& a, const Cfg& c, const Ptrs& P, const HostView& H,
                  hipStream_t st) {
    if (t_quiet || a.set_begin || a.n <= c.T) return readback(P, H, 0, st);
    memset(H.hc, 0, sizeof *H.hc);
    memset(H.hg, 0, sizeof *H.hg);
    uint32_t d, ulen, tiles, chunks;
    seg_shape(a.n, SetP{c.T, c.dmax, c.tile_min}, d, ulen, tiles, chunks);
    H.hc->n_large = 1;
    H.hc->tiles = tiles;
    H.hc->chunks = chunks;
    H.hc->kmax = 2 * ((1u << d) - 1) + 1;
    H.hc->moved = a.n;
    H.hc->pad0 = c.mode == S5_SPLIT_LEARNED && a.n >= kLearnMin ? 1u : 0u;
    return S5_OK;
}

void final_stats(const HostView& H, s5_stats* stats) {
    stats->fallbacks = H.hg->fallbacks;
    stats->learned_proposals = H.hg->learned_props;
    stats->moved_one_bucket = H.hg->one_bucket;
    {  // the depth every root segment started at (as the planner computed it)
        const unsigned long long mx = H.hg->pre_max, mn = ~H.hg->pre_cmin;
        stats->root_depth = H.hg->pre_bad || mn > mx ? 0u : lcp8(mn, mx);
    }
    stats->imbalance_max = H.hg->imb_max_milli / 1000.0;
    stats->imbalance_mean =
        H.hg->learned_props ? H.hg->imb_sum_milli / 1000.0 / H.hg->learned_props : 0.0;
    stats->base_items = 0;
    for (int q = 0; q < kBaseClasses; ++q) stats->base_items += H.hg->n_base[q];
}

// The whole sort on one workspace, host-driven.  `host` is a pinned block of
// >= 4 KiB.
int run_sort(const SortArgs& a, const Cfg& c0, void* ws, size_t ws_bytes, void* host,
             hipStream_t st, s5_stats* stats) {
    memset(stats, 0, sizeof *stats);
    Cfg c = c0;
    const Layout L = make_layout(a.n, c, 0);
    if (ws_bytes < L.total) return S5_ERR_NOMEM;
    const Ptrs P = make_ptrs(L, (char*)ws);
    const HostView H = host_view(host, !t_quiet);
    int rc = choose_alphabet(a, c, P, host, st);
    if (rc) return rc;
    uint32_t retries = 0;
    for (;;) {
        memset(stats, 0, sizeof *stats);
        stats->workspace_bytes = L.total;
        start_sort(a, c, L, P, st);
        S5_HIP(hipGetLastError());
        rc = root_counters(a, c, P, H, st);
        if (!rc) rc = host_passes(a, c, L, P, H, 0, st, stats);
        if (!rc) {
            // the globals after the last kernel (with counters that are not used)
            if (readback(P, H, 0, st) == S5_ERR_HIP) return S5_ERR_HIP;
            final_stats(H, stats);
            rc = status_rc(H.hg->status);
        }
        prof_collect();
        if (rc != kRetryBytes || c.b == 8) break;
        S5_HIP(hipStreamSynchronize(st));  // every kernel of the packed attempt is done
        c.b = 8;  // a byte outside the sampled alphabet: byte keys
        ++retries;
    }
    stats->char_bits = c.b;
    stats->alphabet_retries = retries;
    return rc;
}

// ---- graph-captured sorts --------------------------------------------------
// The first `levels` passes, the base case and the boundary LCPs are captured
// once into a hipGraph (kernels only: counters are cleared by a kernel) and
// replayed by one launch.  Every pass kernel reads its work count on the
// device; the base case and the LCP completion run only if no segment is left
// for a further pass, otherwise the host finishes the remaining passes.

struct GraphKey {
    const void *chars, *offsets, *set_begin, *perm, *lcp, *ws;
    size_t ws_bytes;
    uint64_t chars_len;
    uint32_t num_sets, n, levels, tuned;
    Cfg c;
    int dev;
};

struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec;
};

std::vector<GraphEntry> g_graphs;  // most recent last
std::unordered_map<int, hipStream_t> g_capture_streams;
constexpr size_t kGraphCache = 8;

bool same_key(const GraphKey& x, const GraphKey& y) { return memcmp(&x, &y, sizeof x) == 0; }

void graphs_release() {
    for (auto& e : g_graphs) (void)hipGraphExecDestroy(e.exec);
    g_graphs.clear();
}

void enqueue_graph_body(const SortArgs& a, const Cfg& c, const Layout& L, const Ptrs& P,
                        uint32_t levels, hipStream_t st) {
    start_sort(a, c, L, P, st);
    for (uint32_t level = 0; level < levels; ++level) {
        const int cur = (int)(level & 1u), buf = cur;
        const PassShape S = graph_shape(P, L, c, cur);
        pass_front(a, c, L, P, S, cur, buf, 0u, st);
        if (c.mode == S5_SPLIT_LEARNED) {
            launch_learn_check(0, P.lseg[cur], P.learn_seg, P.cs, c.beta, P.glob, S.learn, st);
            pass_front(a, c, L, P, S, cur, buf, 1u, st);
        }
        pass_back(a, c, L, P, S, cur, buf, level, st);
        launch_pass_stats(P.cnt[cur], P.cnt[cur ^ 1], P.glob, level, st);
    }
    const uint32_t* guard = &P.cnt[levels & 1u]->n_large;
    Dyn bd[kBaseClasses];
    for (int q = 0; q < kBaseClasses; ++q) {
        const uint32_t units = q == 0 ? (L.caps.base[0] + kWaves - 1) / kWaves : L.caps.base[q];
        bd[q] = dyn_of(&P.glob->n_base[q], L.caps.base[q], std::min(units, kGraphBaseGrid));
    }
    const uint32_t zero[kBaseClasses] = {};
    launch_base_sort(zero, P.base_list, P.key[0], P.key[1], P.key2[0], P.key2[1], P.idx[0],
                     P.idx[1], a.chars, a.offsets, a.perm, a.lcp, c.T, P.glob, bd, guard,
                     codec_of(c, P), st);
    launch_lcp_fix(a.chars, a.offsets, a.set_begin, a.num_sets, a.n, a.perm, a.lcp, guard, P.glob,
                   st);
}

int get_graph(const GraphKey& key, const SortArgs& a, const Cfg& c, const Layout& L,
              const Ptrs& P, hipGraphExec_t* out) {
    for (size_t i = 0; i < g_graphs.size(); ++i)
        if (same_key(g_graphs[i].key, key)) {
            GraphEntry e = g_graphs[i];
            g_graphs.erase(g_graphs.begin() + i);
            g_graphs.push_back(e);
            *out = e.exec;
            return S5_OK;
        }
    hipStream_t& cs = g_capture_streams[key.dev];
    if (!cs) S5_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    S5_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const bool prof = g_prof_on;
    g_prof_on = false;  // no event records inside the capture
    enqueue_graph_body(a, c, L, P, key.levels, cs);
    g_prof_on = prof;
    hipGraph_t graph = nullptr;
    const hipError_t le = hipGetLastError();
    const hipError_t ee = hipStreamEndCapture(cs, &graph);
    if (le != hipSuccess || ee != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return S5_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return S5_ERR_HIP;
    if (g_graphs.size() >= kGraphCache) {
        (void)hipGraphExecDestroy(g_graphs.front().exec);
        g_graphs.erase(g_graphs.begin());
    }
    g_graphs.push_back(GraphEntry{key, exec});
    *out = exec;
    return S5_OK;
}

int run_graph(const SortArgs& a, const Cfg& c0, uint32_t levels, void* ws, size_t ws_bytes,
              void* host, hipStream_t st, s5_stats* stats) {
    memset(stats, 0, sizeof *stats);
    Cfg c = c0;
    const uint32_t tune_sets = a.tune_host ? a.num_sets : 0u;
    const Layout L = make_layout(a.n, c, tune_sets);
    if (ws_bytes < L.total) return S5_ERR_NOMEM;
    const Ptrs P = make_ptrs(L, (char*)ws);
    const HostView H = host_view(host, !t_quiet);
    int rc = choose_alphabet(a, c, P, host, st);
    if (rc) return rc;
    uint32_t retries = 0;
    for (;;) {
        memset(stats, 0, sizeof *stats);
        stats->workspace_bytes = L.total;
        GraphKey key;
        memset(&key, 0, sizeof key);
        key.chars = a.chars;
        key.chars_len = a.chars_len;
        key.offsets = a.offsets;
        key.set_begin = a.set_begin;
        key.perm = a.perm;
        key.lcp = a.lcp;
        key.ws = ws;
        key.ws_bytes = ws_bytes;
        key.num_sets = a.num_sets;
        key.n = a.n;
        key.levels = levels;
        key.tuned = tune_sets ? 1u : 0u;
        key.c = c;
        S5_HIP(hipGetDevice(&key.dev));
        if (tune_sets)
            S5_HIP(hipMemcpyAsync(P.set_tune, a.tune_host, (size_t)tune_sets * 4,
                                  hipMemcpyHostToDevice, st));
        hipGraphExec_t exec = nullptr;
        rc = get_graph(key, a, c, L, P, &exec);
        if (rc) return rc;
        timed(K_GRAPH, a.n, st, [&] { (void)hipGraphLaunch(exec, st); });
        S5_HIP(hipGetLastError());
        rc = readback(P, H, (int)(levels & 1u), st);
        if (!rc) {
            stats->passes = H.hg->passes;
            stats->moved_M = H.hg->moved;
            stats->segments = H.hg->segments;
            stats->max_bucket = H.hg->max_bucket0;
            stats->entropy_bits =
                H.hg->moved0 ? H.hg->entropy_sum0 / (double)H.hg->moved0 : 0.0;
            if (H.hc->n_large > 0) {
                // deeper than the captured levels: the host finishes the sort
                s5_stats tail;
                memset(&tail, 0, sizeof tail);
                rc = host_passes(a, c, L, P, H, levels, st, &tail);
                stats->passes = tail.passes;
                stats->moved_M += tail.moved_M;
                stats->segments += tail.segments;
            }
        }
        if (!rc) {
            // the globals after the last kernel (with counters that are not used)
            if (readback(P, H, 0, st) == S5_ERR_HIP) return S5_ERR_HIP;
            final_stats(H, stats);
            rc = status_rc(H.hg->status);
        }
        prof_collect();
        if (rc != kRetryBytes || c.b == 8) break;
        S5_HIP(hipStreamSynchronize(st));
        c.b = 8;  // a byte outside the sampled alphabet: byte keys (another graph)
        ++retries;
    }
    stats->char_bits = c.b;
    stats->alphabet_retries = retries;
    return rc;
}

// ---- the sort without allocations (s5_sort_static) -------------------------
// Its workspace is this file-scope device array; each device holds its own
// copy at its own address, looked up once per device with
// hipGetSymbolAddress (the array's name in host code is not a device address).
static __device__ __align__(256) unsigned char scratch[S5_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void* g_scratch_dev[kMaxDevices];  // device address of `scratch` per device (null: not yet)
// counters of a static sort are read back into static host memory (no pinned block)
alignas(4096) char g_static_host[3 * kHostSlot];
// its statistics go to a fixed table instead of the stream map
constexpr int kStaticRecs = 16;
struct StaticRecord {
    hipStream_t stream;
    StreamRecord rec;
    bool used;
};
StaticRecord g_static_recs[kStaticRecs];

int static_scratch(void** out) {
    int dev = 0;
    S5_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return S5_ERR_HIP;
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return S5_ERR_HIP;
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return S5_OK;
}

// Record the outcome of a sort for s5_stats_get (caller holds g_mu).
void record(hipStream_t st, const s5_stats& stats, int rc, bool fixed_table) {
    StreamRecord r{stats, rc, ++g_seq};
    if (!fixed_table) {
        g_last[st] = r;
        return;
    }
    int slot = -1;
    for (int i = 0; i < kStaticRecs && slot < 0; ++i)
        if (g_static_recs[i].used && g_static_recs[i].stream == st) slot = i;
    for (int i = 0; i < kStaticRecs && slot < 0; ++i)
        if (!g_static_recs[i].used) slot = i;
    if (slot < 0) {  // replace the oldest
        slot = 0;
        for (int i = 1; i < kStaticRecs; ++i)
            if (g_static_recs[i].rec.seq < g_static_recs[slot].rec.seq) slot = i;
    }
    g_static_recs[slot] = StaticRecord{st, r, true};
}

// Where a sort's workspace comes from.
enum class WsFrom { Pool, Caller, Static };

int sort_common(const SortArgs& a, const s5_config* cfg, void* ws, size_t ws_bytes,
                hipStream_t st, bool graph, WsFrom from) {
    Cfg c;
    int rc = resolve_cfg(cfg, &c);
    if (rc) return rc;
    if (from == WsFrom::Static &&
        make_layout(a.n, c, 0).total > (size_t)S5_STATIC_SCRATCH_BYTES)
        return S5_ERR_TOO_LARGE;
    if (a.n == 0) {
        std::lock_guard<std::mutex> g(g_mu);
        s5_stats z;
        memset(&z, 0, sizeof z);
        record(st, z, S5_OK, from == WsFrom::Static);
        return S5_OK;
    }
    // per-set parameters raise the launch-wide limits they must fit in
    if (a.tune_host) {
        for (uint32_t s = 0; s < a.num_sets; ++s) {
            const SetP t = unpack_set_tune(a.tune_host[s]);
            c.T = std::max(c.T, t.T);
            c.dmax = std::max(c.dmax, t.d_max);
            c.T_caps = std::min(c.T_caps, t.T);
            c.tile_caps = std::min(c.tile_caps, t.tile_min);
        }
    }
    std::lock_guard<std::mutex> g(g_mu);
    const size_t need = make_layout(a.n, c, a.tune_host ? a.num_sets : 0u).total;
    void* host = nullptr;
    if (from == WsFrom::Static) {
        rc = static_scratch(&ws);
        if (rc) return rc;
        ws_bytes = S5_STATIC_SCRATCH_BYTES;
        host = g_static_host;
    } else if (from == WsFrom::Pool) {
        DevPool* P = nullptr;
        rc = pool_get(need, &P);
        if (rc) return rc;
        ws = P->ptr;
        ws_bytes = P->bytes;
        host = P->host;
    } else {
        DevPool* P = nullptr;
        rc = pool_get(0, &P);
        if (rc) return rc;
        host = P->host;
    }
    s5_stats stats;
    t_quiet = from == WsFrom::Static;
    rc = graph ? run_graph(a, c, c.graph_levels, ws, ws_bytes, host, st, &stats)
               : run_sort(a, c, ws, ws_bytes, host, st, &stats);
    t_quiet = false;
    record(st, stats, rc, from == WsFrom::Static);
    return rc;
}

}  // namespace

extern "C" {

int s5_sort_ex(const uint8_t* chars, uint64_t chars_len, const uint64_t* offsets, uint32_t n,
               uint32_t* out_perm, uint32_t* out_lcp, const s5_config* cfg, void* workspace,
               size_t workspace_bytes, hipStream_t stream) {
    if (n > 0 && (!chars || !offsets || !out_perm || !out_lcp)) return S5_ERR_INVALID;
    if (n == 0xFFFFFFFFu) return S5_ERR_INVALID;
    SortArgs a{chars, chars_len, offsets, nullptr, 1u, n, out_perm, out_lcp, nullptr};
    return sort_common(a, cfg, workspace, workspace_bytes, stream, false,
                       workspace ? WsFrom::Caller : WsFrom::Pool);
}

int s5_sort_static(const uint8_t* chars, uint64_t chars_len, const uint64_t* offsets, uint32_t n,
                   uint32_t* out_perm, uint32_t* out_lcp, const s5_config* cfg,
                   hipStream_t stream) {
    if (n > 0 && (!chars || !offsets || !out_perm || !out_lcp)) return S5_ERR_INVALID;
    if (n == 0xFFFFFFFFu) return S5_ERR_INVALID;
    SortArgs a{chars, chars_len, offsets, nullptr, 1u, n, out_perm, out_lcp, nullptr};
    return sort_common(a, cfg, nullptr, 0, stream, false, WsFrom::Static);
}

int s5_sort(const uint8_t* chars, const uint64_t* offsets, uint32_t n, uint32_t* out_perm,
            uint32_t* out_lcp, hipStream_t stream) {
    return s5_sort_ex(chars, 0, offsets, n, out_perm, out_lcp, nullptr, nullptr, 0, stream);
}

size_t s5_workspace_bytes(uint32_t n, const s5_config* cfg) {
    Cfg c;
    if (resolve_cfg(cfg, &c)) return 0;
    return make_layout(n, c, 0).total;
}

int s5_sort_batched_tuned(const uint8_t* chars, uint64_t chars_len, const uint64_t* offsets,
                          const uint64_t* set_begin, uint32_t num_sets,
                          const s5_set_tuning* set_tuning, uint32_t* out_perm, uint32_t* out_lcp,
                          const s5_config* cfg, hipStream_t stream) {
    if (num_sets == 0) return S5_OK;
    if (!set_begin || num_sets == 0xFFFFFFFFu) return S5_ERR_INVALID;
    Cfg base;
    if (resolve_cfg(cfg, &base)) return S5_ERR_INVALID;
    // the two-pass distribution runs in host-driven sorts only
    if (base.distribution != S5_DISTRIBUTE_ONE_PASS) return S5_ERR_INVALID;
    // per-set parameters: validated and packed on the host
    std::vector<uint32_t> packed;
    if (set_tuning) {
        packed.resize(num_sets);
        for (uint32_t s = 0; s < num_sets; ++s) {
            const s5_set_tuning& t = set_tuning[s];
            const uint32_t v = t.splitters ? t.splitters : (1u << base.dmax) - 1;
            uint32_t d = 0;
            while (((1u << (d + 1)) - 1) <= v && d < 31) ++d;
            if (v < 7 || v > 1023 || ((1u << d) - 1) != v) return S5_ERR_INVALID;
            const uint32_t T = t.base_threshold ? t.base_threshold : base.T;
            if (T < 64 || T > 2048) return S5_ERR_INVALID;
            const uint32_t tile = t.tile ? t.tile : base.tile_min;
            if (tile % 64 || tile > (1u << 20)) return S5_ERR_INVALID;
            packed[s] = pack_set_tune(T, d, tile);
        }
    }
    uint64_t ends[2];
    if (hipMemcpyAsync(ends, set_begin, 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(ends + 1, set_begin + num_sets, 8, hipMemcpyDeviceToHost, stream) !=
            hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return S5_ERR_HIP;
    if (ends[0] != 0 || ends[1] >= 0xFFFFFFFFull) return S5_ERR_INVALID;
    const uint32_t n = (uint32_t)ends[1];
    if (n > 0 && (!chars || !offsets || !out_perm || !out_lcp)) return S5_ERR_INVALID;
    SortArgs a{chars, chars_len, offsets, set_begin, num_sets, n, out_perm, out_lcp,
               set_tuning ? packed.data() : nullptr};
    return sort_common(a, cfg, nullptr, 0, stream, true, WsFrom::Pool);
}

int s5_sort_batched(const uint8_t* chars, uint64_t chars_len, const uint64_t* offsets,
                    const uint64_t* set_begin, uint32_t num_sets, uint32_t* out_perm,
                    uint32_t* out_lcp, const s5_config* cfg, hipStream_t stream) {
    return s5_sort_batched_tuned(chars, chars_len, offsets, set_begin, num_sets, nullptr, out_perm,
                                 out_lcp, cfg, stream);
}

int s5_stats_get(hipStream_t stream, s5_stats* host_out) {
    if (!host_out) return S5_ERR_INVALID;
    if (hipStreamSynchronize(stream) != hipSuccess) return S5_ERR_HIP;
    std::lock_guard<std::mutex> g(g_mu);
    const StreamRecord* r = nullptr;
    auto it = g_last.find(stream);
    if (it != g_last.end()) r = &it->second;
    for (const StaticRecord& s : g_static_recs)  // the newest record of the stream wins
        if (s.used && s.stream == stream && (!r || s.rec.seq > r->seq)) r = &s.rec;
    if (!r) {
        memset(host_out, 0, sizeof *host_out);
        return S5_OK;
    }
    *host_out = r->stats;
    return r->status == S5_ERR_DEVICE ? S5_ERR_DEVICE : S5_OK;
}

const char* s5_strerror(int status) {
    switch (status) {
        case S5_OK: return "success";
        case S5_ERR_INVALID: return "invalid argument";
        case S5_ERR_NOMEM: return "workspace missing, too small, or device allocation failed";
        case S5_ERR_HIP: return "HIP runtime error";
        case S5_ERR_DEVICE: return "device-side capacity check failed";
        case S5_ERR_TOO_LARGE: return "sort needs more than the static scratch array";
        default: return "unknown status";
    }
}

void s5_release(void) {
    std::lock_guard<std::mutex> g(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_pools) {
        (void)hipSetDevice(kv.first);
        (void)hipDeviceSynchronize();
    }
    graphs_release();
    for (auto& kv : g_capture_streams) {
        (void)hipSetDevice(kv.first);
        if (kv.second) (void)hipStreamDestroy(kv.second);
    }
    g_capture_streams.clear();
    for (auto& kv : g_pools) {
        (void)hipSetDevice(kv.first);
        (void)hipDeviceSynchronize();
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
        if (kv.second.host) (void)hipHostFree(kv.second.host);
    }
    g_pools.clear();
    g_host_dev.clear();
    (void)hipSetDevice(cur);
}

int s5_prefix_keys(const uint8_t* chars, const uint64_t* offsets, uint32_t n, uint32_t depth,
                   uint64_t* out_keys, hipStream_t stream) {
    if (n > 0 && (!chars || !offsets || !out_keys)) return S5_ERR_INVALID;
    launch_prefix_keys(chars, offsets, n, depth, out_keys, stream);
    return hipGetLastError() == hipSuccess ? S5_OK : S5_ERR_HIP;
}

int s5_classify(const uint64_t* keys, uint32_t n, const uint64_t* splitters, uint32_t v,
                uint16_t* out_bucket, hipStream_t stream) {
    return s5_classify_ex(keys, n, splitters, v, S5_CLASSIFY_UNROLL, out_bucket, stream);
}

int s5_classify_ex(const uint64_t* keys, uint32_t n, const uint64_t* splitters, uint32_t v,
                   uint32_t variant, uint16_t* out_bucket, hipStream_t stream) {
    if (variant != S5_CLASSIFY_UNROLL && variant != S5_CLASSIFY_EQUAL &&
        variant != S5_CLASSIFY_JUMP)
        return S5_ERR_INVALID;
    uint32_t d = 0;
    while (d < 11 && ((1u << d) - 1) < v) ++d;
    if (v < 1 || v > 1023 || ((1u << d) - 1) != v || !splitters) return S5_ERR_INVALID;
    if (n > 0 && (!keys || !out_bucket)) return S5_ERR_INVALID;
    std::lock_guard<std::mutex> g(g_mu);
    DevPool* P = nullptr;
    int rc = pool_get((size_t)(v + 1) * (16 + 2 * kJumpPerTreeSlot), &P);
    if (rc) return rc;
    uint64_t* tlo = (uint64_t*)P->ptr;
    uint64_t* tin = tlo + (v + 1);
    uint16_t* jt = (uint16_t*)(tin + (v + 1));
    launch_classify_plain(keys, n, splitters, v, d, variant, tlo, tin, jt, out_bucket, stream);
    if (hipGetLastError() != hipSuccess) return S5_ERR_HIP;
    // the pool may be reused by the next call: finish before returning
    return hipStreamSynchronize(stream) == hipSuccess ? S5_OK : S5_ERR_HIP;
}


int s5_profile_enable(int on) {
    std::lock_guard<std::mutex> g(g_mu);
    g_prof_on = on != 0;
    for (auto& A : g_prof) A = ProfAcc();
    return S5_OK;
}

int s5_profile_only(const char* kernel) {
    std::lock_guard<std::mutex> g(g_mu);
    if (!kernel || !kernel[0]) {
        g_prof_only = -1;
        return S5_OK;
    }
    for (int k = 0; k < K_COUNT; ++k)
        if (strcmp(kernel, kKName[k]) == 0) {
            g_prof_only = k;
            return S5_OK;
        }
    return S5_ERR_INVALID;
}

int s5_profile_read(s5_kernel_profile* out, uint32_t max, uint32_t* count) {
    if (!out || !count) return S5_ERR_INVALID;
    std::lock_guard<std::mutex> g(g_mu);
    uint32_t c = 0;
    for (int k = 0; k < K_COUNT; ++k) {
        if (!g_prof[k].launches) continue;
        if (c < max) {
            s5_kernel_profile& p = out[c];
            memset(&p, 0, sizeof p);
            strncpy(p.name, kKName[k], sizeof p.name - 1);
            p.launches = g_prof[k].launches;
            p.total_ms = g_prof[k].ms;
            p.items = g_prof[k].items;
            p.alg_bytes = g_prof[k].bytes;
        }
        ++c;
    }
    *count = c;
    return S5_OK;
}


static int mlp_check_m(uint32_t m) {
    return (m >= kLearnGrp && m <= kLearnM && m % kLearnGrp == 0) ? S5_OK : S5_ERR_INVALID;
}

int s5_mlp_train(const uint64_t* sorted_keys, uint32_t m, uint32_t steps, float lr, uint64_t seed,
                 float* out_params, hipStream_t stream) {
    if (!sorted_keys || !out_params || mlp_check_m(m) || steps > 100000) return S5_ERR_INVALID;
    std::lock_guard<std::mutex> g(g_mu);
    DevPool* P = nullptr;
    int rc = pool_get(learn_bytes(1, m), &P);
    if (rc) return rc;
    launch_mlp_train(learn_ctx(P->ptr, 1, m), sorted_keys, m, steps, lr, seed, out_params, stream);
    if (hipGetLastError() != hipSuccess) return S5_ERR_HIP;
    return hipStreamSynchronize(stream) == hipSuccess ? S5_OK : S5_ERR_HIP;
}

int s5_mlp_grad(const float* params, const uint64_t* sorted_keys, uint32_t m, float* out_grad,
                hipStream_t stream) {
    if (!params || !sorted_keys || !out_grad || mlp_check_m(m)) return S5_ERR_INVALID;
    std::lock_guard<std::mutex> g(g_mu);
    DevPool* P = nullptr;
    int rc = pool_get(learn_bytes(1, m), &P);
    if (rc) return rc;
    launch_mlp_grad(learn_ctx(P->ptr, 1, m), params, sorted_keys, m, out_grad, stream);
    if (hipGetLastError() != hipSuccess) return S5_ERR_HIP;
    return hipStreamSynchronize(stream) == hipSuccess ? S5_OK : S5_ERR_HIP;
}

int s5_debug_limit_capacity(uint32_t which, uint32_t limit) {
    if (which > S5_CAP_BASE3) return S5_ERR_INVALID;
    std::lock_guard<std::mutex> g(g_mu);
    g_cap_limit[which] = limit;
    graphs_release();  // their layouts were planned with the old capacities
    return S5_OK;
}

int s5_debug_miss_publish(int on) {
    std::lock_guard<std::mutex> g(g_mu);
    g_miss_publish = on != 0;
    return S5_OK;
}

int s5_debug_count_writes(uint32_t* perm, uint32_t* lcp, uint64_t n, uint32_t* perm_counts,
                          uint32_t* lcp_counts, uint32_t* stray) {
    if (perm_counts && (!perm || !lcp || !lcp_counts || !stray)) return S5_ERR_INVALID;
    WriteCount w;
    w.perm_base = perm;
    w.lcp_base = lcp;
    w.perm_cnt = perm_counts;
    w.lcp_cnt = perm_counts ? lcp_counts : nullptr;
    w.stray = perm_counts ? stray : nullptr;
    w.n = n;
    std::lock_guard<std::mutex> g(g_mu);
    return set_write_count(w) ? S5_OK : S5_ERR_INVALID;
}

int s5_mlp_propose(const float* params, const uint64_t* sorted_keys, uint32_t m, uint32_t v,
                   float beta, uint64_t* out_splitters, float* out_cdf, uint32_t* out_reject,
                   hipStream_t stream) {
    if (!params || !sorted_keys || !out_splitters || !out_cdf || !out_reject) return S5_ERR_INVALID;
    if (mlp_check_m(m) || v < 1 || v > 1023 || !(beta > 0.0f)) return S5_ERR_INVALID;
    launch_mlp_propose(params, sorted_keys, m, v, beta, out_splitters, out_cdf, out_reject, stream);
    return hipGetLastError() == hipSuccess ? S5_OK : S5_ERR_HIP;
}

int s5_mlp_eval(const float* params, const uint64_t* keys, uint32_t n, uint64_t lo, uint64_t hi,
                float* out, hipStream_t stream) {
    if (n > 0 && (!params || !keys || !out)) return S5_ERR_INVALID;
    launch_mlp_eval(params, keys, n, lo, hi, out, stream);
    return hipGetLastError() == hipSuccess ? S5_OK : S5_ERR_HIP;
}

}  // extern "C"
