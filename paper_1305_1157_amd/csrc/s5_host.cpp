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
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/s5.h"
#include "../../include/s5_profile.h"
#include "../../include/s5_learned.h"
#include "s5_internal.h"

namespace s5 {
void launch_init_keys(const uint8_t*, const uint64_t*, uint32_t, uint64_t*, uint32_t*, hipStream_t);
void launch_prefix_keys(const uint8_t*, const uint64_t*, uint32_t, uint32_t, uint64_t*, hipStream_t);
void launch_plan_roots(const uint64_t*, uint32_t, uint32_t, uint32_t*, uint32_t*, const PlanCtx&,
                       hipStream_t);
void launch_sample_tree(uint32_t, const LSeg*, const uint64_t*, uint32_t, uint32_t, uint64_t,
                        uint64_t*, uint64_t*, uint8_t*, uint32_t*, uint32_t*, Counters*,
                        hipStream_t);
void launch_classify(uint32_t, uint32_t, const LSeg*, const uint32_t*, const uint64_t*,
                     const uint64_t*, const uint64_t*, uint16_t*, uint32_t*, uint32_t, uint32_t,
                     hipStream_t);
void launch_colscan(uint32_t, uint32_t, const LSeg*, const uint32_t*, uint32_t*, uint32_t*,
                    hipStream_t);
void launch_bucket_plan(uint32_t, const LSeg*, uint32_t*, uint32_t*, const uint64_t*,
                        const uint8_t*, const PlanCtx&, uint32_t, hipStream_t);
void launch_scatter(uint32_t, uint32_t, const LSeg*, const uint32_t*, const uint16_t*,
                    const uint64_t*, const uint32_t*, uint64_t*, uint32_t*, const uint32_t*,
                    const uint32_t*, const uint32_t*, const uint64_t*, const uint8_t*,
                    const uint8_t*, const uint64_t*, uint32_t*, uint32_t*, uint32_t, uint32_t,
                    hipStream_t);
void launch_base_sort(const uint32_t*, Seg* const*, const uint64_t*, const uint64_t*,
                      const uint32_t*, const uint32_t*, const uint8_t*, const uint64_t*, uint32_t*,
                      uint32_t*, uint32_t, hipStream_t);
void launch_lcp_fix(const uint8_t*, const uint64_t*, const uint64_t*, uint32_t, uint32_t,
                    const uint32_t*, uint32_t*, hipStream_t);
void launch_classify_plain(const uint64_t*, uint32_t, const uint64_t*, uint32_t, uint32_t,
                           uint64_t*, uint64_t*, uint16_t*, hipStream_t);
size_t learn_bytes(uint32_t slots, uint32_t m);
LearnCtx learn_ctx(void* mem, uint32_t slots, uint32_t m);
void launch_learn_sort_trees(const LearnCtx&, uint32_t, LSeg*, const uint32_t*, const uint64_t*,
                             uint64_t, uint32_t, float, float, Globals*, uint64_t*, uint64_t*,
                             uint8_t*, hipStream_t);
void launch_learn_check(uint32_t, LSeg*, const uint32_t*, const uint32_t*, float, Globals*,
                        hipStream_t);
void launch_mlp_train(const LearnCtx&, const uint64_t*, uint32_t, uint32_t, float, uint64_t,
                      float*, hipStream_t);
void launch_mlp_grad(const LearnCtx&, const float*, const uint64_t*, uint32_t, float*,
                     hipStream_t);
void launch_mlp_eval(const float*, const uint64_t*, uint32_t, uint64_t, uint64_t, float*,
                     hipStream_t);
}  // namespace s5

using namespace s5;

namespace {

// learned splitters: samples per segment, Adam steps and learning rate
constexpr uint32_t kLearnSamples = kLearnM, kLearnSteps = 64;
constexpr float kLearnRate = 0.03f;

struct Cfg {
    uint32_t dmax, alpha, unroll, tile_min, T, mode;
    float beta;
    uint64_t seed;
};

int resolve_cfg(const s5_config* c, Cfg* o) {
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
    o->mode = c->splitter_mode;
    if (o->mode != S5_SPLIT_SAMPLED && o->mode != S5_SPLIT_LEARNED) return S5_ERR_INVALID;
    o->beta = c->imbalance_bound > 0 ? c->imbalance_bound : 4.0f;
    o->seed = c->seed;
    return S5_OK;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace regions (byte offsets into one device allocation).
struct Layout {
    size_t key[2], idx[2], bid, lseg[2], tile_tab, chunk_tab, tree_lo, tree_in, tree_lcp, cm, cs,
        bstart, base_list, learn, learn_seg, counters[2], glob, total;
    uint32_t learn_cap;
    Caps caps;
};

Layout make_layout(uint64_t n, const Cfg& c) {
    Layout L;
    const uint64_t kmax = (2ull << c.dmax) - 1;
    Caps cp;
    uint64_t large = n / (c.T + 1) + 2;
    // tiles of a segment: ceil(|S| / tile_len) with tile_len >= tile_min
    uint64_t tiles = n / c.tile_min + large + 1;
    uint64_t chunks = tiles / kChunkRows + large + 1;
    // sum over segments of 2^d < 4 |S| / T (plus the d >= 1 floor)
    uint64_t tree = 4 * n / c.T + 2 * large + 2;
    cp.large = (uint32_t)large;
    cp.tiles = (uint32_t)std::min<uint64_t>(tiles, 0xFFFFFFFFull);
    cp.chunks = (uint32_t)chunks;
    cp.tree = (uint32_t)tree;
    cp.bstart = (uint32_t)(2 * tree + large + 2);
    // every base item holds >= 2 strings, and > 64 / > 512 in the larger classes
    cp.base[0] = (uint32_t)(n / 2 + 2);
    cp.base[1] = (uint32_t)(n / (kBaseWave + 1) + 2);
    cp.base[2] = (uint32_t)(n / (kBaseMid + 1) + 2);
    // sum over segments of tiles x k: tiles_s <= |S|/tile_min + 1 and
    // k_s <= max(3, min(kmax, 8 |S| / T))
    const uint64_t ksum = 3 * large + 8 * n / c.T + kmax;
    cp.cm = (unsigned long long)(kmax * (n / c.tile_min + 1) + 4 * ksum);
    cp.cs = (unsigned long long)(cp.cm / kChunkRows + ksum);
    size_t p = 0;
    auto take = [&](size_t bytes) {
        size_t o = p;
        p = align_up(p + bytes);
        return o;
    };
    for (int b = 0; b < 2; ++b) L.key[b] = take(n * 8);
    for (int b = 0; b < 2; ++b) L.idx[b] = take(n * 4);
    L.bid = take(n * 2);
    for (int b = 0; b < 2; ++b) L.lseg[b] = take((size_t)cp.large * sizeof(LSeg));
    L.tile_tab = take((size_t)cp.tiles * 4);
    L.chunk_tab = take((size_t)cp.chunks * 4);
    L.tree_lo = take((size_t)cp.tree * 8);
    L.tree_in = take((size_t)cp.tree * 8);
    L.tree_lcp = take((size_t)cp.tree);
    L.cm = take((size_t)cp.cm * 4);
    L.cs = take((size_t)cp.cs * 4);
    L.bstart = take((size_t)cp.bstart * 4);
    L.base_list = take((size_t)(cp.base[0] + cp.base[1] + cp.base[2]) * sizeof(Seg));
    // learned splitters: one slot per segment of >= kLearnMin strings in a pass
    L.learn_cap = c.mode == S5_SPLIT_LEARNED ? (uint32_t)std::min<uint64_t>(large, n / kLearnMin + 1) : 0u;
    L.learn = take(learn_bytes(L.learn_cap, kLearnSamples));
    L.learn_seg = take((size_t)L.learn_cap * 4);
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
};
std::unordered_map<hipStream_t, StreamRecord> g_last;

#define S5_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return S5_ERR_HIP;       \
    } while (0)

// Get the pool of the current device with at least `bytes`.
int pool_get(size_t bytes, DevPool** out) {
    int dev = 0;
    S5_HIP(hipGetDevice(&dev));
    DevPool& P = g_pools[dev];
    if (!P.host) S5_HIP(hipHostMalloc(&P.host, 4096, hipHostMallocDefault));
    if (P.bytes < bytes) {
        if (P.ptr) {
            S5_HIP(hipDeviceSynchronize());
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
           K_LEARN, K_COUNT };
const char* const kKName[K_COUNT] = {"init_keys", "plan_roots", "sample_tree", "classify",
                                     "colscan",   "bucket_plan", "scatter",    "base_sort",
                                     "lcp_fix",   "learn_splitters"};
// algorithmic bytes per string processed: init reads an offset and 8 key bytes
// and writes key + index; classify reads a key and writes a bucket id; a
// redistribution pass reads and writes (key, index); the base case reads
// (key, index) and writes perm + lcp; the LCP completion reads one lcp word
const double kKBytes[K_COUNT] = {28, 0, 0, 10, 0, 0, 24, 20, 4, 0};
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
    if (!g_prof_on) {
        fn();
        return;
    }
    hipEvent_t a = prof_event(), b = prof_event();
    if (a) (void)hipEventRecord(a, st);
    fn();
    if (b) (void)hipEventRecord(b, st);
    if (a && b) g_pending.push_back({k, a, b, items});
}

// After the stream has been synchronized: fold pending events into totals.
void prof_collect() {
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
    const uint64_t* offsets;
    const uint64_t* set_begin;  // device, or null for a single set
    uint32_t num_sets, n;
    uint32_t* perm;
    uint32_t* lcp;
};

// The whole sort on one workspace.  `host` is a pinned block of >= 4 KiB.
int run_sort(const SortArgs& a, const Cfg& c, void* ws, size_t ws_bytes, void* host,
             hipStream_t st, s5_stats* stats) {
    memset(stats, 0, sizeof *stats);
    const Layout L = make_layout(a.n, c);
    if (ws_bytes < L.total) return S5_ERR_NOMEM;
    stats->workspace_bytes = L.total;
    char* W = (char*)ws;
    uint64_t* key[2] = {(uint64_t*)(W + L.key[0]), (uint64_t*)(W + L.key[1])};
    uint32_t* idx[2] = {(uint32_t*)(W + L.idx[0]), (uint32_t*)(W + L.idx[1])};
    uint16_t* bid = (uint16_t*)(W + L.bid);
    LSeg* lseg[2] = {(LSeg*)(W + L.lseg[0]), (LSeg*)(W + L.lseg[1])};
    uint32_t* tile_tab = (uint32_t*)(W + L.tile_tab);
    uint32_t* chunk_tab = (uint32_t*)(W + L.chunk_tab);
    uint64_t* tree_lo = (uint64_t*)(W + L.tree_lo);
    uint64_t* tree_in = (uint64_t*)(W + L.tree_in);
    uint8_t* tree_lcp = (uint8_t*)(W + L.tree_lcp);
    uint32_t* cm = (uint32_t*)(W + L.cm);
    uint32_t* cs = (uint32_t*)(W + L.cs);
    uint32_t* bstart = (uint32_t*)(W + L.bstart);
    uint32_t* learn_seg = (uint32_t*)(W + L.learn_seg);
    const LearnCtx lctx = learn_ctx(W + L.learn, L.learn_cap, kLearnSamples);
    Seg* base_list[kBaseClasses];
    base_list[0] = (Seg*)(W + L.base_list);
    base_list[1] = base_list[0] + L.caps.base[0];
    base_list[2] = base_list[1] + L.caps.base[1];
    Counters* cnt[2] = {(Counters*)(W + L.counters[0]), (Counters*)(W + L.counters[1])};
    Globals* glob = (Globals*)(W + L.glob);
    Counters* hc = (Counters*)((char*)host + 1024);
    Globals* hg = (Globals*)((char*)host + 2048);

    auto ctx_for = [&](int next) {
        PlanCtx x;
        x.lseg = lseg[next];
        x.cnt = cnt[next];
        for (int q = 0; q < kBaseClasses; ++q) x.base_list[q] = base_list[q];
        x.glob = glob;
        x.caps = L.caps;
        x.T = c.T;
        x.d_max = c.dmax;
        x.tile_min = c.tile_min;
        x.learn = c.mode == S5_SPLIT_LEARNED ? 1u : 0u;
        x.learn_cap = L.learn_cap;
        x.learn_seg = learn_seg;
        return x;
    };
    auto readback = [&](int which) -> int {
        char* src = which == 0 ? (char*)cnt[0] : (char*)glob;
        S5_HIP(hipMemcpyAsync(host, src, sizeof(Counters) + sizeof(Globals), hipMemcpyDeviceToHost,
                              st));
        S5_HIP(hipStreamSynchronize(st));
        const char* hb = (const char*)host;
        memcpy(hc, which == 0 ? hb : hb + sizeof(Globals), sizeof(Counters));
        memcpy(hg, which == 0 ? hb + sizeof(Counters) : hb, sizeof(Globals));
        return hg->status ? S5_ERR_DEVICE : S5_OK;
    };

    S5_HIP(hipMemsetAsync(cnt[0], 0, 2 * sizeof(Counters) + sizeof(Globals), st));
    timed(K_INIT, a.n, st, [&] { launch_init_keys(a.chars, a.offsets, a.n, key[0], idx[0], st); });
    timed(K_ROOTS, a.num_sets, st, [&] {
        launch_plan_roots(a.set_begin, a.num_sets, a.n, a.perm, a.lcp, ctx_for(0), st);
    });
    S5_HIP(hipGetLastError());
    int rc = readback(0);
    if (rc) {
        prof_collect();
        return rc;
    }

    int cur = 0;  // lseg / counters index of the pass about to run
    int buf = 0;  // work buffer holding the pass's input
    uint32_t level = 0;
    while (hc->n_large > 0) {
        const Counters now = *hc;
        const uint32_t kmax = now.kmax, vmax = (kmax - 1) / 2;
        const int nxt = cur ^ 1;
        // learned proposals first: a proposal that fails on its own sample is
        // switched back to sampled splitters before the sampled trees are built
        const uint32_t n_learn = std::min(now.pad0, L.learn_cap);
        if (n_learn) {
            timed(K_LEARN, n_learn, st, [&] {
                launch_learn_sort_trees(lctx, n_learn, lseg[cur], learn_seg, key[buf], c.seed,
                                        kLearnSteps, kLearnRate, c.beta, glob, tree_lo, tree_in,
                                        tree_lcp, st);
            });
        }
        timed(K_SAMPLE, now.n_large, st, [&] {
            launch_sample_tree(now.n_large, lseg[cur], key[buf], c.alpha, vmax, c.seed, tree_lo,
                               tree_in, tree_lcp, tile_tab, chunk_tab, cnt[nxt], st);
        });
        timed(K_CLASSIFY, now.moved, st, [&] {
            launch_classify(now.tiles, c.unroll, lseg[cur], tile_tab, key[buf], tree_lo, tree_in,
                            bid, cm, vmax, kmax, st);
        });
        timed(K_COLSCAN, now.moved, st,
              [&] { launch_colscan(now.chunks, kmax, lseg[cur], chunk_tab, cm, cs, st); });
        if (n_learn) {
            // learned splitters that leave a range bucket too large are redone sampled
            const uint32_t before = hg->late_fallbacks;
            launch_learn_check(n_learn, lseg[cur], learn_seg, cs, c.beta, glob, st);
            rc = readback(cur);
            if (rc) {
                prof_collect();
                return rc;
            }
            if (hg->late_fallbacks != before) {
                timed(K_SAMPLE, now.n_large, st, [&] {
                    launch_sample_tree(now.n_large, lseg[cur], key[buf], c.alpha, vmax, c.seed,
                                       tree_lo, tree_in, tree_lcp, tile_tab, chunk_tab, cnt[nxt], st);
                });
                timed(K_CLASSIFY, now.moved, st, [&] {
                    launch_classify(now.tiles, c.unroll, lseg[cur], tile_tab, key[buf], tree_lo,
                                    tree_in, bid, cm, vmax, kmax, st);
                });
                timed(K_COLSCAN, now.moved, st, [&] {
                    launch_colscan(now.chunks, kmax, lseg[cur], chunk_tab, cm, cs, st);
                });
            }
        }
        timed(K_PLAN, now.moved, st, [&] {
            launch_bucket_plan(now.n_large, lseg[cur], cs, bstart, tree_in, tree_lcp, ctx_for(nxt),
                               (uint32_t)(buf ^ 1), st);
        });
        timed(K_SCATTER, now.moved, st, [&] {
            launch_scatter(now.tiles, c.unroll, lseg[cur], tile_tab, bid, key[buf], idx[buf],
                           key[buf ^ 1], idx[buf ^ 1], cm, cs, bstart, tree_in, tree_lcp, a.chars,
                           a.offsets, a.perm, a.lcp, vmax, kmax, st);
        });
        S5_HIP(hipGetLastError());
        rc = readback(nxt);
        if (rc) {
            prof_collect();
            return rc;
        }
        stats->moved_M += now.moved;
        stats->segments += now.n_large;
        if (level == 0) {
            stats->max_bucket = hc->max_bucket;
            stats->entropy_bits = now.moved ? hc->entropy_sum / (double)now.moved : 0.0;
        }
        ++level;
        cur = nxt;
        buf ^= 1;
    }
    stats->passes = level;
    stats->fallbacks = hg->fallbacks;
    uint32_t n_base[kBaseClasses];
    for (int q = 0; q < kBaseClasses; ++q) n_base[q] = hg->n_base[q];
    stats->base_items = (uint64_t)n_base[0] + n_base[1] + n_base[2];
    timed(K_BASE, hg->base_elems, st, [&] {
        launch_base_sort(n_base, base_list, key[0], key[1], idx[0], idx[1], a.chars, a.offsets,
                         a.perm, a.lcp, c.T, st);
    });
    timed(K_LCPFIX, a.n, st, [&] {
        launch_lcp_fix(a.chars, a.offsets, a.set_begin, a.num_sets, a.n, a.perm, a.lcp, st);
    });
    S5_HIP(hipGetLastError());
    S5_HIP(hipMemcpyAsync(hg, glob, sizeof(Globals), hipMemcpyDeviceToHost, st));
    S5_HIP(hipStreamSynchronize(st));
    prof_collect();
    return hg->status ? S5_ERR_DEVICE : S5_OK;
}

int sort_common(const SortArgs& a, const s5_config* cfg, void* ws, size_t ws_bytes,
                hipStream_t st) {
    Cfg c;
    int rc = resolve_cfg(cfg, &c);
    if (rc) return rc;
    if (a.n == 0) {
        std::lock_guard<std::mutex> g(g_mu);
        StreamRecord& r = g_last[st];
        memset(&r.stats, 0, sizeof r.stats);
        r.status = S5_OK;
        return S5_OK;
    }
    std::lock_guard<std::mutex> g(g_mu);
    const size_t need = make_layout(a.n, c).total;
    void* host = nullptr;
    if (!ws) {
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
    rc = run_sort(a, c, ws, ws_bytes, host, st, &stats);
    StreamRecord& r = g_last[st];
    r.stats = stats;
    r.status = rc;
    return rc;
}

}  // namespace

extern "C" {

int s5_sort_ex(const uint8_t* chars, uint64_t chars_len, const uint64_t* offsets, uint32_t n,
               uint32_t* out_perm, uint32_t* out_lcp, const s5_config* cfg, void* workspace,
               size_t workspace_bytes, hipStream_t stream) {
    (void)chars_len;
    if (n > 0 && (!chars || !offsets || !out_perm || !out_lcp)) return S5_ERR_INVALID;
    if (n == 0xFFFFFFFFu) return S5_ERR_INVALID;
    SortArgs a{chars, offsets, nullptr, 1u, n, out_perm, out_lcp};
    return sort_common(a, cfg, workspace, workspace_bytes, stream);
}

int s5_sort(const uint8_t* chars, const uint64_t* offsets, uint32_t n, uint32_t* out_perm,
            uint32_t* out_lcp, hipStream_t stream) {
    return s5_sort_ex(chars, 0, offsets, n, out_perm, out_lcp, nullptr, nullptr, 0, stream);
}

size_t s5_workspace_bytes(uint32_t n, const s5_config* cfg) {
    Cfg c;
    if (resolve_cfg(cfg, &c)) return 0;
    return make_layout(n, c).total;
}

int s5_sort_batched(const uint8_t* chars, uint64_t chars_len, const uint64_t* offsets,
                    const uint64_t* set_begin, uint32_t num_sets, uint32_t* out_perm,
                    uint32_t* out_lcp, const s5_config* cfg, hipStream_t stream) {
    (void)chars_len;
    if (num_sets == 0) return S5_OK;
    if (!set_begin) return S5_ERR_INVALID;
    uint64_t ends[2];
    if (hipMemcpyAsync(ends, set_begin, 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(ends + 1, set_begin + num_sets, 8, hipMemcpyDeviceToHost, stream) !=
            hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return S5_ERR_HIP;
    if (ends[0] != 0 || ends[1] >= 0xFFFFFFFFull) return S5_ERR_INVALID;
    const uint32_t n = (uint32_t)ends[1];
    if (n > 0 && (!chars || !offsets || !out_perm || !out_lcp)) return S5_ERR_INVALID;
    SortArgs a{chars, offsets, set_begin, num_sets, n, out_perm, out_lcp};
    return sort_common(a, cfg, nullptr, 0, stream);
}

int s5_stats_get(hipStream_t stream, s5_stats* host_out) {
    if (!host_out) return S5_ERR_INVALID;
    if (hipStreamSynchronize(stream) != hipSuccess) return S5_ERR_HIP;
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_last.find(stream);
    if (it == g_last.end()) {
        memset(host_out, 0, sizeof *host_out);
        return S5_OK;
    }
    *host_out = it->second.stats;
    return it->second.status == S5_ERR_DEVICE ? S5_ERR_DEVICE : S5_OK;
}

const char* s5_strerror(int status) {
    switch (status) {
        case S5_OK: return "success";
        case S5_ERR_INVALID: return "invalid argument";
        case S5_ERR_NOMEM: return "workspace missing, too small, or device allocation failed";
        case S5_ERR_HIP: return "HIP runtime error";
        case S5_ERR_DEVICE: return "device-side capacity check failed";
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
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
        if (kv.second.host) (void)hipHostFree(kv.second.host);
    }
    g_pools.clear();
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
    uint32_t d = 0;
    while (d < 11 && ((1u << d) - 1) < v) ++d;
    if (v < 1 || v > 1023 || ((1u << d) - 1) != v || !splitters) return S5_ERR_INVALID;
    if (n > 0 && (!keys || !out_bucket)) return S5_ERR_INVALID;
    std::lock_guard<std::mutex> g(g_mu);
    DevPool* P = nullptr;
    int rc = pool_get((size_t)(v + 1) * 16, &P);
    if (rc) return rc;
    uint64_t* tlo = (uint64_t*)P->ptr;
    uint64_t* tin = tlo + (v + 1);
    launch_classify_plain(keys, n, splitters, v, d, tlo, tin, out_bucket, stream);
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

int s5_mlp_eval(const float* params, const uint64_t* keys, uint32_t n, uint64_t lo, uint64_t hi,
                float* out, hipStream_t stream) {
    if (n > 0 && (!params || !keys || !out)) return S5_ERR_INVALID;
    launch_mlp_eval(params, keys, n, lo, hi, out, stream);
    return hipGetLastError() == hipSuccess ? S5_OK : S5_ERR_HIP;
}

}  // extern "C"
