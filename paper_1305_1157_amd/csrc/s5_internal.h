// Internal definitions shared by the S^5 kernels (s5_kernels.hip) and the
// host orchestrator (s5_host.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "s5_word.h"

namespace s5 {

// A distribution pass works on "tiles": contiguous runs of a segment that one
// workgroup classifies and redistributes; each tile owns one row of bucket
// counts.  The redistribution stages sub-tiles of kSubTile strings in LDS.
constexpr int kWG = 256;                 // threads per workgroup
constexpr int kWaves = kWG / 64;         // wavefronts per workgroup
constexpr uint32_t kMaxTiles = 1024;     // tiles per segment, at most
constexpr uint32_t kSubTile = 2048;      // strings staged at once by the redistribution
constexpr uint32_t kChunkRows = 64;      // count-matrix rows per column-scan chunk
constexpr int kDMax = 10;                // tree depth limit: v <= 1023 splitters
// values of the larger (low) digit of a bucket id in the two-pass distribution
constexpr uint32_t kDigitMax = 1u << ((kDMax + 2) / 2);
constexpr uint32_t kLcpFlag = 0x80000000u;  // out_lcp entry still to be completed
constexpr uint32_t kBufBit = 0x80000000u;   // work-buffer bit packed into a depth

// classification variants (Section 3.1, "Implementation Details"): "Unroll"
// descends every level without branches and tests equality once at the leaf;
// "Equal" tests equality at every node and stops at the first equal splitter
// "Jump" is the Unroll descent started from a jump table over the top key
// bits (appendix A, "Jump tables"); its table has 4 (v + 1) entries per tree
constexpr uint32_t kClassifyUnroll = 0, kClassifyEqual = 1, kClassifyJump = 2;
constexpr uint32_t kJumpPerTreeSlot = 4;

// status-word bits (device side capacity checks)
constexpr uint32_t kErrLargeCap = 1u, kErrBaseCap = 2u, kErrTileCap = 4u, kErrCmCap = 8u,
                   kErrTreeCap = 16u;
// an argument the device checks is invalid (an offset at or past chars_len, an
// arena whose last byte is not a terminator, a set table that is not
// non-decreasing or ends past n): reported as S5_ERR_INVALID
constexpr uint32_t kErrArgs = 32u;
// a byte outside the alphabet of a sort with packed keys (alphabet
// compression): the host sorts again with byte keys
constexpr uint32_t kErrAlphabet = 64u;

// A bucket that still has to be sorted.
struct Seg {
    uint32_t begin;  // first position in the work arrays
    uint32_t size;   // number of strings
    uint32_t depth;  // common prefix length of all its strings (bit 31: work buffer for base items)
    uint32_t base;   // first index of the set the strings belong to
};

// A segment distributed in the current pass, with its per-pass storage.
struct LSeg {
    uint32_t begin, size, depth, base;
    uint32_t d, v, k, tile_len;     // tree depth, splitters (2^d-1), buckets (2v+1), strings per tile
    uint32_t tiles, tile_base;      // tiles and first tile id
    uint32_t chunks, chunk_base;    // column-scan chunks and first chunk id
    uint32_t tree_base, bstart_base;
    uint32_t pad0;                  // learned-splitter slot, or 0xFFFFFFFF for sampled splitters
    uint32_t redo_tune;             // kRedoBit: redo with sampled splitters (exact learned
                                    // check); the other bits: the set's pack_set_tune word
    unsigned long long cm_base;     // tiles x k count matrix (row-major)
    unsigned long long cs_base;     // chunks x k chunk sums / prefixes
};
constexpr uint32_t kRedoBit = 0x80000000u;  // (pack_set_tune leaves bit 31 clear)

// Counters written by one planning step and read back by the host.
// Every workgroup of the planning step adds to these counters with one atomic
// each.  Device-scope atomics on one 128-byte line are serialized (≈12 ns
// each, measured); on different lines they proceed in parallel, so each
// counter that many workgroups update has a line of its own.
#define S5_LINE alignas(128)
struct Counters {
    S5_LINE uint32_t n_large;
    S5_LINE uint32_t tiles;
    S5_LINE uint32_t chunks;
    S5_LINE uint32_t tree;
    S5_LINE uint32_t bstart;
    S5_LINE uint32_t kmax;
    S5_LINE uint32_t pad0;  // learned segments planned
    uint32_t pad1;
    S5_LINE unsigned long long cm;
    S5_LINE unsigned long long cs;
    S5_LINE unsigned long long moved;       // strings in the planned large segments
    S5_LINE unsigned long long max_bucket;  // largest bucket seen by the planning step
    S5_LINE double entropy_sum;             // sum over buckets of |b| log2(|S|/|b|)
};

// Device-global state that survives the whole sort.
// Base-case items go to one of four lists by size: <= 64 strings (one
// wavefront each, in registers), <= 256 (a one-wavefront workgroup), <= 512
// (two wavefronts) and <= T (four wavefronts, eight for T > 1024), so that
// small items hold little LDS and many of them are in flight on a compute unit.
constexpr int kBaseClasses = 4;
constexpr uint32_t kBaseWave = 64, kBaseSmall = 256, kBaseMid = 512;
__host__ __device__ inline int base_class(uint32_t size) {
    return size <= kBaseWave ? 0 : (size <= kBaseSmall ? 1 : (size <= kBaseMid ? 2 : 3));
}

struct Globals {
    S5_LINE uint32_t n_base[kBaseClasses];  // base-case items appended so far, per class
    uint32_t status;                        // error bits
    S5_LINE unsigned long long base_elems;  // strings in those items
    S5_LINE uint32_t fallbacks;             // learned segments redone with sampled splitters
    uint32_t late_fallbacks;        // those of them rejected only on the exact histogram
    // statistics kept on the device by graph-captured sorts (no per-pass readback)
    uint32_t passes, pad;
    unsigned long long moved, segments;        // sums over the passes
    unsigned long long moved0, max_bucket0;    // first pass
    double entropy_sum0;
    // learned proposals: how many, and the largest range bucket of each one's
    // own sample in thousandths of the ideal share m / (v + 1) (sum and maximum)
    S5_LINE uint32_t learned_props, imb_max_milli;
    unsigned long long imb_sum_milli;
    // strings of distributed segments that all fell into one bucket (moved
    // only to advance their depth), summed over the passes
    S5_LINE unsigned long long one_bucket;
    // the largest first key of a sample of the strings and the complement of
    // the smallest (both start at zero), and whether the key cache found a
    // string without their common prefix
    S5_LINE unsigned long long pre_max, pre_cmin;
    uint32_t pre_bad, pre_pad;
};

// Bytes that the sampled strings share at their start (byte keys): the
// common prefix of the smallest and largest sampled first key (0 without a
// sample).
__device__ inline uint32_t sample_prefix(const Globals* g) {
    const unsigned long long mx = g->pre_max, mn = ~g->pre_cmin;
    return mn > mx ? 0u : lcp8(mn, mx);
}

// Depth of every root segment: the sampled common prefix, unless some string
// lacks it (the key cache then holds keys at depth 0).
__device__ inline uint32_t root_depth(const Globals* g) {
    return g->pre_bad ? 0u : sample_prefix(g);
}

// Learned splitters apply to segments of at least this many strings.
constexpr uint32_t kLearnMin = 65536;
constexpr uint32_t kLearnM = 4096;    // sampled keys per learned segment, at most
constexpr uint32_t kLearnGrp = 256;   // samples per training workgroup (one per thread)

// Learned-splitter state of all learned segments of one pass (one slot each).
struct LearnCtx {
    uint64_t* samples;  // [slot][kLearnM] sorted sampled keys
    float* W;           // [slot][2][stride] weights, double-buffered by step parity
    float* M1;          // [slot][2][stride] Adam first moments
    float* M2;          // [slot][2][stride] Adam second moments
    float* part;        // [slot][2][groups][stride] partial gradients of the workgroups
    uint64_t* range;    // [slot][2] byte-wise minimum and maximum of the sample
    uint32_t m;         // samples per slot (multiple of kLearnGrp, <= kLearnM)
    uint32_t groups;    // m / kLearnGrp
};

// Capacities of the per-pass storage.
struct Caps {
    uint32_t large, tiles, chunks, tree, bstart, base[kBaseClasses];
    unsigned long long cm, cs;
};

// Launch mode of one pass kernel: host-driven (cnt == nullptr, the grid is
// the work read back by the host) or graph mode (a fixed grid striding over
// the device count at cnt, clamped to cap).
struct Dyn {
    const uint32_t* cnt = nullptr;
    uint32_t cap = 0;
    uint32_t grid = 0;
};

// Everything a planning step needs to append work.
struct PlanCtx {
    const uint64_t* set_begin;  // first string of every set (with per-set tuning)
    const uint32_t* set_tune;   // packed per-set parameters, or nullptr
    uint32_t num_sets;
    LSeg* lseg;           // next pass's segment list
    Counters* cnt;        // next pass's counters
    Seg* base_list[kBaseClasses];  // base-case items (all passes), per size class
    Globals* glob;
    Caps caps;
    uint32_t* learn_seg;  // learned slot -> next pass's segment index
    uint32_t learn;       // 1: learned splitters for segments >= kLearnMin
    uint32_t learn_cap;   // learned slots available
    uint32_t T;           // base threshold
    uint32_t d_max;       // tree depth limit for this sort
    uint32_t tile_min;    // minimum strings per tile
    uint32_t stats;       // 1: accumulate bucket entropy and max bucket (first pass only)
    KeyCodec kc;          // characters per key and the end-of-string test
};

// Per-set parameters of a batched sort, packed in one word: base threshold T
// (bits 0..11), tree depth limit (bits 12..15), minimum tile / 64 (bits 16..31).
__host__ __device__ inline uint32_t pack_set_tune(uint32_t T, uint32_t d_max, uint32_t tile_min) {
    return (T & 0xFFFu) | ((d_max & 0xFu) << 12) | ((tile_min / 64u) << 16);
}

// Planning parameters of one set: base threshold, tree depth limit, minimum tile.
struct SetP {
    uint32_t T, d_max, tile_min;
};

__host__ __device__ inline SetP unpack_set_tune(uint32_t w) {
    return SetP{w & 0xFFFu, (w >> 12) & 0xFu, (w >> 16) * 64u};
}

__host__ __device__ inline SetP default_set_params(const PlanCtx& c) {
    return SetP{c.T, c.d_max, c.tile_min};
}

// tree depth and tiles of a large segment of `size` strings
__host__ __device__ __forceinline__ void seg_shape(uint32_t size, const SetP& c, uint32_t& d,
                                                   uint32_t& ulen, uint32_t& tiles, uint32_t& chunks) {
    d = 1;
    while (d < c.d_max && ((uint64_t)c.T << d) < 2ull * size) ++d;  // 2^d * T/2 >= size
    ulen = (uint32_t)(((uint64_t)size + kMaxTiles - 1) / kMaxTiles);
    ulen = (ulen + 63u) & ~63u;
    if (ulen < c.tile_min) ulen = c.tile_min;
    tiles = (uint32_t)(((uint64_t)size + ulen - 1) / ulen);
    chunks = (tiles + kChunkRows - 1) / kChunkRows;
}

// Parameters of a segment's set: carried in its record (no search of the sets).
// The word is kept in a vector register: the planning kernel's scalar
// registers are all taken.
__device__ inline SetP seg_set_params(const PlanCtx& c, const LSeg& g) {
    if (!c.set_tune) return default_set_params(c);
    uint32_t w = g.redo_tune & ~kRedoBit;
    asm volatile("" : "+v"(w));
    return unpack_set_tune(w);
}


// Writes of the sort's outputs (out_perm, out_lcp) go through S5_OUT.  The
// write-check build (S5_COUNT_WRITES) also counts, per output slot, how often
// it is written, and counts writes that land in neither output; the product
// build compiles S5_OUT to the plain store.
struct WriteCount {
    uint32_t* perm_base;  // the sort's out_perm and out_lcp
    uint32_t* lcp_base;
    uint32_t* perm_cnt;   // n counters each (null: counting off)
    uint32_t* lcp_cnt;
    uint32_t* stray;      // one counter: writes outside both outputs
    unsigned long long n;
};
#ifdef S5_COUNT_WRITES
extern __device__ WriteCount g_wc;
__device__ inline void wc_note(const uint32_t* p) {
    const WriteCount w = g_wc;
    if (!w.perm_cnt) return;
    if (p >= w.perm_base && p < w.perm_base + w.n)
        atomicAdd(&w.perm_cnt[p - w.perm_base], 1u);
    else if (p >= w.lcp_base && p < w.lcp_base + w.n)
        atomicAdd(&w.lcp_cnt[p - w.lcp_base], 1u);
    else
        atomicAdd(w.stray, 1u);
}
#define S5_OUT(slot, value)                \
    do {                                   \
        uint32_t* s5p_ = &(slot);          \
        *s5p_ = (value);                   \
        ::s5::wc_note(s5p_);               \
    } while (0)
#else
#define S5_OUT(slot, value) ((slot) = (value))
#endif

// Work units of one launch.  A host-driven launch sizes its grid to the work
// (wcnt == nullptr: the grid is the count).  A graph-captured launch reads the
// count from a counter written by an earlier kernel, clamps it to the storage
// capacity, and does nothing once the status word holds an error or while
// *guard is non-zero.  One thread reads and broadcasts it, so every wavefront
// of the block runs the same number of iterations.
__device__ inline uint32_t block_work_count(const uint32_t* wcnt, uint32_t cap,
                                            const Globals* glob, uint32_t grid_units,
                                            const uint32_t* guard = nullptr) {
    if (!wcnt) return grid_units;
    __shared__ uint32_t s_units;
    if (threadIdx.x == 0) {
        uint32_t u = 0;
        if (!glob->status && !(guard && *guard)) {
            u = *wcnt;
            if (u > cap) u = cap;
        }
        s_units = u;
    }
    __syncthreads();
    return s_units;
}

}  // namespace s5
