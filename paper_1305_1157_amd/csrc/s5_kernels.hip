// HIP kernels of super scalar string sample sort (S^5) for gfx950.
//
// Method: Bingmann & Sanders, "Parallel String Sample Sort", Section 3.1.
// Strings are classified by their next w = 8 characters, packed big-endian
// into one 64-bit key (Section 2.2 "caching of characters", "super-alphabets";
// Section 3.1 "as many characters as fit into a machine word").  A perfect
// binary tree of v = 2^d - 1 splitters, stored in level order, is descended
// without branches (i := 2i + [key > x_i]); one equality test against the
// in-order splitter array then yields one of k = 2v + 1 buckets, the odd ones
// being equality buckets (Figure 1).  Classification stores each string's
// bucket number (the paper's "oracle", here the bucket-id array), counts,
// prefix-sums, and redistributes out of place into a second work array whose
// role swaps with the first on recursion (Section 3.1, parallelization).
// Buckets keep their common prefix length (b_0, b_2v), gain lcp of the
// neighbouring splitters (other even buckets) or gain w (equality buckets).
//
// GPU mapping, per distribution pass over all large segments at once:
//   k_sample_tree  one workgroup per segment: sample, sort, recursive
//                  splitter selection, level-order/in-order arrays, splitter LCPs
//   k_classify     one wavefront per unit of a segment: unrolled, interleaved
//                  descents over coalesced keys; bucket ids; per-wavefront
//                  histograms in LDS summed into the unit's row
//   k_colscan      exclusive scan down each bucket column of the count matrix,
//                  within chunks of 64 unit rows
//   k_bucket_plan  one workgroup per segment: chunk prefixes, bucket starts,
//                  and the plan of every bucket (finished / base case / next pass)
//   k_scatter      stable redistribution of (key, second key word, index); keys
//                  of buckets whose depth grows are advanced from the carried
//                  words or refreshed from the arena on the way; buckets that
//                  are finished write their final output directly
//   (two-pass distribution: k_digit_count, k_colscan and k_digit_starts per
//   digit of the bucket ids, then k_scatter by the low digit, and the same
//   by the high digit)
// followed, once every bucket is small, by k_base_sort (LDS sorter that emits
// LCPs) and k_lcp_fix (LCPs at bucket boundaries).
#include <hip/hip_ext.h>

#include "s5_internal.h"
#include "s5_launch.h"
#include "s5_word.h"

namespace s5 {

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

// Lanes of `active` whose bucket equals this lane's bucket b (b < 2^nbits).
__device__ __forceinline__ uint64_t match_bucket(uint32_t b, uint32_t nbits, uint64_t active) {
    uint64_t m = active;
    for (uint32_t i = 0; i < nbits; ++i) {
        bool bit = (b >> i) & 1u;
        uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// block-wide exclusive scan of cnt[0..count) into out[0..count), count <= 8 * kWG;
// `tmp` holds kWG + 1 words.  Returns the total.  All threads must call.
__device__ uint32_t block_exclusive_scan(const uint32_t* cnt, uint32_t* out, uint32_t count,
                                         uint32_t* tmp) {
    const uint32_t per = (count + kWG - 1) / kWG;
    const uint32_t b0 = threadIdx.x * per;
    uint32_t s = 0;
    for (uint32_t i = 0; i < per; ++i)
        if (b0 + i < count) s += cnt[b0 + i];
    tmp[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over kWG partial sums
    for (uint32_t off = 1; off < (uint32_t)kWG; off <<= 1) {
        uint32_t v = threadIdx.x >= off ? tmp[threadIdx.x - off] : 0u;
        __syncthreads();
        tmp[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = threadIdx.x ? tmp[threadIdx.x - 1] : 0u;
    uint32_t total = tmp[kWG - 1];
    for (uint32_t i = 0; i < per; ++i)
        if (b0 + i < count) {
            uint32_t c = cnt[b0 + i];
            out[b0 + i] = run;
            run += c;
        }
    __syncthreads();
    return total;
}

// ---------------------------------------------------------------------------
// planning: decide what happens to every bucket of >= 2 strings.  Every thread
// adds up the requests of its buckets in registers (PlanAcc); a block-wide
// exclusive scan turns them into each thread's offsets and the block's totals;
// one global allocation per counter and block turns the totals into bases; the
// threads then hand out slots from base + offset.  (Contended LDS atomics on a
// few counters cost tens of microseconds per workgroup; the scan costs about
// one.)

// 32-bit counters of a plan, by index; 64-bit ones below
constexpr int kPU_Base = 0;                   // kBaseClasses counters: base items per class
constexpr int kPU_Large = kBaseClasses;       // large segments
constexpr int kPU_Tiles = kBaseClasses + 1;
constexpr int kPU_Chunks = kBaseClasses + 2;
constexpr int kPU_Tree = kBaseClasses + 3;    // tree slots (v + 1 per segment)
constexpr int kPU_Bstart = kBaseClasses + 4;  // bucket-start slots (k + 1 per segment)
constexpr int kPU_Learn = kBaseClasses + 5;   // learned-splitter slots
constexpr int kPU = kBaseClasses + 6;
constexpr int kPQ_Cm = 0, kPQ_Cs = 1, kPQ_Moved = 2, kPQ_BaseElems = 3, kPQ = 4;

struct PlanAcc {
    uint32_t u[kPU];
    unsigned long long q[kPQ];
    uint32_t kmax;
};

// block totals, then (after plan_allocate) global bases
struct PlanTally {
    PlanAcc a;
    uint32_t err;
};

__device__ __forceinline__ void acc_clear(PlanAcc& a) {
#pragma unroll
    for (int i = 0; i < kPU; ++i) a.u[i] = 0;
#pragma unroll
    for (int i = 0; i < kPQ; ++i) a.q[i] = 0;
    a.kmax = 0;
}

// Count one request (a bucket of size >= 2 that needs sorting).
__device__ __forceinline__ void plan_count(uint32_t size, const PlanCtx& c, const SetP& sp,
                                           PlanAcc& a) {
    if (size <= sp.T) {
        const int cls = base_class(size);
#pragma unroll
        for (int i = 0; i < kBaseClasses; ++i) a.u[kPU_Base + i] += cls == i ? 1u : 0u;
        a.q[kPQ_BaseElems] += size;
        return;
    }
    uint32_t d, ulen, tiles, chunks;
    seg_shape(size, sp, d, ulen, tiles, chunks);
    const uint32_t v = (1u << d) - 1, k = 2 * v + 1;
    a.u[kPU_Large] += 1;
    a.u[kPU_Tiles] += tiles;
    a.u[kPU_Chunks] += chunks;
    a.u[kPU_Tree] += v + 1;
    a.u[kPU_Bstart] += k + 1;
    a.q[kPQ_Cm] += (unsigned long long)tiles * k;
    a.q[kPQ_Cs] += (unsigned long long)chunks * k;
    a.q[kPQ_Moved] += size;
    a.kmax = k > a.kmax ? k : a.kmax;
    if (c.learn && size >= kLearnMin) a.u[kPU_Learn] += 1;
}

__device__ __forceinline__ unsigned long long shfl_up_u64(unsigned long long v, uint32_t d) {
    const uint32_t lo = __shfl_up((uint32_t)v, d), hi = __shfl_up((uint32_t)(v >> 32), d);
    return ((unsigned long long)hi << 32) | lo;
}

// Block-wide: a (this thread's counts) becomes its exclusive prefix over the
// threads before it; T->a receives the block totals and T->err is cleared.
// All threads of the block call; the block has kWG threads (kWaves
// wavefronts, a compile-time count, so that every wavefront's totals are
// read from LDS at once rather than one dependent read after another).
__device__ void plan_scan(PlanAcc& a, PlanTally* T) {
    __shared__ PlanAcc ws[kWaves];
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    constexpr uint32_t nw = kWaves;
    PlanAcc inc = a;
    for (uint32_t o = 1; o < 64; o <<= 1) {
#pragma unroll
        for (int i = 0; i < kPU; ++i) {
            const uint32_t x = __shfl_up(inc.u[i], o);
            if (lane >= o) inc.u[i] += x;
        }
#pragma unroll
        for (int i = 0; i < kPQ; ++i) {
            const unsigned long long x = shfl_up_u64(inc.q[i], o);
            if (lane >= o) inc.q[i] += x;
        }
        const uint32_t x = __shfl_up(inc.kmax, o);
        if (lane >= o && x > inc.kmax) inc.kmax = x;
    }
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    // field by field: offsets of the waves before this one, and block totals
#pragma unroll
    for (int i = 0; i < kPU; ++i) {
        uint32_t pre = 0, tot = 0;
#pragma unroll
        for (uint32_t qw = 0; qw < nw; ++qw) {
            const uint32_t x = ws[qw].u[i];
            pre += qw < w ? x : 0u;
            tot += x;
        }
        a.u[i] = pre + inc.u[i] - a.u[i];
        if (threadIdx.x == 0) T->a.u[i] = tot;
    }
#pragma unroll
    for (int i = 0; i < kPQ; ++i) {
        unsigned long long pre = 0, tot = 0;
#pragma unroll
        for (uint32_t qw = 0; qw < nw; ++qw) {
            const unsigned long long x = ws[qw].q[i];
            pre += qw < w ? x : 0ull;
            tot += x;
        }
        a.q[i] = pre + inc.q[i] - a.q[i];
        if (threadIdx.x == 0) T->a.q[i] = tot;
    }
    if (threadIdx.x == 0) {
        uint32_t mx = 0;
#pragma unroll
        for (uint32_t qw = 0; qw < nw; ++qw) mx = ws[qw].kmax > mx ? ws[qw].kmax : mx;
        T->a.kmax = mx;
        T->err = 0;
    }
    __syncthreads();
}

// By the 64 lanes of wavefront 0: turn the block totals in T into global
// bases (stored back into T).  Each lane owns one global counter, so the
// block's atomics are independent and in flight together; every counter that
// many workgroups update sits on a cache line of its own.
__device__ void plan_allocate(const PlanCtx& c, PlanTally* T) {
    constexpr uint32_t kLane = 8;  // first lane of the next pass's counters
    const uint32_t l = threadIdx.x;
    PlanAcc& a = T->a;
    const uint32_t nl = a.u[kPU_Large];
    uint32_t err = 0;
    if (l == 0) {
        if (a.q[kPQ_BaseElems]) atomicAdd(&c.glob->base_elems, a.q[kPQ_BaseElems]);
    } else if (l <= (uint32_t)kBaseClasses) {  // lanes 1..kBaseClasses: base lists
        const int q = (int)l - 1;
        const uint32_t nb = a.u[kPU_Base + q];
        if (nb) {
            const uint32_t b0 = atomicAdd(&c.glob->n_base[q], nb);
            if (b0 + nb > c.caps.base[q]) err = kErrBaseCap;
            a.u[kPU_Base + q] = b0;
        }
    } else if (nl) {
        switch (l) {
            case kLane + 0: {
                const uint32_t x = atomicAdd(&c.cnt->n_large, nl);
                if (x + nl > c.caps.large) err = kErrLargeCap;
                a.u[kPU_Large] = x;
            } break;
            case kLane + 1: {
                const uint32_t v = a.u[kPU_Tiles], x = atomicAdd(&c.cnt->tiles, v);
                if (x + v > c.caps.tiles) err = kErrTileCap;
                a.u[kPU_Tiles] = x;
            } break;
            case kLane + 2: {
                const uint32_t v = a.u[kPU_Chunks], x = atomicAdd(&c.cnt->chunks, v);
                if (x + v > c.caps.chunks) err = kErrTileCap;
                a.u[kPU_Chunks] = x;
            } break;
            case kLane + 3: {
                const uint32_t v = a.u[kPU_Tree], x = atomicAdd(&c.cnt->tree, v);
                if (x + v > c.caps.tree) err = kErrTreeCap;
                a.u[kPU_Tree] = x;
            } break;
            case kLane + 4: {
                const uint32_t v = a.u[kPU_Bstart], x = atomicAdd(&c.cnt->bstart, v);
                if (x + v > c.caps.bstart) err = kErrTreeCap;
                a.u[kPU_Bstart] = x;
            } break;
            case kLane + 5: {
                const unsigned long long v = a.q[kPQ_Cm], x = atomicAdd(&c.cnt->cm, v);
                if (x + v > c.caps.cm) err = kErrCmCap;
                a.q[kPQ_Cm] = x;
            } break;
            case kLane + 6: {
                const unsigned long long v = a.q[kPQ_Cs], x = atomicAdd(&c.cnt->cs, v);
                if (x + v > c.caps.cs) err = kErrCmCap;
                a.q[kPQ_Cs] = x;
            } break;
            case kLane + 7: atomicAdd(&c.cnt->moved, a.q[kPQ_Moved]); break;
            case kLane + 8: atomicMax(&c.cnt->kmax, a.kmax); break;
            case kLane + 9: {
                const uint32_t v = a.u[kPU_Learn];
                a.u[kPU_Learn] = v ? atomicAdd(&c.cnt->pad0, v) : 0u;
            } break;
            default: break;
        }
    }
    if (err) {
        atomicOr(&T->err, err);
        atomicOr(&c.glob->status, err);
    }
}

// Write the record of one request; slots come from the global bases in T plus
// this thread's running offsets `off` (its exclusive prefix, advanced here).
__device__ void plan_emit(uint32_t begin, uint32_t size, uint32_t depth, uint32_t base,
                          uint32_t buf, const PlanCtx& c, const SetP& sp, const PlanTally* T,
                          PlanAcc& off) {
    const PlanAcc& g0 = T->a;
    if (size <= sp.T) {
        const int q = base_class(size);
        uint32_t o = 0;  // this thread's next offset in class q (unrolled: no indexed registers)
#pragma unroll
        for (int i = 0; i < kBaseClasses; ++i)
            if (q == i) o = off.u[kPU_Base + i]++;
        const uint32_t slot = g0.u[kPU_Base + q] + o;
        Seg s;
        s.begin = begin;
        s.size = size;
        s.depth = depth | (buf ? kBufBit : 0u);
        s.base = base;
        c.base_list[q][slot] = s;
        return;
    }
    uint32_t d, ulen, tiles, chunks;
    seg_shape(size, sp, d, ulen, tiles, chunks);
    const uint32_t v = (1u << d) - 1, k = 2 * v + 1;
    LSeg g;
    g.begin = begin;
    g.size = size;
    g.depth = depth;
    g.base = base;
    g.d = d;
    g.v = v;
    g.k = k;
    g.tile_len = ulen;
    g.tiles = tiles;
    g.tile_base = g0.u[kPU_Tiles] + off.u[kPU_Tiles];
    off.u[kPU_Tiles] += tiles;
    g.chunks = chunks;
    g.chunk_base = g0.u[kPU_Chunks] + off.u[kPU_Chunks];
    off.u[kPU_Chunks] += chunks;
    g.tree_base = g0.u[kPU_Tree] + off.u[kPU_Tree];
    off.u[kPU_Tree] += v + 1;
    g.bstart_base = g0.u[kPU_Bstart] + off.u[kPU_Bstart];
    off.u[kPU_Bstart] += k + 1;
    g.pad0 = 0xFFFFFFFFu;
    g.redo_tune = pack_set_tune(sp.T, sp.d_max, sp.tile_min);
    g.cm_base = g0.q[kPQ_Cm] + off.q[kPQ_Cm];
    off.q[kPQ_Cm] += (unsigned long long)tiles * k;
    g.cs_base = g0.q[kPQ_Cs] + off.q[kPQ_Cs];
    off.q[kPQ_Cs] += (unsigned long long)chunks * k;
    const uint32_t slot = g0.u[kPU_Large] + off.u[kPU_Large]++;
    if (c.learn && size >= kLearnMin) {
        const uint32_t ls = g0.u[kPU_Learn] + off.u[kPU_Learn]++;
        if (ls < c.learn_cap) {  // beyond the cap the segment keeps sampled splitters
            g.pad0 = ls;
            c.learn_seg[ls] = slot;
        }
    }
    c.lseg[slot] = g;
}

// the code table of a packed sort in LDS (every thread of the block calls;
// a barrier follows before first use)
#define S5_CODE_TABLE(PK, kc, tab)                                  \
    const uint8_t* tab = nullptr;                                   \
    if constexpr (PK) {                                             \
        __shared__ uint8_t ctab_[256];                              \
        for (uint32_t c_ = threadIdx.x; c_ < 256; c_ += blockDim.x) \
            ctab_[c_] = (kc).table[c_];                             \
        tab = ctab_;                                                \
    }

// ---------------------------------------------------------------------------
// K1: prefix cache at depth 0 (and the building-block entry point)

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
    uint32_t lo = __shfl_xor((uint32_t)v, m), hi = __shfl_xor((uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

// The common start of the strings, estimated from a sample of up to
// kPrefixSamples strings, one per thread: the largest sampled first key and
// the complement of the smallest (one atomic each per workgroup).  The key
// cache checks every string against their common prefix.
constexpr uint32_t kPrefixSamples = 64 * kWG;
__global__ __launch_bounds__(256) void k_prefix_sample(const uint8_t* chars, uint64_t chars_len,
                                                       const uint64_t* offsets, uint32_t n,
                                                       Globals* glob) {
    const uint32_t S = n < kPrefixSamples ? n : kPrefixSamples;
    unsigned long long mx = 0, cmin = 0;
    for (uint32_t j = blockIdx.x * kWG + threadIdx.x; j < S; j += gridDim.x * kWG) {
        const uint64_t off = offsets[(uint32_t)(((uint64_t)j * n) / S)];
        if (chars_len && off >= chars_len) continue;  // rejected by the key cache
        const uint64_t k = load_key(chars, off);
        mx = k > mx ? k : mx;
        cmin = ~k > cmin ? ~k : cmin;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long a = shfl_xor64(mx, o), b = shfl_xor64(cmin, o);
        mx = a > mx ? a : mx;
        cmin = b > cmin ? b : cmin;
    }
    __shared__ unsigned long long smx[kWaves], scm[kWaves];
    if (lane_id() == 0) {
        smx[threadIdx.x >> 6] = mx;
        scm[threadIdx.x >> 6] = cmin;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWaves; ++w) {
            mx = smx[w] > mx ? smx[w] : mx;
            cmin = scm[w] > cmin ? scm[w] : cmin;
        }
        if (mx) atomicMax(&glob->pre_max, mx);
        if (cmin) atomicMax(&glob->pre_cmin, cmin);
    }
}

// Key cache of string i with its keys at depth d0 (byte keys only for
// d0 > 0): the string must start with the first d0 bytes of `pfx`, else the
// flag pre_bad is raised (the keys of every string are then loaded again at
// depth 0).  The first d0 + 24 bytes come from one run of aligned words.
template <bool PK>
__device__ __forceinline__ void init_one(uint32_t i, const uint8_t* chars, uint64_t chars_len,
                                         const uint64_t* offsets, uint64_t* key, uint64_t* key2,
                                         uint64_t* key3, uint32_t* idx, Globals* glob,
                                         const KeyCodec& kc, const uint8_t* tab, uint32_t d0,
                                         uint64_t pfx) {
    idx[i] = i;
    const uint64_t off = offsets[i];
    if (chars_len) {
        // with the arena's length known: every string starts inside it and the
        // arena ends with a terminator, so every string ends inside it
        const bool bad = off >= chars_len || (i == 0 && chars[chars_len - 1] != 0);
        if (bad) {
            atomicOr(&glob->status, kErrArgs);
            key[i] = 0;
            key2[i] = 0;
            return;
        }
    }
    uint64_t w[3];
    if constexpr (PK) {
        uint64_t raw[8];
        load_key_run<8>(chars, off, raw);
        if (pack3<8, 3>(tab, raw, w)) atomicOr(kc.status, kErrAlphabet);
    } else if (d0 == 0) {
        load_key_run<3>(chars, off, w);
    } else {
        uint64_t r[4];
        load_key_run<4>(chars, off, r);
        const bool ok = d0 == 8 ? r[0] == pfx : ((r[0] ^ pfx) >> (64 - 8 * d0)) == 0;
        if (!ok) {
            atomicOr(&glob->pre_bad, 1u);
            return;
        }
#pragma unroll
        for (int j = 0; j < 3; ++j)
            w[j] = d0 == 8 ? r[j + 1] : (r[j] << (8 * d0)) | (r[j + 1] >> (64 - 8 * d0));
    }
    key[i] = w[0];
    key2[i] = w[1];
    // the third word is all zero (and never read) unless the string
    // continues past its first two keys
    if (!(PK ? codec_has_end(kc, w[1]) : has_zero(w[1]))) key3[i] = w[2];
}

template <bool PK>
__global__ __launch_bounds__(256) void k_init_keys(const uint8_t* chars, uint64_t chars_len,
                                                   const uint64_t* offsets, uint32_t n,
                                                   uint64_t* key, uint64_t* key2, uint64_t* key3,
                                                   uint32_t* idx, Globals* glob, KeyCodec kc) {
    S5_CODE_TABLE(PK, kc, tab)
    if constexpr (PK) __syncthreads();
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // byte keys start at the sampled common prefix (checked string by string)
    const uint32_t d0 = PK ? 0u : sample_prefix(glob);
    init_one<PK>(i, chars, chars_len, offsets, key, key2, key3, idx, glob, kc, tab, d0,
                 ~glob->pre_cmin);
}

// Byte keys again at depth 0, only if some string lacked the sampled prefix
// (grid-stride over the strings; every other launch exits at once).
__global__ __launch_bounds__(256) void k_init_redo(const uint8_t* chars, uint64_t chars_len,
                                                   const uint64_t* offsets, uint32_t n,
                                                   uint64_t* key, uint64_t* key2, uint64_t* key3,
                                                   uint32_t* idx, Globals* glob, KeyCodec kc) {
    if (!glob->pre_bad) return;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        init_one<false>(i, chars, chars_len, offsets, key, key2, key3, idx, glob, kc, nullptr, 0u,
                        0ull);
}

__global__ __launch_bounds__(256) void k_prefix_keys(const uint8_t* chars, const uint64_t* offsets,
                                                     uint32_t n, uint32_t depth, uint64_t* key) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = load_key(chars, offsets[i] + depth);
}

// Root segments: one per set (or the whole input).  Sizes 0 and 1 are done here.
__global__ __launch_bounds__(256) void k_plan_roots(const uint64_t* set_begin, uint32_t num_sets,
                                                    uint32_t n, uint32_t* out_perm,
                                                    uint32_t* out_lcp, PlanCtx ctx) {
    __shared__ PlanTally T;
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t b = 0, e = 0;
    if (s < num_sets) {
        const uint64_t b64 = set_begin ? set_begin[s] : 0u, e64 = set_begin ? set_begin[s + 1] : n;
        if (b64 > e64 || e64 > n) {
            // not a non-decreasing table within n: nothing of this set is written
            atomicOr(&ctx.glob->status, kErrArgs);
        } else {
            b = (uint32_t)b64;
            e = (uint32_t)e64;
        }
        if (e > b) {
            S5_OUT(out_lcp[b], 0u);
            if (e - b == 1) S5_OUT(out_perm[b], 0u);
        }
    }
    const bool req = e > b + 1;
    const SetP sp = (ctx.set_tune && s < num_sets) ? unpack_set_tune(ctx.set_tune[s])
                                                   : default_set_params(ctx);
    PlanAcc acc;
    acc_clear(acc);
    if (req) plan_count(e - b, ctx, sp, acc);
    plan_scan(acc, &T);
    if (threadIdx.x < 64) plan_allocate(ctx, &T);
    __syncthreads();
    if (T.err) return;
    // every string of every set starts with the root depth's bytes
    if (req) plan_emit(b, e - b, ctx.kc.b == 8 ? root_depth(ctx.glob) : 0u, b, 0, ctx, sp, &T, acc);
}

// Graph-captured sorts keep their statistics on the device: after each pass,
// add the pass's totals (and the first pass's bucket statistics).
__global__ void k_pass_stats(const Counters* cur, const Counters* next, Globals* glob,
                             uint32_t level) {
    if (threadIdx.x != 0 || glob->status || !cur->n_large) return;
    glob->passes += 1;
    glob->moved += cur->moved;
    glob->segments += cur->n_large;
    if (level == 0) {
        glob->moved0 = cur->moved;
        glob->max_bucket0 = next->max_bucket;
        glob->entropy_sum0 = next->entropy_sum;
    }
}

// zero n words (a kernel, so that graph captures hold no memset nodes)
__global__ void k_zero_words(uint32_t* p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Copy `words` words of counters into pinned host memory, release them to
// the system, then raise *flag to `seq` (one wavefront).  The host polls the
// flag instead of waiting for a copy and an event, and the kernels queued
// after this one start at once.
constexpr uint32_t kPublishWords = 1024;  // at most (all loads in flight together)
__global__ __launch_bounds__(64) void k_publish(const uint32_t* src, uint32_t words,
                                                uint32_t* dst, uint32_t* flag, uint32_t seq) {
    constexpr uint32_t R = kPublishWords / 64;
    uint32_t v[R];
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        const uint32_t i = threadIdx.x + 64 * r;
        v[r] = i < words ? src[i] : 0u;
    }
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        const uint32_t i = threadIdx.x + 64 * r;
        if (i < words) dst[i] = v[r];
    }
    // the release orders every lane's stores of this wavefront before the flag
    if (threadIdx.x == 0)
        __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ---------------------------------------------------------------------------
// K2: sample, sort the sample, select splitters recursively, build the tree

__device__ __forceinline__ void sample_tree_body(uint32_t slot, uint32_t redo, const LSeg* lseg,
                                                 const uint64_t* key_in, uint32_t alpha,
                                                 uint64_t seed, uint64_t* tree_lo,
                                                 uint64_t* tree_in, uint8_t* tree_lcp,
                                                 uint16_t* jump, uint32_t* tile_tab,
                                                 uint32_t* chunk_tab, const KeyCodec& kc) {
    extern __shared__ uint64_t smp[];  // sample, padded to a power of two
    __shared__ uint32_t ra[1u << kDMax], rb[1u << kDMax];
    __shared__ uint64_t t[1u << kDMax];
    const LSeg g = lseg[slot];
    const uint32_t tid = threadIdx.x;
    if (!redo) {
        for (uint32_t u = tid; u < g.tiles; u += kWG) tile_tab[g.tile_base + u] = slot;
        for (uint32_t c = tid; c < g.chunks; c += kWG) chunk_tab[g.chunk_base + c] = slot;
    } else if (!(g.redo_tune & kRedoBit)) {
        return;  // only segments whose learned splitters failed are redone
    }
    if (g.pad0 != 0xFFFFFFFFu) return;  // learned splitters: the tree comes from the model
    const uint32_t m = alpha * (g.v + 1) - 1;
    uint32_t P = 1;
    while (P < m) P <<= 1;
    // pseudo-random sample of m keys (Section 3.1: alpha = 2 oversampling)
    const uint64_t sseed = mix64(seed ^ mix64(((uint64_t)g.begin << 32) | g.depth));
    for (uint32_t r = tid; r < P; r += kWG) {
        uint64_t x = ~0ull;
        if (r < m) {
            uint64_t h = mix64(sseed + 0x9E3779B97F4A7C15ull * (r + 1));
            uint32_t off = (uint32_t)(((h >> 32) * (uint64_t)g.size) >> 32);
            x = key_in[g.begin + off];
        }
        smp[r] = x;
    }
    __syncthreads();
    // bitonic sort of the sample in LDS
    for (uint32_t kk = 2; kk <= P; kk <<= 1) {
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
            for (uint32_t i = tid; i < P / 2; i += kWG) {
                uint32_t lo = 2 * i - (i & (j - 1)), hi = lo + j;
                bool up = (lo & kk) == 0;
                uint64_t a = smp[lo], b = smp[hi];
                if ((a > b) == up) {
                    smp[lo] = b;
                    smp[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    // recursive selection (Section 3.1): the middle sample of a range is the
    // node's splitter; the children recurse on the parts left and right of the
    // run of samples equal to it.  An empty range repeats the parent's key.
    if (tid == 0) {
        ra[1] = 0;
        rb[1] = m;
    }
    __syncthreads();
    for (uint32_t L = 0; L < g.d; ++L) {
        for (uint32_t i = (1u << L) + tid; i < (2u << L); i += kWG) {
            uint32_t a = ra[i], b = rb[i];
            uint64_t x;
            uint32_t lo = 0, hi = 0;
            if (a < b) {
                select_node(smp, a, b, &x, &lo, &hi);
            } else {
                x = t[i >> 1];
            }
            t[i] = x;
            if (L + 1 < g.d) {
                ra[2 * i] = a < b ? a : 0;
                rb[2 * i] = a < b ? lo : 0;
                ra[2 * i + 1] = a < b ? hi : 0;
                rb[2 * i + 1] = a < b ? b : 0;
            }
        }
        __syncthreads();
    }
    uint64_t* lo_out = tree_lo + g.tree_base;
    uint64_t* in_out = tree_in + g.tree_base;
    uint8_t* lcp_out = tree_lcp + g.tree_base;
    for (uint32_t i = tid; i <= g.v; i += kWG) {
        lo_out[i] = i ? t[i] : 0ull;
        if (i < g.v) {
            uint64_t x = t[inorder_node(i, g.d)];
            in_out[i] = x;
            uint8_t l = 0;
            if (i > 0) {
                uint64_t p = t[inorder_node(i - 1, g.d)];
                l = p == x ? 0 : (uint8_t)codec_lcp(kc, p, x);
            }
            lcp_out[i] = l;
        } else {
            in_out[i] = 0;
            lcp_out[i] = 0;
        }
    }
    if (jump) build_jump_table(t, g.d, g.v, jump + (uint64_t)g.tree_base * kJumpPerTreeSlot,
                               threadIdx.x, blockDim.x);
}

// One workgroup per segment (G: grid-stride over a device count, graph mode).
// redo = 1: only segments flagged by the exact learned-splitter check.
template <bool G>
__global__ __launch_bounds__(256) void k_sample_tree(const LSeg* lseg, const uint64_t* key_in,
                                                     uint32_t alpha, uint64_t seed,
                                                     uint64_t* tree_lo, uint64_t* tree_in,
                                                     uint8_t* tree_lcp, uint16_t* jump,
                                                     uint32_t* tile_tab, uint32_t* chunk_tab,
                                                     Counters* next_cnt, const uint32_t* wcnt,
                                                     uint32_t cap, const Globals* glob,
                                                     uint32_t redo, KeyCodec kc) {
    // the next pass's counters are planned later in this pass: clear them here
    if (!redo && blockIdx.x == 0)
        for (uint32_t i = threadIdx.x; i < sizeof(Counters) / 4; i += blockDim.x)
            ((uint32_t*)next_cnt)[i] = 0;
    if (!G) {
        sample_tree_body(blockIdx.x, redo, lseg, key_in, alpha, seed, tree_lo, tree_in, tree_lcp,
                         jump, tile_tab, chunk_tab, kc);
        return;
    }
    const uint32_t units = block_work_count(wcnt, cap, glob, gridDim.x);
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
        sample_tree_body(u, redo, lseg, key_in, alpha, seed, tree_lo, tree_in, tree_lcp, jump,
                         tile_tab, chunk_tab, kc);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// K3: classification + per-tile histogram.  The workgroup walks its tile in
// steps of kWG * U strings; every wavefront classifies U chunks of 64 coalesced
// keys at once and counts them in its own LDS histogram (ballot match, the
// lowest lane of each group adds).  The per-wavefront histograms are summed
// into the tile's row of the count matrix.

// The Equal variant for U interleaved keys: level by level, every descent not
// yet finished tests its node for equality and steps down; the wavefront
// leaves the tree as soon as none of its descents is still going (so inputs
// with many keys equal to splitters near the root stop early).
template <int U>
__device__ __forceinline__ void classify_equal_u(const uint64_t* t, uint32_t d,
                                                 const uint64_t (&key)[U], uint32_t (&b)[U]) {
    uint32_t i[U];
    bool done[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
        i[q] = 1;
        done[q] = false;
        b[q] = 0;
    }
    for (uint32_t L = 0; L < d; ++L) {
        bool going = false;
#pragma unroll
        for (int q = 0; q < U; ++q) {
            equal_step(t, d, key[q], i[q], done[q], b[q]);
            going = going || !done[q];
        }
        if (!__ballot(going)) break;
    }
#pragma unroll
    for (int q = 0; q < U; ++q)
        if (!done[q]) b[q] = equal_leaf_bucket(i[q], d);
}

// The Jump variant: every descent starts at its jump-table entry (keys outside
// the splitter range at their leaf), then descends like Unroll; the
// wavefront stops once all its descents have reached the leaves.
template <int U>
__device__ __forceinline__ void classify_jump_u(const uint64_t* t, const uint64_t* tin,
                                                const uint16_t* jt, uint32_t d, uint32_t v,
                                                const uint64_t (&key)[U], uint32_t (&b)[U]) {
    const uint64_t first = tin[0], last = tin[v - 1];
    const JumpShape js = jump_shape(first, last, d);
    const uint32_t leaf0 = 1u << d;
    uint32_t i[U];
#pragma unroll
    for (int q = 0; q < U; ++q)
        i[q] = key[q] < first ? leaf0 : (key[q] > last ? leaf0 + v : jt[jump_index(key[q], js)]);
    for (uint32_t L = 0; L < d; ++L) {
        bool going = false;
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const bool g = i[q] < leaf0;
            const uint64_t x = t[g ? i[q] : 0u];
            i[q] = g ? 2u * i[q] + (key[q] > x ? 1u : 0u) : i[q];
            going = going || g;
        }
        if (!__ballot(going)) break;
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
        const uint32_t j = i[q] - leaf0;
        b[q] = 2u * j + ((j < v && tin[j] == key[q]) ? 1u : 0u);
    }
}

template <int U, int VAR>
__device__ __forceinline__ void classify_keys(const uint64_t* t, const uint64_t* tin,
                                              const uint16_t* jt, uint32_t d, uint32_t v,
                                              const uint64_t (&kk)[U], uint32_t (&b)[U]) {
    if (VAR == (int)kClassifyEqual)
        classify_equal_u<U>(t, d, kk, b);
    else if (VAR == (int)kClassifyJump)
        classify_jump_u<U>(t, tin, jt, d, v, kk, b);
    else
        classify_u<U>(t, tin, d, v, kk, b);
}

template <int U, int VAR>
__device__ __forceinline__ void classify_body(uint32_t tile, uint32_t redo, const LSeg* lseg,
                                              const uint32_t* tile_tab, const uint64_t* key_in,
                                              const uint64_t* tree_lo, const uint64_t* tree_in,
                                              const uint16_t* jump, uint16_t* bid, uint32_t* cm,
                                              uint32_t vmax, uint32_t kmax) {
    extern __shared__ uint64_t dyn[];
    uint64_t* t = dyn;
    uint64_t* tin = t + (vmax + 1);
    uint32_t* hist = (uint32_t*)(tin + (vmax + 1));  // kWaves * kmax
    uint16_t* jt = (uint16_t*)(hist + kWaves * kmax);  // Jump: kJumpPerTreeSlot (vmax + 1)
    const LSeg g = lseg[tile_tab[tile]];
    if (redo && !(g.redo_tune & kRedoBit)) return;
    for (uint32_t i = threadIdx.x; i <= g.v; i += kWG) {
        t[i] = tree_lo[g.tree_base + i];
        tin[i] = tree_in[g.tree_base + i];
    }
    if (VAR == (int)kClassifyJump) {
        const JumpShape js = jump_shape(tree_in[g.tree_base], tree_in[g.tree_base + g.v - 1], g.d);
        const uint16_t* src = jump + (uint64_t)g.tree_base * kJumpPerTreeSlot;
        for (uint32_t p = threadIdx.x; p < (1u << js.a); p += kWG) jt[p] = src[p];
    }
    for (uint32_t b = threadIdx.x; b < g.k; b += kWG) {
#pragma unroll
        for (int q = 0; q < kWaves; ++q) hist[q * kmax + b] = 0;
    }
    __syncthreads();
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    uint32_t* h = hist + w * kmax;
    const uint32_t row = tile - g.tile_base;
    const uint64_t tb = (uint64_t)row * g.tile_len;
    const uint32_t start = g.begin + (uint32_t)(tb < g.size ? tb : g.size);
    const uint32_t end = g.begin + (uint32_t)(tb + g.tile_len < g.size ? tb + g.tile_len : g.size);
    for (uint32_t c = start + w * 64 * U; c < end; c += kWG * U) {
        uint64_t kk[U];
        uint32_t b[U];
        bool valid[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const uint32_t pos = c + q * 64 + lane;
            valid[q] = pos < end;
            kk[q] = valid[q] ? key_in[pos] : 0ull;
        }
        classify_keys<U, VAR>(t, tin, jt, g.d, g.v, kk, b);
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const uint32_t pos = c + q * 64 + lane;
            if (valid[q]) bid[pos] = (uint16_t)b[q];
            const uint64_t act = __ballot(valid[q]);
            if (!act) continue;
            // the wavefront's own histogram: one add when every key of the
            // chunk falls into one bucket (skewed inputs), else an LDS add per
            // key (spread buckets rarely collide within an instruction)
            const int lead = __ffsll((long long)act) - 1;
            const uint32_t b0 = (uint32_t)__builtin_amdgcn_readlane((int)b[q], lead);
            if (__ballot(valid[q] && b[q] == b0) == act) {
                if (lane == (uint32_t)lead) h[b0] += (uint32_t)__popcll(act);
            } else if (valid[q]) {
                atomicAdd(&h[b[q]], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t* out = cm + g.cm_base + (uint64_t)row * g.k;
    for (uint32_t b = threadIdx.x; b < g.k; b += kWG) {
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) s += hist[q * kmax + b];
        out[b] = s;
    }
}

template <int U, bool G, int VAR>
__global__ __launch_bounds__(256) void k_classify(const LSeg* lseg, const uint32_t* tile_tab,
                                                  const uint64_t* key_in, const uint64_t* tree_lo,
                                                  const uint64_t* tree_in, const uint16_t* jump,
                                                  uint16_t* bid, uint32_t* cm, uint32_t vmax,
                                                  uint32_t kmax, const uint32_t* wcnt,
                                                  uint32_t cap, const Globals* glob,
                                                  uint32_t redo) {
    if (!G) {
        classify_body<U, VAR>(blockIdx.x, redo, lseg, tile_tab, key_in, tree_lo, tree_in, jump,
                              bid, cm, vmax, kmax);
        return;
    }
    const uint32_t units = block_work_count(wcnt, cap, glob, gridDim.x);
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
        classify_body<U, VAR>(u, redo, lseg, tile_tab, key_in, tree_lo, tree_in, jump, bid, cm,
                              vmax, kmax);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// K4a: exclusive scan down every bucket column within a chunk of unit rows

// dig: the columns are those of a digit of the bucket ids (two-pass
// distribution) instead of the buckets
__device__ __forceinline__ void colscan_body(uint32_t cg, uint32_t redo, const LSeg* lseg,
                                             const uint32_t* chunk_tab, uint32_t* cm,
                                             uint32_t* cs, uint32_t dig) {
    const LSeg g = lseg[chunk_tab[cg]];
    if (redo && !(g.redo_tune & kRedoBit)) return;
    const uint32_t b = blockIdx.y * kWG + threadIdx.x;
    const uint32_t kc = digit_values(g.k, g.d, dig);
    if (b >= kc) return;
    const uint32_t c = cg - g.chunk_base;
    const uint32_t r0 = c * kChunkRows;
    const uint32_t r1 = r0 + kChunkRows < g.tiles ? r0 + kChunkRows : g.tiles;
    uint32_t run = 0;
    uint32_t* col = cm + g.cm_base + b;
    // 16 rows at a time: their loads are in flight together
    for (uint32_t r = r0; r < r1; r += 16) {
        const uint32_t m = r1 - r < 16 ? r1 - r : 16u;
        uint32_t x[16];
#pragma unroll
        for (uint32_t i = 0; i < 16; ++i) x[i] = i < m ? col[(uint64_t)(r + i) * kc] : 0u;
#pragma unroll
        for (uint32_t i = 0; i < 16; ++i)
            if (i < m) {
                col[(uint64_t)(r + i) * kc] = run;
                run += x[i];
            }
    }
    cs[g.cs_base + (uint64_t)c * kc + b] = run;
}

template <bool G>
__global__ __launch_bounds__(256) void k_colscan(const LSeg* lseg, const uint32_t* chunk_tab,
                                                 uint32_t* cm, uint32_t* cs, const uint32_t* wcnt,
                                                 uint32_t cap, const Globals* glob, uint32_t redo,
                                                 uint32_t dig) {
    if (!G) {
        colscan_body(blockIdx.x, redo, lseg, chunk_tab, cm, cs, dig);
        return;
    }
    const uint32_t units = block_work_count(wcnt, cap, glob, gridDim.x);
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x)
        colscan_body(u, redo, lseg, chunk_tab, cm, cs, dig);
}

// ---------------------------------------------------------------------------
// K4b: chunk prefixes, bucket starts, and the plan of every bucket

// Column b of a segment's chunk sums (kc columns): the exclusive prefix down
// the chunks, written back, and the column's total in tot[b].  16 chunks'
// loads are in flight at once.
__device__ __forceinline__ void chunk_prefixes(const LSeg& g, uint32_t* cs, uint32_t kc,
                                               uint32_t* tot) {
    for (uint32_t b = threadIdx.x; b < kc; b += kWG) {
        uint32_t run = 0;
        uint32_t* col = cs + g.cs_base + b;
        for (uint32_t c = 0; c < g.chunks; c += 16) {
            const uint32_t m = g.chunks - c < 16 ? g.chunks - c : 16u;
            uint32_t x[16];
#pragma unroll
            for (uint32_t i = 0; i < 16; ++i) x[i] = i < m ? col[(uint64_t)(c + i) * kc] : 0u;
#pragma unroll
            for (uint32_t i = 0; i < 16; ++i)
                if (i < m) {
                    col[(uint64_t)(c + i) * kc] = run;
                    run += x[i];
                }
        }
        tot[b] = run;
    }
}

// s0 (the column's start in the segment) added to every chunk prefix of column b
__device__ __forceinline__ void add_column_start(const LSeg& g, uint32_t* cs, uint32_t kc,
                                                 uint32_t b, uint32_t s0) {
    uint32_t* col = cs + g.cs_base + b;
    for (uint32_t c = 0; c < g.chunks; c += 16) {
        const uint32_t m = g.chunks - c < 16 ? g.chunks - c : 16u;
        uint32_t x[16];
#pragma unroll
        for (uint32_t i = 0; i < 16; ++i) x[i] = i < m ? col[(uint64_t)(c + i) * kc] : 0u;
#pragma unroll
        for (uint32_t i = 0; i < 16; ++i)
            if (i < m) col[(uint64_t)(c + i) * kc] = x[i] + s0;
    }
}

__device__ __forceinline__ void add_starts(const LSeg& g, uint32_t* cs, uint32_t kc,
                                           const uint32_t* st) {
    for (uint32_t b = threadIdx.x; b < kc; b += kWG) add_column_start(g, cs, kc, b, st[b]);
}

__device__ __forceinline__ void bucket_plan_body(uint32_t seg, const LSeg* lseg, uint32_t* cs,
                                                 uint32_t* bstart, const uint64_t* tree_in,
                                                 const uint8_t* tree_lcp, const PlanCtx& ctx,
                                                 uint32_t next_buf, uint32_t kmax) {
    // per bucket (kmax entries each, dynamic LDS): sizes, starts, new depths
    extern __shared__ uint32_t plan_lds[];
    uint32_t* tot = plan_lds;
    uint32_t* st = tot + kmax;
    uint32_t* ndl = st + kmax;
    __shared__ uint32_t tmp[kWG + 1];
    const LSeg g = lseg[seg];
    const SetP sp = seg_set_params(ctx, g);
    const uint32_t k = g.k;
    chunk_prefixes(g, cs, k, tot);
    __syncthreads();
    block_exclusive_scan(tot, st, k, tmp);
    uint32_t* bs = bstart + g.bstart_base;
    double ent = 0.0;
    unsigned long long mx = 0;
    __shared__ PlanTally T;
    for (uint32_t b = threadIdx.x; b < k; b += kWG) {
        const uint32_t s0 = st[b];
        bs[b] = s0;
        add_column_start(g, cs, k, b, s0);
        const uint32_t sz = tot[b];
        if (sz == 0 || !ctx.stats) continue;
        ent += (double)sz * log2((double)g.size / (double)sz);
        if (sz > mx) mx = sz;
    }
    if (threadIdx.x == 0) bs[k] = g.size;
    {  // a segment whose strings all fell into one bucket
        int one = 0;
        for (uint32_t b = threadIdx.x; b < k; b += kWG) one |= tot[b] == g.size ? 1 : 0;
        if (__syncthreads_or(one) && threadIdx.x == 0)
            atomicAdd(&ctx.glob->one_bucket, (unsigned long long)g.size);
    }
    if (ctx.stats) {
        // block-reduce the statistics, then one atomic each per block
        __shared__ double s_ent;
        __shared__ unsigned long long s_mx;
        if (threadIdx.x == 0) {
            s_ent = 0.0;
            s_mx = 0;
        }
        __syncthreads();
        for (uint32_t o = 32; o > 0; o >>= 1) {
            ent += __shfl_xor(ent, (int)o);
            const unsigned long long om = __shfl_xor(mx, (int)o);
            mx = om > mx ? om : mx;
        }
        if (lane_id() == 0) {
            atomicAdd(&s_ent, ent);
            atomicMax(&s_mx, mx);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            if (s_mx) atomicMax(&ctx.cnt->max_bucket, s_mx);
            if (s_ent != 0.0) atomicAdd(&ctx.cnt->entropy_sum, s_ent);
        }
    }
    // new depth of bucket b, or 0xFFFFFFFF if it needs no further sorting
    // (empty, a single string, or an equality bucket whose splitter ends the
    // strings: all its strings are identical and the scatter finishes them)
    auto next_depth = [&](uint32_t b) -> uint32_t {
        const uint32_t sz = tot[b];
        if (sz < 2) return 0xFFFFFFFFu;
        const uint32_t j = b >> 1;
        if (b & 1u) {
            if (codec_has_end(ctx.kc, tree_in[g.tree_base + j])) return 0xFFFFFFFFu;
            return g.depth + ctx.kc.w;
        }
        return g.depth + ((j == 0 || j == g.v) ? 0u : (uint32_t)tree_lcp[g.tree_base + j]);
    };
    // every thread counts, then emits, its buckets b = tid, tid + kWG, ... in
    // the same order (their new depths kept in LDS: loops stay rolled)
    PlanAcc acc;
    acc_clear(acc);
    for (uint32_t b = threadIdx.x; b < k; b += kWG) {
        const uint32_t nd = next_depth(b);
        ndl[b] = nd;
        if (nd != 0xFFFFFFFFu) plan_count(tot[b], ctx, sp, acc);
    }
    plan_scan(acc, &T);
    if (threadIdx.x < 64) plan_allocate(ctx, &T);
    __syncthreads();
    if (T.err) return;
    for (uint32_t b = threadIdx.x; b < k; b += kWG) {
        const uint32_t nd = ndl[b];
        if (nd != 0xFFFFFFFFu)
            plan_emit(g.begin + st[b], tot[b], nd, g.base, next_buf, ctx, sp, &T, acc);
    }
}

template <bool G>
__global__ __launch_bounds__(256) void k_bucket_plan(const LSeg* lseg, uint32_t* cs,
                                                     uint32_t* bstart, const uint64_t* tree_in,
                                                     const uint8_t* tree_lcp, PlanCtx ctx,
                                                     uint32_t next_buf, const uint32_t* wcnt,
                                                     uint32_t cap, uint32_t kmax) {
    if (!G) {
        bucket_plan_body(blockIdx.x, lseg, cs, bstart, tree_in, tree_lcp, ctx, next_buf, kmax);
        return;
    }
    const uint32_t units = block_work_count(wcnt, cap, ctx.glob, gridDim.x);
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
        bucket_plan_body(u, lseg, cs, bstart, tree_in, tree_lcp, ctx, next_buf, kmax);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Packed keys (alphabet compression): one or two keys of 21 characters at
// chars[pos], characters mapped through the LDS code table `tab`; a byte
// outside the alphabet sets kErrAlphabet (the host then sorts again with
// byte keys).  Reads the same words load_key_run reads.
struct SchedFence {
    __device__ void operator()() const { __builtin_amdgcn_sched_barrier(0); }
};
__device__ __forceinline__ uint64_t packed_load1(const KeyCodec& kc, const uint8_t* tab,
                                                 const uint8_t* chars, uint64_t pos) {
    uint64_t raw[3], k[1];
    load_key_run<3>(chars, pos, raw);
    if (pack3<3, 1>(tab, raw, k, SchedFence())) atomicOr(kc.status, kErrAlphabet);
    return k[0];
}
__device__ __forceinline__ void packed_load2(const KeyCodec& kc, const uint8_t* tab,
                                             const uint8_t* chars, uint64_t pos, uint64_t* k0,
                                             uint64_t* k1) {
    uint64_t raw[6], k[2];
    load_key_run<6>(chars, pos, raw);
    if (pack3<6, 2>(tab, raw, k, SchedFence())) atomicOr(kc.status, kErrAlphabet);
    *k0 = k[0];
    *k1 = k[1];
}

// ---------------------------------------------------------------------------
// K5: stable redistribution (Section 3.1, out-of-place into the second work
// array).  A tile is processed in sub-tiles of kSubTile strings:
//   A. every wavefront loads its 512 strings (8 chunks of 64, in order),
//      advances the two key words of buckets whose depth grows (from the words
//      themselves when they hold the bytes -- in the first pass always, with
//      the third word from init -- else a 16-byte gather from the arena), and
//      ranks them by bucket with ballots into its own LDS counters;
//   B. per bucket: prefix over the wavefronts and the bucket's start inside the
//      sub-tile (block-wide scan over the buckets);
//   C. every string is staged in LDS at its rank in bucket order;
//   D. consecutive threads write consecutive staged strings, i.e. contiguous
//      runs per bucket, to their final places.  Buckets that need no further
//      sorting write the output permutation (and the LCPs inside an equality
//      bucket of identical strings) directly; every bucket start gets its
//      boundary depth flagged in out_lcp.
constexpr uint32_t kPerWave = kSubTile / kWaves;  // strings per wavefront per sub-tile
constexpr int kChunks = (int)(kPerWave / 64);     // chunks of 64 per wavefront

// bucket / rank word of a lane that holds no string (never a (bucket << 16 | rank))
constexpr uint32_t kNoString = 0xFFFFFFFFu;

// per-bucket byte: mode in bits 5..6, depth increase in characters (0..w,
// w <= 21) in bits 0..4
constexpr uint32_t kModeLive = 0, kModeSingle = 1, kModeIdentical = 2;
constexpr uint32_t kModeShift = 5, kDeltaMask = 31;

// exclusive block-wide sum of one value per thread; `wl` holds kWaves words
__device__ uint32_t block_excl_add(uint32_t v, uint32_t* wl, uint32_t* total) {
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t inc = v;
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const uint32_t x = __shfl_up(inc, o);
        if (lane >= o) inc += x;
    }
    if (lane == 63) wl[w] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
        if ((uint32_t)q < w) pre += wl[q];
        tot += wl[q];
    }
    *total = tot;
    __syncthreads();
    return pre + inc - v;
}

// Slots are ranked by "rank buckets": the bucket itself (DIG = 0, one move per
// level), or one digit of it in the two-pass distribution (DIG = kDigitLow:
// keys advanced and everything moved, bucket ids included, into the other
// arrays by the low digit; DIG = kDigitHigh: moved back by the high digit,
// which leaves every bucket in place, and finished there as with DIG = 0).
// krmax: LDS entries of the rank-bucket counters.
template <int DIG>
__host__ __device__ constexpr uint32_t scatter_krmax(uint32_t kmax) {
    return DIG ? kDigitMax : kmax;
}

template <bool K3, bool PK, int DIG>
__device__ __forceinline__ void scatter_body(
    uint32_t tile, const LSeg* lseg, const uint32_t* tile_tab, const uint16_t* bid,
    const uint64_t* key_in, const uint64_t* key2_in, const uint32_t* idx_in, uint64_t* key_out,
    uint64_t* key2_out, uint32_t* idx_out, const uint32_t* cm, const uint32_t* cs, const uint32_t* bstart, const uint64_t* tree_in,
    const uint8_t* tree_lcp, const uint8_t* chars, const uint64_t* offsets, uint32_t* out_perm,
    uint32_t* out_lcp, uint32_t vmax, uint32_t kmax, const uint64_t* key3, const KeyCodec& kc,
    uint16_t* bid_out) {
    static_assert(DIG == 0 || !K3 || DIG == (int)kDigitLow, "the third word is read where keys advance");
    extern __shared__ uint64_t dyn[];
    const uint32_t krmax = scatter_krmax<DIG>(kmax);
    uint64_t* SK = dyn;                                   // kSubTile staged keys
    uint32_t* SI = (uint32_t*)(SK + kSubTile);            // kSubTile staged indices
    uint32_t* base = SI + kSubTile;                       // krmax: next slot of each rank bucket
    uint32_t* bst = base + krmax;                         // kmax: bucket starts in the segment
    uint16_t* SB = (uint16_t*)(bst + kmax);               // kSubTile staged buckets
    uint16_t* whist = SB + kSubTile;                      // kWaves * krmax per-wave counts
    uint16_t* tstart = whist + kWaves * krmax;            // krmax + 1: starts in the sub-tile
    uint8_t* binfo = (uint8_t*)(tstart + (krmax + 1));    // kmax: mode | depth increase
    uint8_t* ident = binfo + kmax;                        // kmax: LCP inside identical buckets
    __shared__ uint32_t wl[kWaves];
    (void)vmax;
    const uint8_t* tab = nullptr;  // packed keys: the code table in LDS
    if constexpr (PK) {
        __shared__ uint8_t ctab[256];
        ctab[threadIdx.x] = kc.table[threadIdx.x];
        tab = ctab;
    }

    const LSeg g = lseg[tile_tab[tile]];
    const uint32_t k = g.k, tid = threadIdx.x;
    const uint32_t kr = digit_values(k, g.d, DIG);  // rank buckets (k when DIG = 0)
    const uint32_t row = tile - g.tile_base, chunk = row / kChunkRows;
    if (DIG) {
        for (uint32_t r = tid; r < kr; r += kWG) {
            base[r] = cs[g.cs_base + (uint64_t)chunk * kr + r] + cm[g.cm_base + (uint64_t)row * kr + r];
#pragma unroll
            for (int q = 0; q < kWaves; ++q) whist[q * krmax + r] = 0;
        }
    }
    for (uint32_t b = tid; b < k; b += kWG) {
        const uint32_t s0 = bstart[g.bstart_base + b], s1 = bstart[g.bstart_base + b + 1];
        bst[b] = s0;
        if (!DIG)
            base[b] = cs[g.cs_base + (uint64_t)chunk * k + b] + cm[g.cm_base + (uint64_t)row * k + b];
        const uint32_t j = b >> 1;
        uint32_t info;
        if (s1 - s0 == 1) {
            info = kModeSingle << kModeShift;
        } else if (b & 1u) {
            const uint64_t x = tree_in[g.tree_base + j];
            if (PK ? codec_has_end(kc, x) : has_zero(x)) {
                info = kModeIdentical << kModeShift;
                ident[b] = (uint8_t)(PK ? codec_before_end(kc, x) : nz_bytes(x));
            } else {
                info = PK ? kc.w : 8u;
            }
        } else {
            info = (j == 0 || j == g.v) ? 0u : (uint32_t)tree_lcp[g.tree_base + j];
        }
        binfo[b] = (uint8_t)info;
        if (!DIG) {
#pragma unroll
            for (int q = 0; q < kWaves; ++q) whist[q * krmax + b] = 0;
        }
    }
    __syncthreads();

    const uint32_t w = tid >> 6, lane = lane_id();
    uint16_t* wh = whist + w * krmax;
    const uint64_t ltmask = (1ull << lane) - 1ull;
    const uint32_t nbits = digit_bits(g.d, DIG);
    const uint64_t tb = (uint64_t)row * g.tile_len;
    const uint32_t start = g.begin + (uint32_t)(tb < g.size ? tb : g.size);
    const uint32_t end = g.begin + (uint32_t)(tb + g.tile_len < g.size ? tb + g.tile_len : g.size);
    const uint32_t per = (kr + kWG - 1) / kWG;  // rank buckets per thread in phase B (<= 8)
    const uint32_t b0 = tid * per;

    for (uint32_t sub = start; sub < end; sub += kSubTile) {
        const uint32_t se = sub + kSubTile < end ? sub + kSubTile : end;
        const uint32_t pw = sub + w * kPerWave + lane;
        // A: load, refresh, rank inside the wavefront
        uint64_t nk[kChunks], n2[kChunks], n3[kChunks];
        uint32_t id[kChunks], bb[kChunks];
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            const uint32_t p = pw + c * 64;
            const bool valid = p < se;
            // streamed once per pass: non-temporal, so the cache keeps the gathers' lines
            bb[c] = valid ? __builtin_nontemporal_load(bid + p) : kNoString;
            nk[c] = valid ? __builtin_nontemporal_load(key_in + p) : 0ull;
            n2[c] = valid ? __builtin_nontemporal_load(key2_in + p) : 0ull;
            n3[c] = K3 && valid && !(PK ? codec_has_end(kc, n2[c]) : has_zero(n2[c]))
                        ? __builtin_nontemporal_load(key3 + p)
                        : 0ull;
            id[c] = valid ? __builtin_nontemporal_load(idx_in + p) : 0u;
        }
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            // the two-pass distribution advances the keys in its first move
            if (DIG == (int)kDigitHigh || bb[c] == kNoString) continue;
            const uint32_t info = binfo[bb[c]];
            const uint32_t delta = info & kDeltaMask;
            if ((info >> kModeShift) != kModeLive || delta == 0) continue;
            // the first pass has the third word too (from init): both words
            // stay exact without a gather
            if (K3) {
                if constexpr (PK)
                    codec_advance3(kc, &nk[c], &n2[c], n3[c], delta);
                else
                    advance_key24(&nk[c], &n2[c], n3[c], delta);
            } else if constexpr (PK) {
                // a packed gather brings one key (21 characters); the eight
                // chunks' raw words and lookups would not fit in registers together
                if (!codec_advance2(kc, &nk[c], &n2[c], delta)) {
                    nk[c] = packed_load1(kc, tab, chars, offsets[id[c]] + g.depth + delta);
                    n2[c] = codec_has_end(kc, nk[c]) ? 0ull : kKeyUnknown;
                }
                __builtin_amdgcn_sched_barrier(0);
            } else if (!advance_key16(&nk[c], &n2[c], delta)) {
                load_key16(chars, offsets[id[c]] + g.depth + delta, &nk[c], &n2[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            // a chunk past the sub-tile's end leaves every later chunk kNoString too
            const bool valid = bb[c] != kNoString;
            const uint64_t act = __ballot(valid);
            if (!act) break;
            const uint32_t b = valid ? bb[c] : 0u;
            const uint32_t rb = digit_of(b, g.d, DIG);
            const uint64_t m = match_bucket(rb, nbits, act);
            const uint32_t old = valid ? wh[rb] : 0u;
            if (valid && lane == (uint32_t)(__ffsll((long long)m) - 1))
                wh[rb] = (uint16_t)(old + (uint32_t)__popcll(m));
            bb[c] = valid ? ((b << 16) | (old + (uint32_t)__popcll(m & ltmask))) : kNoString;
        }
        __syncthreads();
        // B: prefix over wavefronts per bucket, then bucket starts inside the sub-tile
        uint32_t tot[8];
        uint32_t mysum = 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t b = b0 + e;
            tot[e] = 0;
            if ((uint32_t)e < per && b < kr) {
                uint32_t r = 0;
#pragma unroll
                for (int q = 0; q < kWaves; ++q) {
                    const uint32_t x = whist[q * krmax + b];
                    whist[q * krmax + b] = (uint16_t)r;
                    r += x;
                }
                tot[e] = r;
                mysum += r;
            }
        }
        uint32_t nsub;
        uint32_t run = block_excl_add(mysum, wl, &nsub);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t b = b0 + e;
            if ((uint32_t)e < per && b < kr) {
                tstart[b] = (uint16_t)run;
                run += tot[e];
            }
        }
        if (tid == 0) tstart[kr] = (uint16_t)nsub;
        __syncthreads();
        // C: stage in bucket order
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            if (bb[c] == kNoString) continue;
            const uint32_t b = bb[c] >> 16, rb = digit_of(b, g.d, DIG);
            const uint32_t s = (uint32_t)tstart[rb] + whist[w * krmax + rb] + (bb[c] & 0xFFFFu);
            SK[s] = nk[c];
            SI[s] = id[c];
            SB[s] = (uint16_t)b;
            // the second key word goes straight to its place (runs of a bucket
            // are consecutive within a chunk)
            if (DIG == (int)kDigitLow || (binfo[b] >> kModeShift) == kModeLive)
                key2_out[g.begin + base[rb] + s - tstart[rb]] = n2[c];
        }
        __syncthreads();
        // D: write contiguous runs
        for (uint32_t s = tid; s < nsub; s += kWG) {
            const uint32_t b = SB[s], rb = digit_of(b, g.d, DIG);
            const uint32_t dr = base[rb] + s - tstart[rb];
            const uint32_t dest = g.begin + dr;
            if (DIG == (int)kDigitLow) {  // everything moves, with its bucket id
                key_out[dest] = SK[s];
                idx_out[dest] = SI[s];
                bid_out[dest] = (uint16_t)b;
                continue;
            }
            const uint32_t s0 = bst[b];
            if (dr == s0 && dr != 0) S5_OUT(out_lcp[dest], kLcpFlag | g.depth);
            const uint32_t mode = binfo[b] >> kModeShift;
            if (mode == kModeLive) {
                key_out[dest] = SK[s];
                idx_out[dest] = SI[s];
            } else {
                S5_OUT(out_perm[dest], SI[s] - g.base);
                if (mode == kModeIdentical && dr != s0) S5_OUT(out_lcp[dest], g.depth + ident[b]);
            }
        }
        __syncthreads();
        // E: advance the tile's bucket bases, clear the counters
        for (uint32_t b = tid; b < kr; b += kWG) {
            base[b] += (uint32_t)tstart[b + 1] - tstart[b];
#pragma unroll
            for (int q = 0; q < kWaves; ++q) whist[q * krmax + b] = 0;
        }
        __syncthreads();
    }
}

// K3: the first pass, which also reads the third key word (a separate
// instantiation, so that the other passes keep their smaller register budget)
template <bool G, bool K3, bool PK, int DIG>
__global__ __launch_bounds__(256) void k_scatter(
    const LSeg* lseg, const uint32_t* tile_tab, const uint16_t* bid, const uint64_t* key_in,
    const uint64_t* key2_in, const uint32_t* idx_in, uint64_t* key_out, uint64_t* key2_out,
    uint32_t* idx_out, const uint32_t* cm, const uint32_t* cs, const uint32_t* bstart,
    const uint64_t* tree_in, const uint8_t* tree_lcp, const uint8_t* chars,
    const uint64_t* offsets, uint32_t* out_perm, uint32_t* out_lcp, uint32_t vmax, uint32_t kmax,
    const uint32_t* wcnt, uint32_t cap, const Globals* glob, const uint64_t* key3,
    KeyCodec kc, uint16_t* bid_out) {
    // neighbouring tiles write adjacent runs of every bucket: on one XCD the
    // partial cache lines where their runs meet are merged in its L2
    if (!G) {
        scatter_body<K3, PK, DIG>(xcd_unit(blockIdx.x, gridDim.x), lseg, tile_tab, bid, key_in,
                                  key2_in, idx_in, key_out, key2_out, idx_out, cm, cs, bstart,
                                  tree_in, tree_lcp, chars, offsets, out_perm, out_lcp, vmax,
                                  kmax, key3, kc, bid_out);
        return;
    }
    const uint32_t units = block_work_count(wcnt, cap, glob, gridDim.x);
    for (uint32_t r0 = 0; r0 + blockIdx.x < units; r0 += gridDim.x) {
        const uint32_t m = units - r0 < gridDim.x ? units - r0 : gridDim.x;
        const uint32_t u = r0 + xcd_unit(blockIdx.x, m);
        scatter_body<K3, PK, DIG>(u, lseg, tile_tab, bid, key_in, key2_in, idx_in, key_out,
                                  key2_out, idx_out, cm, cs, bstart, tree_in, tree_lcp, chars,
                                  offsets, out_perm, out_lcp, vmax, kmax, key3, kc, bid_out);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// K5a/K5b (two-pass distribution): the histogram of one digit of the bucket
// ids per tile (the tile's row of the count matrix, kd columns), and after
// the column scan, every digit's start in its segment added into the chunk
// prefixes -- the counting half of one least-significant-digit pass.
__device__ __forceinline__ void digit_count_body(uint32_t tile, const LSeg* lseg,
                                                 const uint32_t* tile_tab, const uint16_t* bid,
                                                 uint32_t* cm, uint32_t dig) {
    __shared__ uint32_t h[kDigitMax];
    const LSeg g = lseg[tile_tab[tile]];
    const uint32_t kd = digit_values(g.k, g.d, dig);
    for (uint32_t r = threadIdx.x; r < kd; r += kWG) h[r] = 0;
    __syncthreads();
    const uint32_t row = tile - g.tile_base, lane = lane_id();
    const uint64_t tb = (uint64_t)row * g.tile_len;
    const uint32_t start = g.begin + (uint32_t)(tb < g.size ? tb : g.size);
    const uint32_t end = g.begin + (uint32_t)(tb + g.tile_len < g.size ? tb + g.tile_len : g.size);
    for (uint32_t p0 = start + (threadIdx.x & ~63u); p0 < end; p0 += kWG) {
        const uint32_t p = p0 + lane;
        const bool valid = p < end;
        const uint32_t r = valid ? digit_of(bid[p], g.d, dig) : 0u;
        const uint64_t act = __ballot(valid);
        // one add when the chunk's digits are all equal, else one per string
        const int lead = __ffsll((long long)act) - 1;
        const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)r, lead);
        if (__ballot(valid && r == r0) == act) {
            if (lane == (uint32_t)lead) atomicAdd(&h[r0], (uint32_t)__popcll(act));
        } else if (valid) {
            atomicAdd(&h[r], 1u);
        }
    }
    __syncthreads();
    uint32_t* out = cm + g.cm_base + (uint64_t)row * kd;
    for (uint32_t r = threadIdx.x; r < kd; r += kWG) out[r] = h[r];
}

__global__ __launch_bounds__(256) void k_digit_count(const LSeg* lseg, const uint32_t* tile_tab,
                                                     const uint16_t* bid, uint32_t* cm,
                                                     uint32_t dig) {
    digit_count_body(blockIdx.x, lseg, tile_tab, bid, cm, dig);
}

__global__ __launch_bounds__(256) void k_digit_starts(const LSeg* lseg, uint32_t* cs,
                                                      uint32_t dig) {
    __shared__ uint32_t tot[kDigitMax], st[kDigitMax], tmp[kWG + 1];
    const LSeg g = lseg[blockIdx.x];
    const uint32_t kd = digit_values(g.k, g.d, dig);
    chunk_prefixes(g, cs, kd, tot);
    __syncthreads();
    block_exclusive_scan(tot, st, kd, tmp);
    add_starts(g, cs, kd, st);
}

// ---------------------------------------------------------------------------
// K8: base case.  A bucket of n <= T strings that share `depth` leading
// bytes is finished on chip:
//   1. sort by (key, local index); local index order is input order, because
//      every distribution pass is stable;
//   2. neighbours with different keys, or equal keys that hold the
//      terminator, are decided: their LCP is depth + common key bytes;
//   3. maximal runs of undecided neighbours ("groups") are re-keyed 8 bytes
//      deeper and only their members are sorted again, by (group, key, local
//      index) -- the multikey refinement of Section 2.1 -- until every
//      neighbouring pair is decided.
// Buckets of <= 64 strings are finished by one wavefront each, entirely in
// registers (shuffle bitonic network, ballots for the groups).  Larger buckets
// use a workgroup and LDS; once <= 64 strings remain undecided, wavefront 0
// finishes them the same way without further workgroup barriers.

// The sorting networks order elements (key, a = group << 16 | local index) by
// (group, key, local index).  Inside a network an element is the 96-bit number
// group:16 | key:64 | local:16, held as hi = group << 48 | key >> 16 and
// lo = (key & 0xFFFF) << 16 | local, so that one three-word subtraction
// compares two elements (no branches; the compiler turns the three-way
// comparison into divergent control flow with scalar mask logic otherwise).
__device__ __forceinline__ void pack96(uint64_t k, uint32_t a, uint64_t& h, uint32_t& l) {
    h = ((uint64_t)(a >> 16) << 48) | (k >> 16);
    l = ((uint32_t)k << 16) | (a & 0xFFFFu);
}
__device__ __forceinline__ void unpack96(uint64_t h, uint32_t l, uint64_t& k, uint32_t& a) {
    k = (h << 16) | (l >> 16);
    a = ((uint32_t)(h >> 48) << 16) | (l & 0xFFFFu);
}

// (h, l) := (ph, pl) iff ((ph, pl) < (h, l)) != flip  (flip is 0 or 1).
// Vector instructions only: the borrow of (ph, pl) - (h, l) is the comparison.
__device__ __forceinline__ void take96(uint64_t& h, uint32_t& l, uint64_t ph, uint32_t pl,
                                       uint32_t flip) {
    uint32_t h0 = (uint32_t)h, h1 = (uint32_t)(h >> 32), t;
    asm("v_sub_co_u32 %[t], vcc, %[pl], %[l]\n\t"
        "v_subb_co_u32 %[t], vcc, %[ph0], %[h0], vcc\n\t"
        "v_subb_co_u32 %[t], vcc, %[ph1], %[h1], vcc\n\t"
        "v_cndmask_b32_e64 %[t], 0, 1, vcc\n\t"
        "v_cmp_ne_u32 vcc, %[t], %[flip]\n\t"
        "v_cndmask_b32 %[l], %[l], %[pl], vcc\n\t"
        "v_cndmask_b32 %[h0], %[h0], %[ph0], vcc\n\t"
        "v_cndmask_b32 %[h1], %[h1], %[ph1], vcc"
        : [t] "=&v"(t), [l] "+v"(l), [h0] "+v"(h0), [h1] "+v"(h1)
        : [pl] "v"(pl), [ph0] "v"((uint32_t)ph), [ph1] "v"((uint32_t)(ph >> 32)), [flip] "v"(flip)
        : "vcc");
    h = ((uint64_t)h1 << 32) | h0;
}

// (x, y) := (y, x) iff (y < x) != flip: ascending pair for flip 0, descending for 1.
__device__ __forceinline__ void cex96(uint64_t& xh, uint32_t& xl, uint64_t& yh, uint32_t& yl,
                                      uint32_t flip) {
    const uint32_t x0 = (uint32_t)xh, x1 = (uint32_t)(xh >> 32);
    const uint32_t y0 = (uint32_t)yh, y1 = (uint32_t)(yh >> 32);
    uint32_t t, nxl, nx0, nx1, nyl, ny0, ny1;
    asm("v_sub_co_u32 %[t], vcc, %[yl], %[xl]\n\t"
        "v_subb_co_u32 %[t], vcc, %[y0], %[x0], vcc\n\t"
        "v_subb_co_u32 %[t], vcc, %[y1], %[x1], vcc\n\t"
        "v_cndmask_b32_e64 %[t], 0, 1, vcc\n\t"
        "v_cmp_ne_u32 vcc, %[t], %[flip]\n\t"
        "v_cndmask_b32 %[nxl], %[xl], %[yl], vcc\n\t"
        "v_cndmask_b32 %[nx0], %[x0], %[y0], vcc\n\t"
        "v_cndmask_b32 %[nx1], %[x1], %[y1], vcc\n\t"
        "v_cndmask_b32 %[nyl], %[yl], %[xl], vcc\n\t"
        "v_cndmask_b32 %[ny0], %[y0], %[x0], vcc\n\t"
        "v_cndmask_b32 %[ny1], %[y1], %[x1], vcc"
        : [t] "=&v"(t), [nxl] "=&v"(nxl), [nx0] "=&v"(nx0), [nx1] "=&v"(nx1),
          [nyl] "=&v"(nyl), [ny0] "=&v"(ny0), [ny1] "=&v"(ny1)
        : [xl] "v"(xl), [x0] "v"(x0), [x1] "v"(x1), [yl] "v"(yl), [y0] "v"(y0), [y1] "v"(y1),
          [flip] "v"(flip)
        : "vcc");
    xl = nxl;
    xh = ((uint64_t)nx1 << 32) | nx0;
    yl = nyl;
    yh = ((uint64_t)ny1 << 32) | ny0;
}

// bitonic direction: 1 where element e keeps the larger of its pair in the
// stage (j, kk), i.e. where ((e & j) == 0) != ((e & kk) == 0)
__device__ __forceinline__ uint32_t bitonic_flip(uint32_t e, uint32_t j, uint32_t kk) {
    return ((e & j) ? 1u : 0u) ^ ((e & kk) ? 1u : 0u);
}

__device__ __forceinline__ uint64_t shfl_up64(uint64_t v, int d) {
    uint32_t lo = __shfl_up((uint32_t)v, d), hi = __shfl_up((uint32_t)(v >> 32), d);
    return ((uint64_t)hi << 32) | lo;
}

// Bitonic sort of one element per lane over the wavefront.
__device__ __forceinline__ void wave_sort(uint64_t& k, uint32_t& a) {
    const uint32_t lane = lane_id();
    uint64_t h;
    uint32_t l;
    pack96(k, a, h, l);
    for (uint32_t kk = 2; kk <= 64; kk <<= 1) {
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
            const uint64_t ph = shfl_xor64(h, (int)j);
            const uint32_t pl = __shfl_xor(l, (int)j);
            take96(h, l, ph, pl, bitonic_flip(lane, j, kk));
        }
    }
    unpack96(h, l, k, a);
}

// Key operations of the base case for byte keys (PK = false) or packed keys
// (alphabet compression).
template <bool PK>
__device__ __forceinline__ bool key_ends(const KeyCodec& kc, uint64_t k) {
    if constexpr (PK) return codec_has_end(kc, k);
    else return has_zero(k);
}
template <bool PK>
__device__ __forceinline__ uint32_t key_lcp(const KeyCodec& kc, uint64_t a, uint64_t b) {
    if constexpr (PK) return codec_lcp(kc, a, b);
    else return lcp8(a, b);
}
template <bool PK>
__device__ __forceinline__ uint32_t key_chars(const KeyCodec& kc) {
    if constexpr (PK) return kc.w;
    else return 8u;
}
template <bool PK>
__device__ __forceinline__ uint64_t key_load1(const KeyCodec& kc, const uint8_t* tab,
                                              const uint8_t* chars, uint64_t pos) {
    if constexpr (PK) return packed_load1(kc, tab, chars, pos);
    else return load_key(chars, pos);
}
template <bool PK>
__device__ __forceinline__ void key_load2(const KeyCodec& kc, const uint8_t* tab,
                                          const uint8_t* chars, uint64_t pos, uint64_t* k0,
                                          uint64_t* k1) {
    if constexpr (PK) packed_load2(kc, tab, chars, pos, k0, k1);
    else load_key16(chars, pos, k0, k1);
}
// Rounds of decide / re-key / sort inside one wavefront.  Lane r owns output
// position pos; lanes are sorted by (group, key, local index) and padding
// lanes (valid == false) are last.  Returns the final packed element of the lane.
// Refinement rounds of one wavefront (<= 64 elements, sorted by (group, key,
// local index)).  offl[local] holds the string start of element `local` (LDS);
// with fill set, the members fill their own entries (from iin and offsets) on
// the first round that gathers -- later members are among them.  k2 (or
// nullptr): the item's second key words by local index, exact or kKeyUnknown,
// which serve the first re-key without a gather.  A round re-keys the
// undecided members one key deeper; it re-sorts only if some group's keys now
// differ (equal keys keep their local-index order).
template <bool PK>
__device__ uint32_t wave_rounds(uint64_t k, uint32_t a, bool valid, uint32_t h, uint32_t pos,
                                uint64_t* offl, bool fill, const uint64_t* k2,
                                const uint32_t* iin, const uint8_t* chars,
                                const uint64_t* offsets, uint32_t* olcp, const KeyCodec& kc,
                                const uint8_t* tab) {
    const uint32_t lane = lane_id();
    const uint64_t upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    bool filled = !fill;
    for (;;) {
        const uint64_t kp = shfl_up64(k, 1);
        const uint32_t ap = __shfl_up(a, 1);
        bool und = false;
        if (valid && lane > 0 && (ap >> 16) == (a >> 16)) {
            if (kp == k && !key_ends<PK>(kc, k))
                und = true;
            else
                S5_OUT(olcp[pos], h + key_lcp<PK>(kc, kp, k));
        }
        const uint64_t U = __ballot(und);
        if (!U) break;
        const bool member = ((U >> lane) & 1ull) || (lane < 63 && ((U >> (lane + 1)) & 1ull));
        const uint32_t st = 63u - (uint32_t)__builtin_clzll((unsigned long long)(~U & upto));
        const uint32_t l = a & 0xFFFFu;
        const uint64_t x2 = k2 && member ? k2[l] : kKeyUnknown;
        k2 = nullptr;  // only the first re-key is at the second word's depth
        const bool gather = member && x2 == kKeyUnknown;
        if (!filled && __ballot(gather)) {
            if (member) offl[l] = offsets[iin[l]];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            filled = true;
        }
        h += key_chars<PK>(kc);
        if (member) {
            k = gather ? key_load1<PK>(kc, tab, chars, offl[l] + h) : x2;
            a = (st << 16) | l;
        } else if (valid) {
            a = (lane << 16) | (a & 0xFFFFu);
        }
        const uint64_t kq = shfl_up64(k, 1);
        const uint32_t aq = __shfl_up(a, 1);
        const bool split = member && lane > 0 && (aq >> 16) == (a >> 16) && kq != k;
        if (__ballot(split)) wave_sort(k, a);
    }
    return a;
}

template <bool PK>
__device__ __forceinline__ void base_wave_body(uint32_t item, const Seg* items,
                                               const uint64_t* key0, const uint64_t* key1,
                                               const uint64_t* key2_0, const uint64_t* key2_1,
                                               const uint32_t* idx0, const uint32_t* idx1,
                                               const uint8_t* chars, const uint64_t* offsets,
                                               uint32_t* out_perm, uint32_t* out_lcp,
                                               const KeyCodec& kc, const uint8_t* tab) {
    __shared__ uint64_t offl[kWaves][64];  // string starts, by local index
    const uint32_t lane = lane_id();
    const Seg it = items[item];
    const uint32_t buf = it.depth >> 31;
    const uint32_t h = it.depth & ~kBufBit;
    const uint32_t n = it.size;
    const uint64_t* kin = (buf ? key1 : key0) + it.begin;
    const uint64_t* k2in = (buf ? key2_1 : key2_0) + it.begin;
    const uint32_t* iin = (buf ? idx1 : idx0) + it.begin;
    const bool valid = lane < n;
    uint64_t k = valid ? kin[lane] : ~0ull;
    uint32_t a = valid ? lane : 0xFFFFFFFFu;
    wave_sort(k, a);
    const uint32_t fa = wave_rounds<PK>(k, a, valid, h, lane, offl[threadIdx.x >> 6], true, k2in,
                                        iin, chars, offsets, out_lcp + it.begin, kc, tab);
    if (valid) S5_OUT(out_perm[it.begin + lane], iin[fa & 0xFFFFu] - it.base);
}

// One wavefront per item (items are wavefront-uniform; no workgroup barriers).
template <bool G, bool PK>
__global__ __launch_bounds__(256) void k_base_wave(const Seg* items, uint32_t n_items,
                                                   const uint64_t* key0, const uint64_t* key1,
                                                   const uint64_t* key2_0, const uint64_t* key2_1,
                                                   const uint32_t* idx0, const uint32_t* idx1,
                                                   const uint8_t* chars, const uint64_t* offsets,
                                                   uint32_t* out_perm, uint32_t* out_lcp,
                                                   const uint32_t* wcnt, uint32_t cap,
                                                   const Globals* glob, const uint32_t* guard,
                                                   KeyCodec kc) {
    S5_CODE_TABLE(PK, kc, tab)
    if constexpr (PK) __syncthreads();
    if (!G) {
        const uint32_t it = blockIdx.x * kWaves + (threadIdx.x >> 6);
        if (it < n_items)  // uniform per wavefront
            base_wave_body<PK>(it, items, key0, key1, key2_0, key2_1, idx0, idx1, chars, offsets,
                               out_perm, out_lcp, kc, tab);
        return;
    }
    const uint32_t units = block_work_count(wcnt, cap, glob, n_items, guard);
    for (uint32_t it = blockIdx.x * kWaves + (threadIdx.x >> 6); it < units;
         it += gridDim.x * kWaves)
        base_wave_body<PK>(it, items, key0, key1, key2_0, key2_1, idx0, idx1, chars, offsets,
                           out_perm, out_lcp, kc, tab);
}

template <int E, int J>
__device__ __forceinline__ void cex_local(uint64_t (&h)[E], uint32_t (&l)[E], uint32_t t,
                                          uint32_t kk) {
#pragma unroll
    for (int s = 0; s < E; ++s) {
        if ((s & J) == 0) {
            const int s2 = s | J;
            cex96(h[s], l[s], h[s2], l[s2], ((t * E + s) & kk) ? 1u : 0u);
        }
    }
}

// Sort SK/SA[0..P) ascending, P a power of two, P / E <= NT.  All NT threads call.
// Each thread holds E consecutive elements in registers.  A stage whose
// partner is another thread of the same wavefront exchanges by cross-lane
// shuffles; only partners in other wavefronts go through LDS (with barriers).
template <int E, int NT>
__device__ __forceinline__ void block_bitonic(uint64_t* SK, uint32_t* SA, uint32_t P) {
    const uint32_t t = threadIdx.x;
    const bool act = t * E < P;
    // packed elements (see pack96); the partner of an active thread is active,
    // so inactive threads may run the network on padding
    uint64_t h[E];
    uint32_t l[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
        if (act)
            pack96(SK[t * E + s], SA[t * E + s], h[s], l[s]);
        else
            h[s] = ~0ull, l[s] = ~0u;
    }
    for (uint32_t kk = 2; kk <= P; kk <<= 1) {
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
            if (j >= (uint32_t)E && j / E < 64u) {
                // partner thread t ^ (j / E) is in this wavefront; with j >= E
                // the direction is the same for the thread's E elements
                const uint32_t m = j / E, fl = bitonic_flip(t * E, j, kk);
#pragma unroll
                for (int s = 0; s < E; ++s) {
                    const uint64_t ph = shfl_xor64(h[s], (int)m);
                    const uint32_t pl = __shfl_xor(l[s], (int)m);
                    take96(h[s], l[s], ph, pl, fl);
                }
            } else if (j >= (uint32_t)E) {
                // exchange through LDS; slot s of thread t lives at t*E + ((s + t) mod E)
                // so that the lanes of one access hit distinct banks
                __syncthreads();
                if (act) {
#pragma unroll
                    for (int s = 0; s < E; ++s) {
                        SK[t * E + ((s + t) & (E - 1))] = h[s];
                        SA[t * E + ((s + t) & (E - 1))] = l[s];
                    }
                }
                __syncthreads();
                if (act) {
                    const uint32_t tp = t ^ (j / E), fl = bitonic_flip(t * E, j, kk);
#pragma unroll
                    for (int s = 0; s < E; ++s) {
                        const uint64_t ph = SK[tp * E + ((s + tp) & (E - 1))];
                        const uint32_t pl = SA[tp * E + ((s + tp) & (E - 1))];
                        take96(h[s], l[s], ph, pl, fl);
                    }
                }
            } else {
                if constexpr (E >= 2) { if (j == 1) cex_local<E, 1>(h, l, t, kk); }
                if constexpr (E >= 4) { if (j == 2) cex_local<E, 2>(h, l, t, kk); }
                if constexpr (E >= 8) { if (j == 4) cex_local<E, 4>(h, l, t, kk); }
                if constexpr (E >= 16) { if (j == 8) cex_local<E, 8>(h, l, t, kk); }
            }
        }
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int s = 0; s < E; ++s) unpack96(h[s], l[s], SK[t * E + s], SA[t * E + s]);
    }
    __syncthreads();
}

// P <= EMAX * NT; only the instantiations up to EMAX are compiled into a kernel,
// so small-bucket kernels keep a small register footprint.
template <int EMAX, int NT>
__device__ __forceinline__ void sort_pow2(uint64_t* SK, uint32_t* SA, uint32_t P) {
    if (P <= (uint32_t)NT) block_bitonic<1, NT>(SK, SA, P);
    else if constexpr (EMAX >= 2) {
        if (P <= 2u * NT) block_bitonic<2, NT>(SK, SA, P);
        else if constexpr (EMAX >= 4) {
            if (P <= 4u * NT) block_bitonic<4, NT>(SK, SA, P);
            else if constexpr (EMAX >= 8) block_bitonic<8, NT>(SK, SA, P);
        }
    }
}

// Exclusive block scans of two per-thread values at once: running maximum of
// `mx` and running sum of `ad` (in thread order).  `wl` holds 2 * NT / 64
// words.  Returns the block-wide sum of `ad`.
template <int NT>
__device__ uint32_t block_scan_max_add(uint32_t& mx, uint32_t& ad, uint32_t* wl) {
    constexpr uint32_t kW = NT / 64;
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t im = mx, ia = ad;
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const uint32_t xm = __shfl_up(im, o), xa = __shfl_up(ia, o);
        if (lane >= o) {
            im = xm > im ? xm : im;
            ia += xa;
        }
    }
    if (lane == 63) {
        wl[w] = im;
        wl[kW + w] = ia;
    }
    __syncthreads();
    uint32_t pm = 0, pa = 0, total = 0;
    for (uint32_t q = 0; q < kW; ++q) {
        if (q < w) {
            pm = wl[q] > pm ? wl[q] : pm;
            pa += wl[kW + q];
        }
        total += wl[kW + q];
    }
    uint32_t em = __shfl_up(im, 1), ea = __shfl_up(ia, 1);
    if (lane == 0) em = ea = 0;
    mx = em > pm ? em : pm;
    ad = pa + ea;
    __syncthreads();
    return total;
}

// (key, a) < (key2, a2) in (group, key, local index) order
__device__ __forceinline__ bool elem_lt(uint64_t k1, uint32_t a1, uint64_t k2, uint32_t a2) {
    uint64_t h1, h2;
    uint32_t l1, l2;
    pack96(k1, a1, h1, l1);
    pack96(k2, a2, h2, l2);
    return h1 < h2 || (h1 == h2 && l1 < l2);
}

// Merge the sorted runs X = (XK, XA)[0..na) and Y = (YK, YA)[0..nb) (distinct
// elements) into (OK, OA)[0..na+nb).  Thread t writes a contiguous stretch of
// the output, found by a binary search along the merge path.  All NT threads call.
template <int NT>
__device__ void merge_runs(const uint64_t* XK, const uint32_t* XA, uint32_t na,
                           const uint64_t* YK, const uint32_t* YA, uint32_t nb, uint64_t* OK,
                           uint32_t* OA) {
    const uint32_t n = na + nb, per = (n + NT - 1) / NT;
    uint32_t o = threadIdx.x * per < n ? threadIdx.x * per : n;
    const uint32_t oe = o + per < n ? o + per : n;
    // i = elements of X among the first o outputs
    uint32_t lo = o > nb ? o - nb : 0u, hi = o < na ? o : na;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (elem_lt(XK[mid], XA[mid], YK[o - mid - 1], YA[o - mid - 1]))
            lo = mid + 1;
        else
            hi = mid;
    }
    uint32_t i = lo, j = o - lo;
    for (; o < oe; ++o) {
        const bool fx = j >= nb || (i < na && elem_lt(XK[i], XA[i], YK[j], YA[j]));
        OK[o] = fx ? XK[i] : YK[j];
        OA[o] = fx ? XA[i] : YA[j];
        i += fx ? 1u : 0u;
        j += fx ? 0u : 1u;
    }
}

template <int EMAX, int NT, bool PK>
__device__ __forceinline__ void base_block_body(uint32_t item, const Seg* items,
                                                const uint64_t* key0, const uint64_t* key1,
                                                const uint64_t* key2_0, const uint64_t* key2_1,
                                                const uint32_t* idx0, const uint32_t* idx1,
                                                const uint8_t* chars, const uint64_t* offsets,
                                                uint32_t* out_perm, uint32_t* out_lcp,
                                                uint32_t pmax, const KeyCodec& kc,
                                                const uint8_t* tab) {
    extern __shared__ uint64_t dyn[];
    uint64_t* K = dyn;                          // pmax keys, by position
    uint64_t* SK = K + pmax;                    // pmax keys, compacted members
    uint64_t* OFFL = SK + pmax;                 // pmax string starts, by local index
    uint32_t* A = (uint32_t*)(OFFL + pmax);     // pmax packed group | local, by position
    uint32_t* SA = A + pmax;                    // pmax compacted members
    uint32_t* IDX = SA + pmax;                  // pmax input index of every local index
    uint16_t* POS = (uint16_t*)(IDX + pmax);    // pmax position of each compacted member
    uint8_t* F = (uint8_t*)(POS + pmax);        // pmax: pair (i-1, i) undecided
    __shared__ uint32_t wl[2 * (NT / 64)];
    const Seg it = items[item];
    const uint32_t buf = it.depth >> 31;
    uint32_t h = it.depth & ~kBufBit;
    const uint32_t n = it.size;
    uint32_t P = 1;
    while (P < n) P <<= 1;
    const uint64_t* kin = (buf ? key1 : key0) + it.begin;
    const uint64_t* k2in = (buf ? key2_1 : key2_0) + it.begin;  // exact or kKeyUnknown
    const uint32_t* iin = (buf ? idx1 : idx0) + it.begin;
    uint32_t* olcp = out_lcp + it.begin;
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < P; i += NT) {
        K[i] = i < n ? kin[i] : ~0ull;
        A[i] = i < n ? i : 0xFFFFFFFFu;
        if (i < n) IDX[i] = iin[i];
    }
    __syncthreads();
    if (P >= 128 && n <= (P >> 1) + (P >> 2)) {
        // n just above a power of two: sort the first P/2 and the rest (padded
        // to a smaller power of two) apart and merge them, instead of sorting
        // P mostly padded elements; K/A and SK/SA swap roles
        const uint32_t half = P >> 1, nb = n - half;
        uint32_t PB = 1;
        while (PB < nb) PB <<= 1;
        sort_pow2<EMAX, NT>(K, A, half);
        sort_pow2<EMAX, NT>(K + half, A + half, PB);
        merge_runs<NT>(K, A, half, K + half, A + half, nb, SK, SA);
        __syncthreads();
        uint64_t* tk = K;
        K = SK;
        SK = tk;
        uint32_t* ta = A;
        A = SA;
        SA = ta;
    } else {
        sort_pow2<EMAX, NT>(K, A, P);
    }
    // each thread owns positions [c0, c1)
    const uint32_t per = (n + NT - 1) / NT;
    const uint32_t c0 = tid * per < n ? tid * per : n;
    const uint32_t c1 = c0 + per < n ? c0 + per : n;
    int any = 0;
    for (uint32_t i = c0; i < c1; ++i) {
        uint8_t un = 0;
        if (i > 0) {
            const uint64_t x = K[i - 1], y = K[i];
            if (x == y && !key_ends<PK>(kc, y))
                un = 1;
            else
                S5_OUT(olcp[i], h + key_lcp<PK>(kc, x, y));
        }
        F[i] = un;
        any |= un;
    }
    any = __syncthreads_or(any);
    bool first = true;      // the item's first re-key: second key words serve it where known
    bool have_off = false;  // OFFL holds the string starts of the current members
    while (any) {
        // group start of every position (running max of decided positions) and
        // the rank of every group member among all members
        uint32_t mx = 0, cnt = 0;
        for (uint32_t i = c0; i < c1; ++i) {
            if (!F[i]) mx = i;
            cnt += (F[i] || (i + 1 < n && F[i + 1])) ? 1u : 0u;
        }
        const uint32_t m = block_scan_max_add<NT>(mx, cnt, wl);
        uint32_t run = mx, r = cnt;
        for (uint32_t i = c0; i < c1; ++i) {
            if (!F[i]) run = i;
            if (F[i] || (i + 1 < n && F[i + 1])) {
                POS[r] = (uint16_t)i;
                SK[r] = K[i];
                SA[r] = (run << 16) | (A[i] & 0xFFFFu);
                ++r;
            }
        }
        __syncthreads();
        // string starts of the members (later members are among them), unless
        // this is the first re-key and every member's second key word is known
        auto load_starts = [&]() {
            for (uint32_t q = tid; q < m; q += NT) {
                const uint32_t l = SA[q] & 0xFFFFu;
                OFFL[l] = offsets[IDX[l]];
            }
            have_off = true;
            __syncthreads();
        };
        if (!have_off) {
            int gat = first ? 0 : 1;
            if (first)
                for (uint32_t q = tid; q < m; q += NT)
                    if (k2in[SA[q] & 0xFFFFu] == kKeyUnknown) gat = 1;
            if (__syncthreads_or(gat)) load_starts();
        }
        if (m <= 64) {
            // few undecided strings left: wavefront 0 finishes them in registers
            if (tid < 64) {
                const bool valid = tid < m;
                const uint32_t pos = valid ? POS[tid] : 0u;
                const uint32_t fa = wave_rounds<PK>(
                    valid ? SK[tid] : ~0ull, valid ? SA[tid] : 0xFFFFFFFFu, valid, h, pos, OFFL,
                    !have_off, first ? k2in : nullptr, iin, chars, offsets, olcp, kc, tab);
                if (valid) A[pos] = fa;
            }
            __syncthreads();
            break;
        }
        // re-key the members one key deeper and sort them by (group, key, local index)
        h += key_chars<PK>(kc);
        uint32_t Pm = 1;
        while (Pm < m) Pm <<= 1;
        // up to pmax / NT members per thread: all their gathers in flight at once
        constexpr int G = EMAX;
        uint64_t pos[G], nkey[G];
        bool need[G], gat[G];
#pragma unroll
        for (int e = 0; e < G; ++e) {
            const uint32_t q = tid + e * NT;
            need[e] = q < m;
            const uint32_t l = need[e] ? SA[q] & 0xFFFFu : 0u;
            nkey[e] = first && need[e] ? k2in[l] : kKeyUnknown;
            gat[e] = need[e] && nkey[e] == kKeyUnknown;  // then have_off holds
            pos[e] = need[e] && have_off ? OFFL[l] : 0ull;
        }
        // does member q's key differ from its group predecessor's?
        auto differs = [&](uint32_t q) {
            return q > 0 && (SA[q] >> 16) == (SA[q - 1] >> 16) && SK[q] != SK[q - 1];
        };
        // Re-key 8 bytes deeper.  A depth at which no group's keys differ and
        // no key ends the strings decides nothing, so the groups stay as they
        // are and only the depth moves on (long equal runs such as duplicate
        // strings cost a gather per 8 bytes, not a whole round).
        // can some pair be decided at the current depth (a group's keys differ,
        // or a key ends the strings)?  Block-wide; all threads call.
        auto progress = [&]() {
            int prog = 0;
#pragma unroll
            for (int e = 0; e < G; ++e) {
                const uint32_t q = tid + e * NT;
                if (need[e] && (differs(q) || key_ends<PK>(kc, SK[q]))) prog = 1;
            }
            return __syncthreads_or(prog);
        };
        if constexpr (PK) {
#pragma unroll
            for (int e = 0; e < G; ++e) {
                if (gat[e]) nkey[e] = packed_load1(kc, tab, chars, pos[e] + h);
                __builtin_amdgcn_sched_barrier(0);  // one member's raw words at a time
            }
        } else {
            uint64_t at[G];
#pragma unroll
            for (int e = 0; e < G; ++e) at[e] = pos[e] + h;
            load_keys<G>(chars, at, gat, nkey);
        }
        first = false;
#pragma unroll
        for (int e = 0; e < G; ++e)
            if (need[e]) SK[tid + e * NT] = nkey[e];
        __syncthreads();
        while (!progress()) {
            if (!have_off) {  // the second key words decided nothing: gathers from here on
                load_starts();
#pragma unroll
                for (int e = 0; e < G; ++e)
                    pos[e] = need[e] ? OFFL[SA[tid + e * NT] & 0xFFFFu] : 0ull;
            }
            // a run of equal characters: from here on two keys per gather
            // (packed keys: one key of 21 characters per gather)
            h += key_chars<PK>(kc);
            if constexpr (PK) {
#pragma unroll
                for (int e = 0; e < G; ++e) {
                    if (need[e]) SK[tid + e * NT] = packed_load1(kc, tab, chars, pos[e] + h);
                    __builtin_amdgcn_sched_barrier(0);
                }
                __syncthreads();
                continue;
            }
            uint64_t k2[G];
#pragma unroll
            for (int e = 0; e < G; ++e)
                if (need[e]) key_load2<PK>(kc, tab, chars, pos[e] + h, &nkey[e], &k2[e]);
#pragma unroll
            for (int e = 0; e < G; ++e)
                if (need[e]) SK[tid + e * NT] = nkey[e];
            __syncthreads();
            if (progress()) break;
            h += key_chars<PK>(kc);
#pragma unroll
            for (int e = 0; e < G; ++e)
                if (need[e]) SK[tid + e * NT] = k2[e];
            __syncthreads();
        }
        // re-sort only if some group's keys now differ (equal keys keep their
        // local-index order)
        int split = 0;
#pragma unroll
        for (int e = 0; e < G; ++e)
            if (need[e] && differs(tid + e * NT)) split = 1;
        split = __syncthreads_or(split);
        if (split) {
            for (uint32_t q = m + tid; q < Pm; q += NT) {
                SK[q] = ~0ull;
                SA[q] = 0xFFFFFFFFu;
            }
            __syncthreads();
            sort_pow2<EMAX, NT>(SK, SA, Pm);
            for (uint32_t q = tid; q < m; q += NT) {
                const uint32_t i = POS[q];
                K[i] = SK[q];
                A[i] = SA[q];
            }
        } else {
            for (uint32_t q = tid; q < m; q += NT) K[POS[q]] = SK[q];
        }
        __syncthreads();
        any = 0;
        for (uint32_t i = c0; i < c1; ++i) {
            if (!F[i]) continue;
            const uint64_t x = K[i - 1], y = K[i];
            if (x == y && !key_ends<PK>(kc, y)) {
                any = 1;
            } else {
                F[i] = 0;
                S5_OUT(olcp[i], h + key_lcp<PK>(kc, x, y));
            }
        }
        any = __syncthreads_or(any);
    }
    for (uint32_t i = tid; i < n; i += NT) S5_OUT(out_perm[it.begin + i], IDX[A[i] & 0xFFFFu] - it.base);
}

template <int EMAX, bool G, int NT, bool PK>
__global__ __launch_bounds__(NT, EMAX <= 4 ? 4 : 1) void k_base_block(const Seg* items, const uint64_t* key0,
                                                    const uint64_t* key1, const uint64_t* key2_0,
                                                    const uint64_t* key2_1, const uint32_t* idx0,
                                                    const uint32_t* idx1, const uint8_t* chars,
                                                    const uint64_t* offsets, uint32_t* out_perm,
                                                    uint32_t* out_lcp, uint32_t pmax,
                                                    const uint32_t* wcnt, uint32_t cap,
                                                    const Globals* glob, const uint32_t* guard,
                                                    KeyCodec kc) {
    S5_CODE_TABLE(PK, kc, tab)
    if (!G) {
        base_block_body<EMAX, NT, PK>(blockIdx.x, items, key0, key1, key2_0, key2_1, idx0, idx1, chars, offsets,
                                      out_perm, out_lcp, pmax, kc, tab);
        return;
    }
    const uint32_t units = block_work_count(wcnt, cap, glob, gridDim.x, guard);
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
        base_block_body<EMAX, NT, PK>(u, items, key0, key1, key2_0, key2_1, idx0, idx1, chars, offsets, out_perm,
                                      out_lcp, pmax, kc, tab);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// K9: LCPs at bucket boundaries.  A boundary between two buckets of a pass at
// depth h holds kLcpFlag | h; both strings share h bytes (the bucket
// invariant, Section 3.1 equation (1)) and differ after that.

__global__ __launch_bounds__(256) void k_lcp_fix(const uint8_t* chars, const uint64_t* offsets,
                                                 const uint64_t* set_begin, uint32_t num_sets,
                                                 uint32_t n, const uint32_t* out_perm,
                                                 uint32_t* out_lcp, const uint32_t* guard,
                                                 const Globals* glob) {
    if (guard && *guard) return;  // large segments remain: the host finishes them first
    // after a failed device-side check, perm slots may be unwritten: read none
    if (glob->status) return;
    // last set whose first position is <= q, searched in [lo, num_sets)
    auto set_of = [&](uint32_t q, uint32_t lo) {
        uint32_t hi = num_sets - 1;
        while (lo < hi) {
            uint32_t mid = (lo + hi + 1) >> 1;
            if (set_begin[mid] <= q) lo = mid; else hi = mid - 1;
        }
        return lo;
    };
    // batched: one search per workgroup for its first position; a thread then
    // steps over the few set starts inside the workgroup's 256 positions
    __shared__ uint32_t s_first;
    const uint32_t p0 = blockIdx.x * blockDim.x;
    if (set_begin) {
        if (threadIdx.x == 0) s_first = set_of(p0 < n ? p0 : n - 1, 0);
        __syncthreads();
    }
    uint32_t p = p0 + threadIdx.x;
    if (p == 0 || p >= n) return;
    uint32_t l = out_lcp[p];
    if (!(l & kLcpFlag)) return;
    uint32_t h = l & ~kLcpFlag;
    uint32_t base = 0;
    if (set_begin) {
        uint32_t s = s_first;
        for (int step = 0; step < 8 && s + 1 < num_sets && set_begin[s + 1] <= p; ++step) ++s;
        if (s + 1 < num_sets && set_begin[s + 1] <= p) s = set_of(p, s);
        base = (uint32_t)set_begin[s];
    }
    uint64_t oa = offsets[out_perm[p - 1] + base] + h;
    uint64_t ob = offsets[out_perm[p] + base] + h;
    for (;;) {
        uint64_t ka = load_key(chars, oa), kb = load_key(chars, ob);
        if (ka != kb) {
            h += (uint32_t)(__builtin_clzll((unsigned long long)(ka ^ kb)) >> 3);
            break;
        }
        if (has_zero(ka)) {
            h += nz_bytes(ka);
            break;
        }
        h += 8;
        oa += 8;
        ob += 8;
    }
    S5_OUT(out_lcp[p], h);
}

// ---------------------------------------------------------------------------
// building block: classification against caller-given sorted splitters

__global__ __launch_bounds__(256) void k_tree_from_sorted(const uint64_t* splitters, uint32_t v,
                                                          uint32_t d, uint64_t* tree_lo,
                                                          uint64_t* tree_in, uint16_t* jump) {
    __shared__ uint64_t t[1u << kDMax];
    for (uint32_t j = threadIdx.x; j < v; j += kWG) {
        tree_lo[inorder_node(j, d)] = splitters[j];
        t[inorder_node(j, d)] = splitters[j];
        tree_in[j] = splitters[j];
    }
    if (threadIdx.x == 0) {
        tree_lo[0] = 0;
        tree_in[v] = 0;
    }
    __syncthreads();
    if (jump) build_jump_table(t, d, v, jump, threadIdx.x, blockDim.x);
}

template <int U, int VAR>
__global__ __launch_bounds__(256) void k_classify_plain(const uint64_t* keys, uint32_t n,
                                                        const uint64_t* tree_lo,
                                                        const uint64_t* tree_in,
                                                        const uint16_t* jump, uint32_t v,
                                                        uint32_t d, uint16_t* out) {
    extern __shared__ uint64_t dyn[];
    uint64_t* t = dyn;
    uint64_t* tin = t + (v + 1);
    uint16_t* jt = (uint16_t*)(tin + (v + 1));
    for (uint32_t i = threadIdx.x; i <= v; i += kWG) {
        t[i] = tree_lo[i];
        tin[i] = tree_in[i];
    }
    if (VAR == (int)kClassifyJump)
        for (uint32_t p = threadIdx.x; p < (v + 1) * kJumpPerTreeSlot; p += kWG) jt[p] = jump[p];
    __syncthreads();
    const uint32_t base = blockIdx.x * (kWG * U);
    uint64_t kk[U];
    uint32_t b[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
        uint32_t pos = base + q * kWG + threadIdx.x;
        kk[q] = pos < n ? keys[pos] : 0ull;
    }
    classify_keys<U, VAR>(t, tin, jt, d, v, kk, b);
#pragma unroll
    for (int q = 0; q < U; ++q) {
        uint32_t pos = base + q * kWG + threadIdx.x;
        if (pos < n) out[pos] = (uint16_t)b[q];
    }
}

// ---------------------------------------------------------------------------
// write counting (write-check build only)

#ifdef S5_COUNT_WRITES
__device__ WriteCount g_wc;
#endif

bool set_write_count(const WriteCount& w) {
#ifdef S5_COUNT_WRITES
    return hipMemcpyToSymbol(HIP_SYMBOL(g_wc), &w, sizeof w) == hipSuccess;
#else
    (void)w;
    return false;
#endif
}

// ---------------------------------------------------------------------------
// host-side launchers.  Dyn selects the launch mode: host-driven (cnt ==
// nullptr; the grid is the work the host read back) or graph mode (a fixed
// grid that strides over the count at cnt, clamped to cap).

#define S5_LAUNCH(kern, grid, block, lds, stream, ...)                                  \
    hipLaunchKernelGGL(kern, grid, block, lds, stream, __VA_ARGS__)

static inline uint32_t dyn_grid(const Dyn& dy, uint32_t host_units) {
    return dy.cnt ? dy.grid : host_units;
}

void launch_init_keys(const uint8_t* chars, uint64_t chars_len, const uint64_t* offsets,
                      uint32_t n, uint64_t* key, uint64_t* key2, uint64_t* key3, uint32_t* idx,
                      Globals* glob, const KeyCodec& kc, hipStream_t st) {
    if (!n) return;
    if (kc.b != 8) {
        S5_LAUNCH(k_init_keys<true>, dim3((n + 255) / 256), dim3(256), 0, st, chars, chars_len,
                  offsets, n, key, key2, key3, idx, glob, kc);
        return;
    }
    S5_LAUNCH(k_prefix_sample, dim3((std::min(n, kPrefixSamples) + kWG - 1) / kWG), dim3(kWG), 0,
              st, chars, chars_len, offsets, n, glob);
    S5_LAUNCH(k_init_keys<false>, dim3((n + 255) / 256), dim3(256), 0, st, chars, chars_len,
              offsets, n, key, key2, key3, idx, glob, kc);
    S5_LAUNCH(k_init_redo, dim3(std::min<uint32_t>((n + 255) / 256, 256)), dim3(256), 0, st,
              chars, chars_len, offsets, n, key, key2, key3, idx, glob, kc);
}

// Bytes that occur in a sample of the strings (alphabet compression): string
// i = (j * n) / samples for j < samples, read key by key to its terminator
// (at most 32 keys); bit c of bitmap[c / 32] is set for every byte value c != 0.
// With chars_len > 0 only bytes before chars_len are read (a string at or past
// it is skipped: the key cache rejects the offset afterwards).
__global__ __launch_bounds__(256) void k_alphabet(const uint8_t* chars, uint64_t chars_len,
                                                  const uint64_t* offsets, uint32_t n,
                                                  uint32_t samples, uint32_t* bitmap) {
    __shared__ uint32_t bm[8];
    if (threadIdx.x < 8) bm[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < samples) {
        const uint64_t pos = offsets[(uint32_t)(((uint64_t)j * n) / samples)];
        for (uint32_t q = 0; q < 32; ++q) {
            if (chars_len && pos + 8ull * q >= chars_len) break;
            const uint64_t k = load_key(chars, pos + 8ull * q);
            for (int b = 0; b < 8; ++b) {
                const uint32_t c = (uint32_t)(k >> (56 - 8 * b)) & 0xFFu;
                if (c) atomicOr(&bm[c >> 5], 1u << (c & 31));
            }
            if (has_zero(k)) break;
        }
    }
    __syncthreads();
    if (threadIdx.x < 8 && bm[threadIdx.x]) atomicOr(&bitmap[threadIdx.x], bm[threadIdx.x]);
}

void launch_alphabet(const uint8_t* chars, uint64_t chars_len, const uint64_t* offsets,
                     uint32_t n, uint32_t samples, uint32_t* bitmap, hipStream_t st) {
    S5_LAUNCH(k_zero_words, dim3(1), dim3(256), 0, st, bitmap, 8u);
    if (!n || !samples) return;
    S5_LAUNCH(k_alphabet, dim3((samples + 255) / 256), dim3(256), 0, st, chars, chars_len,
              offsets, n, samples, bitmap);
}

void launch_prefix_keys(const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                        uint32_t depth, uint64_t* key, hipStream_t st) {
    if (!n) return;
    S5_LAUNCH(k_prefix_keys, dim3((n + 255) / 256), dim3(256), 0, st, chars, offsets, n, depth,
              key);
}

void launch_plan_roots(const uint64_t* set_begin, uint32_t num_sets, uint32_t n,
                       uint32_t* out_perm, uint32_t* out_lcp, const PlanCtx& ctx,
                       hipStream_t st) {
    if (!num_sets) return;
    S5_LAUNCH(k_plan_roots, dim3((num_sets + 255) / 256), dim3(256), 0, st, set_begin, num_sets,
              n, out_perm, out_lcp, ctx);
}

void launch_pass_stats(const Counters* cur, const Counters* next, Globals* glob, uint32_t level,
                       hipStream_t st) {
    S5_LAUNCH(k_pass_stats, dim3(1), dim3(64), 0, st, cur, next, glob, level);
}

void launch_publish(const void* src, size_t bytes, void* dst, uint32_t* flag, uint32_t seq,
                    hipStream_t st) {
    const uint32_t words = (uint32_t)std::min<size_t>(bytes / 4, kPublishWords);
    S5_LAUNCH(k_publish, dim3(1), dim3(64), 0, st, (const uint32_t*)src, words, (uint32_t*)dst,
              flag, seq);
}

void launch_zero_words(void* p, size_t bytes, hipStream_t st) {
    const uint32_t n = (uint32_t)(bytes / 4);
    if (n) S5_LAUNCH(k_zero_words, dim3((n + 255) / 256), dim3(256), 0, st, (uint32_t*)p, n);
}

void launch_sample_tree(uint32_t n_large, const LSeg* lseg, const uint64_t* key_in,
                        uint32_t alpha, uint32_t vmax, uint64_t seed, uint64_t* tree_lo,
                        uint64_t* tree_in, uint8_t* tree_lcp, uint16_t* jump, uint32_t* tile_tab,
                        uint32_t* chunk_tab, Counters* next_cnt, const Globals* glob,
                        const Dyn& dy, uint32_t redo, const KeyCodec& kc, hipStream_t st) {
    uint32_t m = alpha * (vmax + 1) - 1, P = 1;
    while (P < m) P <<= 1;
    if (dy.cnt)
        S5_LAUNCH(k_sample_tree<true>, dim3(dy.grid), dim3(kWG), (size_t)P * 8, st, lseg, key_in,
                  alpha, seed, tree_lo, tree_in, tree_lcp, jump, tile_tab, chunk_tab, next_cnt,
                  dy.cnt, dy.cap, glob, redo, kc);
    else
        S5_LAUNCH(k_sample_tree<false>, dim3(n_large), dim3(kWG), (size_t)P * 8, st, lseg, key_in,
                  alpha, seed, tree_lo, tree_in, tree_lcp, jump, tile_tab, chunk_tab, next_cnt,
                  dy.cnt, dy.cap, glob, redo, kc);
}

void launch_classify(uint32_t tiles, uint32_t unroll, uint32_t variant, const LSeg* lseg,
                     const uint32_t* tile_tab, const uint64_t* key_in, const uint64_t* tree_lo,
                     const uint64_t* tree_in, const uint16_t* jump, uint16_t* bid, uint32_t* cm,
                     uint32_t vmax, uint32_t kmax, const Globals* glob, const Dyn& dy,
                     uint32_t redo, hipStream_t st) {
    size_t lds = (size_t)(vmax + 1) * 16 + (size_t)kWaves * kmax * 4;
    if (variant == kClassifyJump) lds += (size_t)(vmax + 1) * kJumpPerTreeSlot * 2;
    dim3 grid(dyn_grid(dy, tiles));
#define S5_CLASSIFY_GE(U, GG, VV)                                                            \
    S5_LAUNCH((k_classify<U, GG, VV>), grid, dim3(kWG), lds, st, lseg, tile_tab, key_in,       \
              tree_lo, tree_in, jump, bid, cm, vmax, kmax, dy.cnt, dy.cap, glob, redo)
#define S5_CLASSIFY_G(U, GG)                                                                 \
    do {                                                                                     \
        if (variant == kClassifyEqual) S5_CLASSIFY_GE(U, GG, 1);                             \
        else if (variant == kClassifyJump) S5_CLASSIFY_GE(U, GG, 2);                         \
        else S5_CLASSIFY_GE(U, GG, 0);                                                       \
    } while (0)
#define S5_CLASSIFY(U)                                                                       \
    do {                                                                                     \
        if (dy.cnt) S5_CLASSIFY_G(U, true);                                                  \
        else S5_CLASSIFY_G(U, false);                                                        \
    } while (0)
    switch (unroll) {
        case 1: S5_CLASSIFY(1); break;
        case 2: S5_CLASSIFY(2); break;
        case 8: S5_CLASSIFY(8); break;
        default: S5_CLASSIFY(4); break;
    }
#undef S5_CLASSIFY
#undef S5_CLASSIFY_G
#undef S5_CLASSIFY_GE
}

void launch_colscan(uint32_t chunks, uint32_t kmax, const LSeg* lseg, const uint32_t* chunk_tab,
                    uint32_t* cm, uint32_t* cs, const Globals* glob, const Dyn& dy, uint32_t redo,
                    hipStream_t st, uint32_t dig) {
    const uint32_t cols = dig ? kDigitMax : kmax;
    const dim3 grid(dyn_grid(dy, chunks), (cols + kWG - 1) / kWG);
    if (dy.cnt)
        S5_LAUNCH(k_colscan<true>, grid, dim3(kWG), 0, st, lseg, chunk_tab, cm, cs, dy.cnt, dy.cap,
                  glob, redo, dig);
    else
        S5_LAUNCH(k_colscan<false>, grid, dim3(kWG), 0, st, lseg, chunk_tab, cm, cs, dy.cnt, dy.cap,
                  glob, redo, dig);
}

void launch_digit_count(uint32_t tiles, const LSeg* lseg, const uint32_t* tile_tab,
                        const uint16_t* bid, uint32_t* cm, uint32_t dig, hipStream_t st) {
    if (tiles) S5_LAUNCH(k_digit_count, dim3(tiles), dim3(kWG), 0, st, lseg, tile_tab, bid, cm, dig);
}

void launch_digit_starts(uint32_t n_large, const LSeg* lseg, uint32_t* cs, uint32_t dig,
                         hipStream_t st) {
    if (n_large) S5_LAUNCH(k_digit_starts, dim3(n_large), dim3(kWG), 0, st, lseg, cs, dig);
}

void launch_bucket_plan(uint32_t n_large, const LSeg* lseg, uint32_t* cs, uint32_t* bstart,
                        const uint64_t* tree_in, const uint8_t* tree_lcp, const PlanCtx& ctx,
                        uint32_t next_buf, uint32_t kmax, const Dyn& dy, hipStream_t st) {
    const size_t lds = (size_t)kmax * 3 * 4;
    if (dy.cnt)
        S5_LAUNCH(k_bucket_plan<true>, dim3(dy.grid), dim3(kWG), lds, st, lseg, cs, bstart,
                  tree_in, tree_lcp, ctx, next_buf, dy.cnt, dy.cap, kmax);
    else
        S5_LAUNCH(k_bucket_plan<false>, dim3(n_large), dim3(kWG), lds, st, lseg, cs, bstart,
                  tree_in, tree_lcp, ctx, next_buf, dy.cnt, dy.cap, kmax);
}

void launch_scatter(uint32_t tiles, uint32_t unroll, const LSeg* lseg, const uint32_t* tile_tab,
                    const uint16_t* bid, const uint64_t* key_in, const uint64_t* key2_in,
                    const uint32_t* idx_in, uint64_t* key_out, uint64_t* key2_out,
                    uint32_t* idx_out, const uint32_t* cm, const uint32_t* cs,
                    const uint32_t* bstart, const uint64_t* tree_in, const uint8_t* tree_lcp,
                    const uint8_t* chars, const uint64_t* offsets, uint32_t* out_perm,
                    uint32_t* out_lcp, uint32_t vmax, uint32_t kmax, const Globals* glob,
                    const Dyn& dy, const uint64_t* key3, const KeyCodec& kc, hipStream_t st,
                    hipEvent_t ev_start, hipEvent_t ev_stop, uint32_t dig, uint16_t* bid_out) {
    (void)unroll;
    const size_t krmax = dig ? kDigitMax : kmax;
    const size_t lds = (size_t)kSubTile * (8 + 4 + 2) + krmax * 4 + (size_t)kmax * 4 +
                       (size_t)kWaves * krmax * 2 + (krmax + 1) * 2 + (size_t)kmax * 2;
    // with events (instrumentation, host-driven passes only) the dispatch
    // itself stamps them: their interval is the kernel's execution
#define S5_SCATTER_P(GG, KK, PP, DD, GRID)                                                        \
    do {                                                                                          \
        if (ev_start || ev_stop)                                                                  \
            hipExtLaunchKernelGGL((k_scatter<GG, KK, PP, DD>), dim3(GRID), dim3(kWG), lds, st,    \
                                  ev_start, ev_stop, 0u, lseg, tile_tab, bid, key_in, key2_in,    \
                                  idx_in, key_out, key2_out, idx_out, cm, cs, bstart, tree_in,    \
                                  tree_lcp, chars, offsets, out_perm, out_lcp, vmax, kmax,        \
                                  dy.cnt, dy.cap, glob, key3, kc, bid_out);                       \
        else                                                                                      \
            S5_LAUNCH((k_scatter<GG, KK, PP, DD>), dim3(GRID), dim3(kWG), lds, st, lseg,          \
                      tile_tab, bid, key_in, key2_in, idx_in, key_out, key2_out, idx_out, cm, cs, \
                      bstart, tree_in, tree_lcp, chars, offsets, out_perm, out_lcp, vmax, kmax,   \
                      dy.cnt, dy.cap, glob, key3, kc, bid_out);                                   \
    } while (0)
#define S5_SCATTER(GG, KK, DD, GRID)                                                              \
    do {                                                                                          \
        if (kc.b != 8) S5_SCATTER_P(GG, KK, true, DD, GRID);                                      \
        else S5_SCATTER_P(GG, KK, false, DD, GRID);                                               \
    } while (0)
    if (dig == kDigitLow) {  // the two-pass distribution runs host-driven only
        if (key3)
            S5_SCATTER(false, true, 1, tiles);
        else
            S5_SCATTER(false, false, 1, tiles);
    } else if (dig == kDigitHigh) {
        S5_SCATTER(false, false, 2, tiles);
    } else if (dy.cnt) {
        if (key3)
            S5_SCATTER(true, true, 0, dy.grid);
        else
            S5_SCATTER(true, false, 0, dy.grid);
    } else {
        if (key3)
            S5_SCATTER(false, true, 0, tiles);
        else
            S5_SCATTER(false, false, 0, tiles);
    }
#undef S5_SCATTER
#undef S5_SCATTER_P
}

// Host-driven: n_items[q] items of class q.  Graph mode (dy[q].cnt set): the
// counts are read on the device, and nothing runs while *guard != 0.
template <bool G, bool PK>
static void base_sort_launch(const uint32_t* n_items, Seg* const* items, const uint64_t* key0,
                             const uint64_t* key1, const uint64_t* key2_0, const uint64_t* key2_1,
                             const uint32_t* idx0, const uint32_t* idx1,
                             const uint8_t* chars, const uint64_t* offsets, uint32_t* out_perm,
                             uint32_t* out_lcp, uint32_t T, const Globals* glob, const Dyn* dy,
                             const uint32_t* guard, const KeyCodec& kc, hipStream_t st) {
    if (G || n_items[0]) {
        const uint32_t g = G ? dy[0].grid : (n_items[0] + kWaves - 1) / kWaves;
        S5_LAUNCH((k_base_wave<G, PK>), dim3(g), dim3(kWG), 0, st, items[0], n_items[0], key0,
                  key1, key2_0, key2_1, idx0, idx1, chars, offsets, out_perm, out_lcp, dy[0].cnt, dy[0].cap, glob,
                  guard, kc);
    }
    uint32_t PT = 1;
    while (PT < T) PT <<= 1;
    const size_t per = 8 + 8 + 8 + 4 + 4 + 4 + 2 + 1;  // K, SK, OFFL, A, SA, IDX, POS, F
    if ((G || n_items[1]) && PT > kBaseWave) {  // <= 256 strings: one wavefront
        const uint32_t P = PT < kBaseSmall ? PT : kBaseSmall;
        S5_LAUNCH((k_base_block<4, G, 64, PK>), dim3(G ? dy[1].grid : n_items[1]), dim3(64),
                  per * P, st, items[1], key0, key1, key2_0, key2_1, idx0, idx1, chars, offsets, out_perm, out_lcp,
                  P, dy[1].cnt, dy[1].cap, glob, guard, kc);
    }
    if ((G || n_items[2]) && PT > kBaseSmall) {  // <= 512 strings: two wavefronts
        const uint32_t P = PT < kBaseMid ? PT : kBaseMid;
        S5_LAUNCH((k_base_block<4, G, 128, PK>), dim3(G ? dy[2].grid : n_items[2]), dim3(128),
                  per * P, st, items[2], key0, key1, key2_0, key2_1, idx0, idx1, chars, offsets, out_perm, out_lcp,
                  P, dy[2].cnt, dy[2].cap, glob, guard, kc);
    }
    if ((G || n_items[3]) && PT > kBaseMid) {  // <= T strings: four (or eight) wavefronts
        const dim3 g(G ? dy[3].grid : n_items[3]);
        if (PT <= 4u * kWG)
            S5_LAUNCH((k_base_block<4, G, kWG, PK>), g, dim3(kWG), per * PT, st, items[3], key0,
                      key1, key2_0, key2_1, idx0, idx1, chars, offsets, out_perm, out_lcp, PT, dy[3].cnt,
                      dy[3].cap, glob, guard, kc);
        else  // <= 2048 strings: eight wavefronts, four strings each
            S5_LAUNCH((k_base_block<4, G, 2 * kWG, PK>), g, dim3(2 * kWG), per * PT, st, items[3],
                      key0, key1, key2_0, key2_1, idx0, idx1, chars, offsets, out_perm, out_lcp, PT, dy[3].cnt,
                      dy[3].cap, glob, guard, kc);
    }
}

// Host-driven: n_items[q] items of class q.  Graph mode (dy[0].cnt set): the
// counts are read on the device, and nothing runs while *guard != 0.
void launch_base_sort(const uint32_t* n_items, Seg* const* items, const uint64_t* key0,
                      const uint64_t* key1, const uint64_t* key2_0, const uint64_t* key2_1,
                      const uint32_t* idx0, const uint32_t* idx1,
                      const uint8_t* chars, const uint64_t* offsets, uint32_t* out_perm,
                      uint32_t* out_lcp, uint32_t T, const Globals* glob, const Dyn* dy,
                      const uint32_t* guard, const KeyCodec& kc, hipStream_t st) {
    const bool pk = kc.b != 8;
    if (dy[0].cnt) {
        if (pk)
            base_sort_launch<true, true>(n_items, items, key0, key1, key2_0, key2_1, idx0, idx1, chars, offsets,
                                         out_perm, out_lcp, T, glob, dy, guard, kc, st);
        else
            base_sort_launch<true, false>(n_items, items, key0, key1, key2_0, key2_1, idx0, idx1, chars, offsets,
                                          out_perm, out_lcp, T, glob, dy, guard, kc, st);
    } else {
        if (pk)
            base_sort_launch<false, true>(n_items, items, key0, key1, key2_0, key2_1, idx0, idx1, chars, offsets,
                                          out_perm, out_lcp, T, glob, dy, guard, kc, st);
        else
            base_sort_launch<false, false>(n_items, items, key0, key1, key2_0, key2_1, idx0, idx1, chars, offsets,
                                           out_perm, out_lcp, T, glob, dy, guard, kc, st);
    }
}

void launch_lcp_fix(const uint8_t* chars, const uint64_t* offsets, const uint64_t* set_begin,
                    uint32_t num_sets, uint32_t n, const uint32_t* out_perm, uint32_t* out_lcp,
                    const uint32_t* guard, const Globals* glob, hipStream_t st) {
    if (n < 2) return;
    S5_LAUNCH(k_lcp_fix, dim3((n + 255) / 256), dim3(256), 0, st, chars, offsets, set_begin,
              num_sets, n, out_perm, out_lcp, guard, glob);
}

void launch_classify_plain(const uint64_t* keys, uint32_t n, const uint64_t* splitters,
                           uint32_t v, uint32_t d, uint32_t variant, uint64_t* tree_lo,
                           uint64_t* tree_in, uint16_t* jump, uint16_t* out, hipStream_t st) {
    S5_LAUNCH(k_tree_from_sorted, dim3(1), dim3(kWG), 0, st, splitters, v, d, tree_lo, tree_in,
              variant == kClassifyJump ? jump : nullptr);
    if (!n) return;
    const dim3 grid((n + kWG * 4 - 1) / (kWG * 4));
    const size_t lds = (size_t)(v + 1) * (16 + 2 * kJumpPerTreeSlot);
    if (variant == kClassifyEqual)
        S5_LAUNCH((k_classify_plain<4, 1>), grid, dim3(kWG), lds, st, keys, n, tree_lo, tree_in,
                  jump, v, d, out);
    else if (variant == kClassifyJump)
        S5_LAUNCH((k_classify_plain<4, 2>), grid, dim3(kWG), lds, st, keys, n, tree_lo, tree_in,
                  jump, v, d, out);
    else
        S5_LAUNCH((k_classify_plain<4, 0>), grid, dim3(kWG), lds, st, keys, n, tree_lo, tree_in,
                  jump, v, d, out);
}

}  // namespace s5
