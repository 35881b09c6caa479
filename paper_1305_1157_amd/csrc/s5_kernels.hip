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
//                  descents over coalesced keys; bucket ids; per-unit histogram
//                  built with wavefront ballots (no atomics)
//   k_colscan      exclusive scan down each bucket column of the count matrix,
//                  within chunks of 64 unit rows
//   k_bucket_plan  one workgroup per segment: chunk prefixes, bucket starts,
//                  and the plan of every bucket (finished / base case / next pass)
//   k_scatter      stable redistribution of (key, index); keys of buckets whose
//                  depth grows are refreshed from the arena on the way; buckets
//                  that are finished write their final output directly
// followed, once every bucket is small, by k_base_sort (LDS sorter that emits
// LCPs) and k_lcp_fix (LCPs at bucket boundaries).
#include "s5_internal.h"
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
// planning: decide what happens to a bucket of >= 2 strings

__device__ void plan_segment(uint32_t begin, uint32_t size, uint32_t depth, uint32_t base,
                             uint32_t buf, const PlanCtx& c) {
    if (size <= c.T) {
        uint32_t slot = atomicAdd(&c.glob->n_base, 1u);
        if (slot >= c.caps.base) {
            atomicOr(&c.glob->status, kErrBaseCap);
            return;
        }
        Seg s;
        s.begin = begin;
        s.size = size;
        s.depth = depth | (buf ? kBufBit : 0u);
        s.base = base;
        c.base_list[slot] = s;
        atomicAdd(&c.glob->base_elems, (unsigned long long)size);
        return;
    }
    // a large segment: sized tree and units for the next distribution pass
    uint32_t d = 1;
    while (d < c.d_max && ((uint64_t)c.T << d) < 2ull * size) ++d;  // 2^d * T/2 >= size
    uint32_t v = (1u << d) - 1, k = 2 * v + 1;
    uint32_t ulen = (uint32_t)(((uint64_t)size + kMaxUnits - 1) / kMaxUnits);
    ulen = (ulen + 63u) & ~63u;
    if (ulen < c.unit_min) ulen = c.unit_min;
    uint32_t units = (uint32_t)(((uint64_t)size + ulen - 1) / ulen);
    units = (units + kWaves - 1) / kWaves * kWaves;
    uint32_t chunks = (units + kChunkRows - 1) / kChunkRows;

    uint32_t slot = atomicAdd(&c.cnt->n_large, 1u);
    uint32_t ub = atomicAdd(&c.cnt->units, units);
    uint32_t cb = atomicAdd(&c.cnt->chunks, chunks);
    uint32_t tb = atomicAdd(&c.cnt->tree, v + 1);
    uint32_t bb = atomicAdd(&c.cnt->bstart, k + 1);
    unsigned long long cmb = atomicAdd(&c.cnt->cm, (unsigned long long)units * k);
    unsigned long long csb = atomicAdd(&c.cnt->cs, (unsigned long long)chunks * k);
    atomicAdd(&c.cnt->moved, (unsigned long long)size);
    atomicMax(&c.cnt->kmax, k);
    uint32_t err = 0;
    if (slot >= c.caps.large) err |= kErrLargeCap;
    if (ub + units > c.caps.units || cb + chunks > c.caps.chunks) err |= kErrUnitCap;
    if (cmb + (unsigned long long)units * k > c.caps.cm ||
        csb + (unsigned long long)chunks * k > c.caps.cs)
        err |= kErrCmCap;
    if (tb + v + 1 > c.caps.tree || bb + k + 1 > c.caps.bstart) err |= kErrTreeCap;
    if (err) {
        atomicOr(&c.glob->status, err);
        return;
    }
    LSeg g;
    g.begin = begin;
    g.size = size;
    g.depth = depth;
    g.base = base;
    g.d = d;
    g.v = v;
    g.k = k;
    g.unit_len = ulen;
    g.units = units;
    g.unit_base = ub;
    g.chunks = chunks;
    g.chunk_base = cb;
    g.tree_base = tb;
    g.bstart_base = bb;
    g.pad0 = g.pad1 = 0;
    g.cm_base = cmb;
    g.cs_base = csb;
    c.lseg[slot] = g;
}

// ---------------------------------------------------------------------------
// K1: prefix cache at depth 0 (and the building-block entry point)

__global__ __launch_bounds__(256) void k_init_keys(const uint8_t* chars, const uint64_t* offsets,
                                                   uint32_t n, uint64_t* key, uint32_t* idx) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    idx[i] = i;
    key[i] = load_key(chars, offsets[i]);
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
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= num_sets) return;
    uint32_t b = set_begin ? (uint32_t)set_begin[s] : 0u;
    uint32_t e = set_begin ? (uint32_t)set_begin[s + 1] : n;
    if (e <= b) return;
    out_lcp[b] = 0;
    if (e - b == 1) {
        out_perm[b] = 0;
        return;
    }
    plan_segment(b, e - b, 0, b, 0, ctx);
}

// ---------------------------------------------------------------------------
// K2: sample, sort the sample, select splitters recursively, build the tree

__global__ __launch_bounds__(256) void k_sample_tree(const LSeg* lseg, const uint64_t* key_in,
                                                     uint32_t alpha, uint64_t seed,
                                                     uint64_t* tree_lo, uint64_t* tree_in,
                                                     uint8_t* tree_lcp, uint32_t* unit_tab,
                                                     uint32_t* chunk_tab) {
    extern __shared__ uint64_t smp[];  // sample, padded to a power of two
    __shared__ uint32_t ra[1u << kDMax], rb[1u << kDMax];
    __shared__ uint64_t t[1u << kDMax];
    const uint32_t slot = blockIdx.x;
    const LSeg g = lseg[slot];
    const uint32_t tid = threadIdx.x;
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
                l = p == x ? 0 : (uint8_t)(__builtin_clzll((unsigned long long)(p ^ x)) >> 3);
            }
            lcp_out[i] = l;
        } else {
            in_out[i] = 0;
            lcp_out[i] = 0;
        }
    }
    for (uint32_t u = tid; u < g.units; u += kWG) unit_tab[g.unit_base + u] = slot;
    for (uint32_t c = tid; c < g.chunks; c += kWG) chunk_tab[g.chunk_base + c] = slot;
}

// ---------------------------------------------------------------------------
// K3: classification + per-unit histograms

template <int U>
__global__ __launch_bounds__(256) void k_classify(const LSeg* lseg, const uint32_t* unit_tab,
                                                  const uint64_t* key_in, const uint64_t* tree_lo,
                                                  const uint64_t* tree_in, uint16_t* bid,
                                                  uint32_t* cm, uint32_t vmax, uint32_t kmax) {
    extern __shared__ uint64_t dyn[];
    uint64_t* t = dyn;
    uint64_t* tin = t + (vmax + 1);
    uint32_t* hist = (uint32_t*)(tin + (vmax + 1));
    const uint32_t unit0 = blockIdx.x * kWaves;
    const uint32_t slot = unit_tab[unit0];
    const LSeg g = lseg[slot];
    for (uint32_t i = threadIdx.x; i <= g.v; i += kWG) {
        t[i] = tree_lo[g.tree_base + i];
        tin[i] = tree_in[g.tree_base + i];
    }
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    uint32_t* h = hist + w * kmax;
    for (uint32_t b = lane; b < g.k; b += 64) h[b] = 0;
    __syncthreads();
    const uint32_t u = unit0 + w - g.unit_base;
    const uint64_t ub = (uint64_t)u * g.unit_len;
    const uint32_t start = g.begin + (uint32_t)(ub < g.size ? ub : g.size);
    const uint32_t end = g.begin + (uint32_t)(ub + g.unit_len < g.size ? ub + g.unit_len : g.size);
    const uint32_t nbits = g.d + 1;
    for (uint32_t c = start; c < end; c += 64 * U) {
        uint64_t kk[U];
        uint32_t b[U];
        bool valid[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            uint32_t pos = c + q * 64 + lane;
            valid[q] = pos < end;
            kk[q] = valid[q] ? key_in[pos] : 0ull;
        }
        classify_u<U>(t, tin, g.d, g.v, kk, b);
#pragma unroll
        for (int q = 0; q < U; ++q) {
            uint32_t pos = c + q * 64 + lane;
            if (valid[q]) bid[pos] = (uint16_t)b[q];
            uint64_t act = __ballot(valid[q]);
            if (act) {
                uint64_t m = match_bucket(b[q], nbits, act);
                if (valid[q] && lane == (uint32_t)(__ffsll((long long)m) - 1))
                    h[b[q]] += (uint32_t)__popcll(m);
            }
        }
    }
    __syncthreads();
    uint32_t* row = cm + g.cm_base + (uint64_t)u * g.k;
    for (uint32_t b = lane; b < g.k; b += 64) row[b] = h[b];
}

// ---------------------------------------------------------------------------
// K4a: exclusive scan down every bucket column within a chunk of unit rows

__global__ __launch_bounds__(256) void k_colscan(const LSeg* lseg, const uint32_t* chunk_tab,
                                                 uint32_t* cm, uint32_t* cs) {
    const uint32_t cg = blockIdx.x;
    const LSeg g = lseg[chunk_tab[cg]];
    const uint32_t b = blockIdx.y * kWG + threadIdx.x;
    if (b >= g.k) return;
    const uint32_t c = cg - g.chunk_base;
    const uint32_t r0 = c * kChunkRows;
    const uint32_t r1 = r0 + kChunkRows < g.units ? r0 + kChunkRows : g.units;
    uint32_t run = 0;
    uint32_t* col = cm + g.cm_base + b;
    for (uint32_t r = r0; r < r1; ++r) {
        uint32_t x = col[(uint64_t)r * g.k];
        col[(uint64_t)r * g.k] = run;
        run += x;
    }
    cs[g.cs_base + (uint64_t)c * g.k + b] = run;
}

// ---------------------------------------------------------------------------
// K4b: chunk prefixes, bucket starts, and the plan of every bucket

__global__ __launch_bounds__(256) void k_bucket_plan(const LSeg* lseg, uint32_t* cs,
                                                     uint32_t* bstart, const uint64_t* tree_in,
                                                     const uint8_t* tree_lcp, PlanCtx ctx,
                                                     uint32_t next_buf) {
    __shared__ uint32_t tot[1u << (kDMax + 1)];
    __shared__ uint32_t st[1u << (kDMax + 1)];
    __shared__ uint32_t tmp[kWG + 1];
    const LSeg g = lseg[blockIdx.x];
    const uint32_t k = g.k;
    for (uint32_t b = threadIdx.x; b < k; b += kWG) {
        uint32_t run = 0;
        for (uint32_t c = 0; c < g.chunks; ++c) {
            uint32_t* p = cs + g.cs_base + (uint64_t)c * k + b;
            uint32_t x = *p;
            *p = run;
            run += x;
        }
        tot[b] = run;
    }
    __syncthreads();
    block_exclusive_scan(tot, st, k, tmp);
    uint32_t* bs = bstart + g.bstart_base;
    double ent = 0.0;
    unsigned long long mx = 0;
    for (uint32_t b = threadIdx.x; b < k; b += kWG) {
        const uint32_t s0 = st[b];
        bs[b] = s0;
        for (uint32_t c = 0; c < g.chunks; ++c) cs[g.cs_base + (uint64_t)c * k + b] += s0;
        const uint32_t sz = tot[b];
        if (sz == 0) continue;
        ent += (double)sz * log2((double)g.size / (double)sz);
        if (sz > mx) mx = sz;
        if (sz < 2) continue;  // single strings are finished by the scatter
        const uint32_t j = b >> 1;
        uint32_t nd;
        if (b & 1u) {
            uint64_t x = tree_in[g.tree_base + j];
            if (has_zero(x)) continue;  // all strings identical: finished by the scatter
            nd = g.depth + 8;
        } else {
            nd = g.depth + ((j == 0 || j == g.v) ? 0u : (uint32_t)tree_lcp[g.tree_base + j]);
        }
        plan_segment(g.begin + s0, sz, nd, g.base, next_buf, ctx);
    }
    if (threadIdx.x == 0) bs[k] = g.size;
    atomicMax(&ctx.cnt->max_bucket, mx);
    if (ent != 0.0) atomicAdd(&ctx.cnt->entropy_sum, ent);
}

// ---------------------------------------------------------------------------
// K5: stable scatter; key refresh for the next depth; finished buckets

template <int U>
__global__ __launch_bounds__(256) void k_scatter(
    const LSeg* lseg, const uint32_t* unit_tab, const uint16_t* bid, const uint64_t* key_in,
    const uint32_t* idx_in, uint64_t* key_out, uint32_t* idx_out, const uint32_t* cm,
    const uint32_t* cs, const uint32_t* bstart, const uint64_t* tree_in, const uint8_t* tree_lcp,
    const uint8_t* chars, const uint64_t* offsets, uint32_t* out_perm, uint32_t* out_lcp,
    uint32_t vmax, uint32_t kmax) {
    extern __shared__ uint64_t dyn[];
    uint64_t* tin = dyn;                                   // vmax + 1
    uint32_t* bst = (uint32_t*)(tin + (vmax + 1));         // kmax + 1
    uint32_t* run = bst + (kmax + 1);                      // kWaves * kmax
    uint8_t* lcpx = (uint8_t*)(run + kWaves * kmax);       // vmax + 1
    const uint32_t unit0 = blockIdx.x * kWaves;
    const uint32_t slot = unit_tab[unit0];
    const LSeg g = lseg[slot];
    for (uint32_t i = threadIdx.x; i <= g.v; i += kWG) {
        tin[i] = tree_in[g.tree_base + i];
        lcpx[i] = tree_lcp[g.tree_base + i];
    }
    for (uint32_t b = threadIdx.x; b <= g.k; b += kWG) bst[b] = bstart[g.bstart_base + b];
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    const uint32_t u = unit0 + w - g.unit_base;
    const uint32_t c = u / kChunkRows;
    uint32_t* r = run + w * kmax;
    for (uint32_t b = lane; b < g.k; b += 64)
        r[b] = cs[g.cs_base + (uint64_t)c * g.k + b] + cm[g.cm_base + (uint64_t)u * g.k + b];
    __syncthreads();
    const uint64_t ub = (uint64_t)u * g.unit_len;
    const uint32_t start = g.begin + (uint32_t)(ub < g.size ? ub : g.size);
    const uint32_t end = g.begin + (uint32_t)(ub + g.unit_len < g.size ? ub + g.unit_len : g.size);
    const uint32_t nbits = g.d + 1;
    const uint64_t ltmask = (1ull << lane) - 1ull;
    for (uint32_t cpos = start; cpos < end; cpos += 64 * U) {
        uint32_t b[U], id[U];
        uint64_t kk[U];
        bool valid[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            uint32_t pos = cpos + q * 64 + lane;
            valid[q] = pos < end;
            b[q] = valid[q] ? bid[pos] : 0u;
            kk[q] = valid[q] ? key_in[pos] : 0ull;
            id[q] = valid[q] ? idx_in[pos] : 0u;
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            uint64_t act = __ballot(valid[q]);
            if (!act) break;
            uint64_t m = match_bucket(b[q], nbits, act);
            uint32_t old = valid[q] ? r[b[q]] : 0u;
            if (valid[q] && lane == (uint32_t)(__ffsll((long long)m) - 1))
                r[b[q]] = old + (uint32_t)__popcll(m);
            if (!valid[q]) continue;
            const uint32_t dr = old + (uint32_t)__popcll(m & ltmask);
            const uint32_t dest = g.begin + dr;
            const uint32_t bb = b[q];
            const uint32_t s0 = bst[bb], size = bst[bb + 1] - s0;
            if (dr == s0 && dr != 0) out_lcp[dest] = kLcpFlag | g.depth;
            const uint32_t j = bb >> 1;
            const bool odd = bb & 1u;
            if (size == 1) {
                out_perm[dest] = id[q] - g.base;
            } else if (odd && has_zero(tin[j])) {
                out_perm[dest] = id[q] - g.base;
                if (dr != s0) out_lcp[dest] = g.depth + nz_bytes(tin[j]);
            } else {
                uint32_t delta = odd ? 8u : ((j == 0 || j == g.v) ? 0u : (uint32_t)lcpx[j]);
                uint64_t nk = kk[q];
                if (delta) {
                    if (has_zero(nk) && delta < 8)
                        nk = nk << (8 * delta);
                    else
                        nk = load_key(chars, offsets[id[q]] + g.depth + delta);
                }
                key_out[dest] = nk;
                idx_out[dest] = id[q];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// K8: base case in LDS.  Sorts a bucket of <= T strings by (key, index);
// equal keys without a terminator are refreshed 8 bytes deeper and sorted
// again inside their run (multikey refinement, Section 2.1), until every
// neighbouring pair is decided.  Emits perm and the LCPs inside the bucket.

__device__ __forceinline__ bool less3(uint16_t ga, uint64_t ka, uint32_t ia, uint16_t gb,
                                      uint64_t kb, uint32_t ib) {
    if (ga != gb) return ga < gb;
    if (ka != kb) return ka < kb;
    return ia < ib;
}

__global__ __launch_bounds__(256) void k_base_sort(const Seg* items, const uint64_t* key0,
                                                   const uint64_t* key1, const uint32_t* idx0,
                                                   const uint32_t* idx1, const uint8_t* chars,
                                                   const uint64_t* offsets, uint32_t* out_perm,
                                                   uint32_t* out_lcp, uint32_t pmax) {
    extern __shared__ uint64_t dyn[];
    uint64_t* K = dyn;                         // pmax
    uint32_t* I = (uint32_t*)(K + pmax);       // pmax
    uint32_t* L = I + pmax;                    // pmax
    uint16_t* G = (uint16_t*)(L + pmax);       // pmax
    uint8_t* Ur = (uint8_t*)(G + pmax);        // pmax
    __shared__ uint32_t tmp[kWG + 1];
    const Seg it = items[blockIdx.x];
    const uint32_t buf = it.depth >> 31;
    uint32_t h = it.depth & ~kBufBit;
    const uint32_t n = it.size;
    uint32_t P = 1;
    while (P < n) P <<= 1;
    const uint64_t* kin = buf ? key1 : key0;
    const uint32_t* iin = buf ? idx1 : idx0;
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < P; i += kWG) {
        if (i < n) {
            K[i] = kin[it.begin + i];
            I[i] = iin[it.begin + i];
            G[i] = 0;
        } else {
            K[i] = ~0ull;
            I[i] = ~0u;
            G[i] = 0xFFFF;
        }
        L[i] = 0;
        Ur[i] = 0;
    }
    __syncthreads();
    for (;;) {
        for (uint32_t kk = 2; kk <= P; kk <<= 1) {
            for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
                for (uint32_t i = tid; i < P / 2; i += kWG) {
                    uint32_t lo = 2 * i - (i & (j - 1)), hi = lo + j;
                    bool up = (lo & kk) == 0;
                    uint16_t ga = G[lo], gb = G[hi];
                    uint64_t ka = K[lo], kb = K[hi];
                    uint32_t ia = I[lo], ib = I[hi];
                    if (less3(gb, kb, ib, ga, ka, ia) == up) {
                        G[lo] = gb; G[hi] = ga;
                        K[lo] = kb; K[hi] = ka;
                        I[lo] = ib; I[hi] = ia;
                    }
                }
                __syncthreads();
            }
        }
        int any = 0;
        for (uint32_t i = tid; i < n; i += kWG) {
            uint8_t un = 0;
            if (i > 0 && G[i] == G[i - 1]) {
                if (K[i] == K[i - 1] && !has_zero(K[i]))
                    un = 1;
                else
                    L[i] = h + lcp8(K[i - 1], K[i]);
            }
            Ur[i] = un;
            any |= un;
        }
        any = __syncthreads_or(any);
        if (!any) break;
        // run starts: st(i) = max_{j <= i, pair (j-1, j) decided} j
        const uint32_t per = (n + kWG - 1) / kWG;
        const uint32_t b0 = tid * per;
        uint32_t mxv = 0;
        for (uint32_t i = b0; i < b0 + per && i < n; ++i)
            if (!Ur[i]) mxv = i;
        tmp[tid] = mxv;
        __syncthreads();
        for (uint32_t off = 1; off < (uint32_t)kWG; off <<= 1) {
            uint32_t x = tid >= off ? tmp[tid - off] : 0u;
            __syncthreads();
            if (x > tmp[tid]) tmp[tid] = x;
            __syncthreads();
        }
        uint32_t runst = tid ? tmp[tid - 1] : 0u;
        for (uint32_t i = b0; i < b0 + per && i < n; ++i) {
            if (!Ur[i]) runst = i;
            bool active = Ur[i] || (i + 1 < n && Ur[i + 1]);
            if (active) {
                G[i] = (uint16_t)runst;
                K[i] = load_key(chars, offsets[I[i]] + h + 8);
            } else {
                G[i] = (uint16_t)i;
            }
        }
        h += 8;
        __syncthreads();
    }
    for (uint32_t i = tid; i < n; i += kWG) {
        out_perm[it.begin + i] = I[i] - it.base;
        if (i) out_lcp[it.begin + i] = L[i];
    }
}

// ---------------------------------------------------------------------------
// K9: LCPs at bucket boundaries.  A boundary between two buckets of a pass at
// depth h holds kLcpFlag | h; both strings share h bytes (the bucket
// invariant, Section 3.1 equation (1)) and differ after that.

__global__ __launch_bounds__(256) void k_lcp_fix(const uint8_t* chars, const uint64_t* offsets,
                                                 const uint64_t* set_begin, uint32_t num_sets,
                                                 uint32_t n, const uint32_t* out_perm,
                                                 uint32_t* out_lcp) {
    uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 || p >= n) return;
    uint32_t l = out_lcp[p];
    if (!(l & kLcpFlag)) return;
    uint32_t h = l & ~kLcpFlag;
    uint32_t base = 0;
    if (set_begin) {  // last set whose first position is <= p
        uint32_t lo = 0, hi = num_sets - 1;
        while (lo < hi) {
            uint32_t mid = (lo + hi + 1) >> 1;
            if (set_begin[mid] <= p) lo = mid; else hi = mid - 1;
        }
        base = (uint32_t)set_begin[lo];
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
    out_lcp[p] = h;
}

// ---------------------------------------------------------------------------
// building block: classification against caller-given sorted splitters

__global__ __launch_bounds__(256) void k_tree_from_sorted(const uint64_t* splitters, uint32_t v,
                                                          uint32_t d, uint64_t* tree_lo,
                                                          uint64_t* tree_in) {
    for (uint32_t j = threadIdx.x; j < v; j += kWG) {
        tree_lo[inorder_node(j, d)] = splitters[j];
        tree_in[j] = splitters[j];
    }
    if (threadIdx.x == 0) {
        tree_lo[0] = 0;
        tree_in[v] = 0;
    }
}

template <int U>
__global__ __launch_bounds__(256) void k_classify_plain(const uint64_t* keys, uint32_t n,
                                                        const uint64_t* tree_lo,
                                                        const uint64_t* tree_in, uint32_t v,
                                                        uint32_t d, uint16_t* out) {
    extern __shared__ uint64_t dyn[];
    uint64_t* t = dyn;
    uint64_t* tin = t + (v + 1);
    for (uint32_t i = threadIdx.x; i <= v; i += kWG) {
        t[i] = tree_lo[i];
        tin[i] = tree_in[i];
    }
    __syncthreads();
    const uint32_t base = blockIdx.x * (kWG * U);
    uint64_t kk[U];
    uint32_t b[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
        uint32_t pos = base + q * kWG + threadIdx.x;
        kk[q] = pos < n ? keys[pos] : 0ull;
    }
    classify_u<U>(t, tin, d, v, kk, b);
#pragma unroll
    for (int q = 0; q < U; ++q) {
        uint32_t pos = base + q * kWG + threadIdx.x;
        if (pos < n) out[pos] = (uint16_t)b[q];
    }
}

// ---------------------------------------------------------------------------
// host-side launchers

#define S5_LAUNCH(kern, grid, block, lds, stream, ...)                                  \
    hipLaunchKernelGGL(kern, grid, block, lds, stream, __VA_ARGS__)

void launch_init_keys(const uint8_t* chars, const uint64_t* offsets, uint32_t n, uint64_t* key,
                      uint32_t* idx, hipStream_t st) {
    if (!n) return;
    S5_LAUNCH(k_init_keys, dim3((n + 255) / 256), dim3(256), 0, st, chars, offsets, n, key, idx);
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

void launch_sample_tree(uint32_t n_large, const LSeg* lseg, const uint64_t* key_in,
                        uint32_t alpha, uint32_t vmax, uint64_t seed, uint64_t* tree_lo,
                        uint64_t* tree_in, uint8_t* tree_lcp, uint32_t* unit_tab,
                        uint32_t* chunk_tab, hipStream_t st) {
    uint32_t m = alpha * (vmax + 1) - 1, P = 1;
    while (P < m) P <<= 1;
    S5_LAUNCH(k_sample_tree, dim3(n_large), dim3(kWG), (size_t)P * 8, st, lseg, key_in, alpha,
              seed, tree_lo, tree_in, tree_lcp, unit_tab, chunk_tab);
}

void launch_classify(uint32_t units, uint32_t unroll, const LSeg* lseg, const uint32_t* unit_tab,
                     const uint64_t* key_in, const uint64_t* tree_lo, const uint64_t* tree_in,
                     uint16_t* bid, uint32_t* cm, uint32_t vmax, uint32_t kmax, hipStream_t st) {
    size_t lds = (size_t)(vmax + 1) * 16 + (size_t)kWaves * kmax * 4;
    dim3 grid(units / kWaves);
    switch (unroll) {
        case 1: S5_LAUNCH(k_classify<1>, grid, dim3(kWG), lds, st, lseg, unit_tab, key_in, tree_lo, tree_in, bid, cm, vmax, kmax); break;
        case 2: S5_LAUNCH(k_classify<2>, grid, dim3(kWG), lds, st, lseg, unit_tab, key_in, tree_lo, tree_in, bid, cm, vmax, kmax); break;
        case 8: S5_LAUNCH(k_classify<8>, grid, dim3(kWG), lds, st, lseg, unit_tab, key_in, tree_lo, tree_in, bid, cm, vmax, kmax); break;
        default: S5_LAUNCH(k_classify<4>, grid, dim3(kWG), lds, st, lseg, unit_tab, key_in, tree_lo, tree_in, bid, cm, vmax, kmax); break;
    }
}

void launch_colscan(uint32_t chunks, uint32_t kmax, const LSeg* lseg, const uint32_t* chunk_tab,
                    uint32_t* cm, uint32_t* cs, hipStream_t st) {
    S5_LAUNCH(k_colscan, dim3(chunks, (kmax + kWG - 1) / kWG), dim3(kWG), 0, st, lseg, chunk_tab,
              cm, cs);
}

void launch_bucket_plan(uint32_t n_large, const LSeg* lseg, uint32_t* cs, uint32_t* bstart,
                        const uint64_t* tree_in, const uint8_t* tree_lcp, const PlanCtx& ctx,
                        uint32_t next_buf, hipStream_t st) {
    S5_LAUNCH(k_bucket_plan, dim3(n_large), dim3(kWG), 0, st, lseg, cs, bstart, tree_in, tree_lcp,
              ctx, next_buf);
}

void launch_scatter(uint32_t units, uint32_t unroll, const LSeg* lseg, const uint32_t* unit_tab,
                    const uint16_t* bid, const uint64_t* key_in, const uint32_t* idx_in,
                    uint64_t* key_out, uint32_t* idx_out, const uint32_t* cm, const uint32_t* cs,
                    const uint32_t* bstart, const uint64_t* tree_in, const uint8_t* tree_lcp,
                    const uint8_t* chars, const uint64_t* offsets, uint32_t* out_perm,
                    uint32_t* out_lcp, uint32_t vmax, uint32_t kmax, hipStream_t st) {
    size_t lds = (size_t)(vmax + 1) * 8 + (size_t)(kmax + 1) * 4 + (size_t)kWaves * kmax * 4 +
                 (size_t)(vmax + 1);
    dim3 grid(units / kWaves);
#define S5_SC(Uv)                                                                            \
    S5_LAUNCH(k_scatter<Uv>, grid, dim3(kWG), lds, st, lseg, unit_tab, bid, key_in, idx_in,   \
              key_out, idx_out, cm, cs, bstart, tree_in, tree_lcp, chars, offsets, out_perm,  \
              out_lcp, vmax, kmax)
    switch (unroll) {
        case 1: S5_SC(1); break;
        case 2: S5_SC(2); break;
        case 8: S5_SC(8); break;
        default: S5_SC(4); break;
    }
#undef S5_SC
}

void launch_base_sort(uint32_t n_items, const Seg* items, const uint64_t* key0,
                      const uint64_t* key1, const uint32_t* idx0, const uint32_t* idx1,
                      const uint8_t* chars, const uint64_t* offsets, uint32_t* out_perm,
                      uint32_t* out_lcp, uint32_t T, hipStream_t st) {
    if (!n_items) return;
    uint32_t P = 1;
    while (P < T) P <<= 1;
    size_t lds = (size_t)P * (8 + 4 + 4 + 2 + 1);
    S5_LAUNCH(k_base_sort, dim3(n_items), dim3(kWG), lds, st, items, key0, key1, idx0, idx1,
              chars, offsets, out_perm, out_lcp, P);
}

void launch_lcp_fix(const uint8_t* chars, const uint64_t* offsets, const uint64_t* set_begin,
                    uint32_t num_sets, uint32_t n, const uint32_t* out_perm, uint32_t* out_lcp,
                    hipStream_t st) {
    if (n < 2) return;
    S5_LAUNCH(k_lcp_fix, dim3((n + 255) / 256), dim3(256), 0, st, chars, offsets, set_begin,
              num_sets, n, out_perm, out_lcp);
}

void launch_classify_plain(const uint64_t* keys, uint32_t n, const uint64_t* splitters,
                           uint32_t v, uint32_t d, uint64_t* tree_lo, uint64_t* tree_in,
                           uint16_t* out, hipStream_t st) {
    S5_LAUNCH(k_tree_from_sorted, dim3(1), dim3(kWG), 0, st, splitters, v, d, tree_lo, tree_in);
    if (!n) return;
    S5_LAUNCH(k_classify_plain<4>, dim3((n + kWG * 4 - 1) / (kWG * 4)), dim3(kWG),
              (size_t)(v + 1) * 16, st, keys, n, tree_lo, tree_in, v, d, out);
}

}  // namespace s5
