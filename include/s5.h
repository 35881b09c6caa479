/*
 * s5.h -- super scalar string sample sort (S^5) on one MI355X (gfx950).
 *
 * Problem (Bingmann & Sanders, "Parallel String Sample Sort", Section 2,
 * "Preliminaries"): n zero-terminated strings over the alphabet {1..255},
 * given as one arena of bytes plus the start offset of every string (the
 * paper's array of string pointers).  Output: the permutation that lists the
 * strings in lexicographic order of their unsigned bytes, and the LCP array of
 * that order, lcp[i] = lcp(x[i-1], x[i]).  The method is S^5 (Section 3.1):
 * splitter sampling, a ternary splitter tree with equality buckets over 8-byte
 * big-endian key prefixes, classification, counting, prefix sum and
 * out-of-place redistribution, recursing on the buckets.
 *
 * Conventions shared by every entry point:
 *   - Pointers named chars, offsets, set_begin, out_perm, out_lcp and
 *     workspace are DEVICE pointers; cfg and host_out are HOST pointers.
 *   - chars: the arena.  Each string runs from chars[offsets[i]] to its first
 *     0 byte.  Strings may overlap (e.g. all suffixes of one text) and offsets
 *     need not be increasing.  The library only reads aligned 8-byte words that
 *     lie in a 4 KiB page holding at least one byte of some string, so it
 *     never touches memory outside the arena's pages.  No string may be 2^31
 *     bytes or longer.
 *   - out_perm[i]: input index of the i-th smallest string; equal strings are
 *     listed by ascending input index, which makes the output unique.
 *   - out_lcp[0] = 0; out_lcp[i] = number of equal leading bytes of strings
 *     out_perm[i-1] and out_perm[i], not counting the terminator.
 *   - Every call is ordered on `stream` (a hipStream_t of the caller's HIP
 *     runtime; 0 = the null stream).  Sorting waits on `stream` between
 *     recursion levels (the host reads one small counter block per level to
 *     size the next launches), so a sort call returns when its results are
 *     complete on the device side of `stream`; it cannot be captured into a
 *     caller's graph (s5_sort_batched captures and replays its own).
 *   - The caller owns every input, output and user workspace; the library
 *     owns only its internal workspace pool, freed by s5_release().
 *   - Inputs are never written.  Outputs may not alias inputs.
 *   - Errors are returned as status codes (never thrown across this ABI).
 */
#ifndef S5_H
#define S5_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define S5_OK 0
#define S5_ERR_INVALID (-1) /* NULL pointer with n > 0, bad config or bad set table */
#define S5_ERR_NOMEM (-2)   /* workspace missing/too small or allocation failed */
#define S5_ERR_HIP (-3)     /* HIP runtime error */
#define S5_ERR_DEVICE (-4)  /* device status word set (a device-side capacity check failed) */
#define S5_ERR_TOO_LARGE (-5) /* s5_sort_static: the sort needs more than the static scratch array */

/* classifier: the descent through the splitter tree (Section 3.1,
 * "Implementation Details"; the output never depends on it) */
#define S5_CLASSIFY_UNROLL 0u /* branch-free descent of every level, one equality
                                 test at the leaf against the in-order splitter */
#define S5_CLASSIFY_EQUAL 1u  /* an equality test at every node; a descent stops at
                                 the first splitter equal to its key (the bucket
                                 index follows from the node's level-order index
                                 by bit operations) and a wavefront leaves the tree
                                 once all its descents have stopped */
#define S5_CLASSIFY_JUMP 2u   /* the Unroll descent started from a jump table
                                 (appendix A, "Jump tables"): the bits of a key
                                 after the common prefix of the first and last
                                 splitter (up to d + 2 of them, at most 12) index a
                                 table, built with the tree, of the node where
                                 the path stops being the same for all keys
                                 with those bits; keys outside the splitter
                                 range take buckets 0 and 2v directly */

/* alphabet: the characters a key holds (appendix A, "Alphabet compression";
 * the output never depends on it) */
#define S5_ALPHABET_BYTES 0u /* 8 characters (bytes) per 64-bit key */
#define S5_ALPHABET_AUTO 1u  /* the bytes of a sample of the strings (up to 65536
                                strings, up to 256 bytes each) are taken as the
                                alphabet; with at most 7 byte values (DNA: 4) each
                                character is sorted as an order-preserving 3-bit
                                code, 21 characters per key.  Every key load
                                checks its bytes; a byte outside the alphabet makes
                                the call sort again with byte keys */

/* distribution: how a level's strings move to their buckets (appendix A,
 * "Multipass data distribution"; the output never depends on it) */
#define S5_DISTRIBUTE_ONE_PASS 0u /* one stable move per level, by bucket id */
#define S5_DISTRIBUTE_TWO_PASS 1u /* two stable moves per level by the two digits of
                                     the bucket id, low digit first (a least-
                                     significant-digit radix sort on the ids): each
                                     move has at most 64 destinations per segment,
                                     whatever the number of buckets.  Host-driven
                                     sorts only: s5_sort_batched and
                                     s5_sort_batched_tuned return S5_ERR_INVALID */

/* splitter_mode */
#define S5_SPLIT_SAMPLED 0u /* splitters from a pseudo-random sample (Section 3.1) */
#define S5_SPLIT_LEARNED 1u /* splitters proposed by a small learned CDF model */

/* Tuning knobs.  A NULL config, or a 0 in any field, selects the default.
 * No choice here changes the output, only the speed. */
typedef struct s5_config {
    uint32_t splitters;      /* most splitters per distribution pass, v = 2^d - 1,
                                7 <= v <= 1023 (Section 3.1 "Implementation
                                Details"; default 255) */
    uint32_t oversample;     /* oversampling factor alpha (Section 2.3; default 2) */
    uint32_t unroll;         /* interleaved tree descents per lane: 1, 2, 4 or 8
                                (Section 3.1; default 4) */
    uint32_t tile;           /* minimum strings per tile (the range one workgroup
                                classifies and redistributes), a multiple of 64
                                (default 2048) */
    uint32_t base_threshold; /* buckets of at most this many strings are finished
                                by the LDS base-case sorter (Section 3.1
                                "Parallelization", the size-classed sub-algorithms;
                                64 <= T <= 2048, default 1024) */
    uint32_t splitter_mode;  /* S5_SPLIT_SAMPLED or S5_SPLIT_LEARNED */
    float imbalance_bound;   /* learned mode: fall back to sampled splitters when a
                                range bucket exceeds this many times the ideal
                                size (default 4) */
    uint64_t seed;           /* sampling / training seed; the output never depends on it */
    uint32_t graph_levels;   /* batched sorts: distribution levels captured in the
                                sort's hipGraph (0 = 12, at most 64); deeper inputs
                                finish with host-driven passes after the graph */
    uint32_t classifier;     /* S5_CLASSIFY_UNROLL (default), S5_CLASSIFY_EQUAL or
                                S5_CLASSIFY_JUMP */
    uint32_t alphabet;       /* S5_ALPHABET_BYTES (default) or S5_ALPHABET_AUTO */
    uint32_t distribution;   /* S5_DISTRIBUTE_ONE_PASS (default) or
                                S5_DISTRIBUTE_TWO_PASS */
} s5_config;

/* Counters of the last completed sort on a stream. */
typedef struct s5_stats {
    uint32_t passes;        /* distribution levels run */
    uint32_t fallbacks;     /* learned-splitter passes replaced by sampled splitters */
    uint64_t moved_M;       /* strings moved by distribution passes, summed over passes */
    uint64_t max_bucket;    /* largest bucket produced by the first pass */
    double entropy_bits;    /* sum_i (|b_i|/n) log2(n/|b_i|) over the first pass's
                               buckets (appendix A, "Adaptivity") */
    size_t workspace_bytes; /* device workspace the sort used */
    uint64_t base_items;    /* buckets finished by the base-case sorter */
    uint64_t segments;      /* segments distributed, summed over passes */
    uint32_t char_bits;     /* bits per character of the keys sorted by (8: bytes;
                               3: alphabet compression) */
    uint32_t alphabet_retries; /* sorts redone with byte keys after a byte outside
                                  the sampled alphabet */
    uint32_t learned_proposals; /* learned splitter proposals made (S5_SPLIT_LEARNED) */
    uint32_t root_depth;    /* bytes every string was found to share at its start
                               (byte keys): the common prefix of a sample's
                               smallest and largest first key, checked for every
                               string and skipped before the first level (0 when
                               some string lacks it) */
    double imbalance_mean;  /* over those proposals: the largest range bucket of the
                               proposal's own training sample, as a multiple of the
                               ideal share m / (v + 1) (mean and maximum; a
                               proposal above imbalance_bound is replaced) */
    double imbalance_max;
    uint64_t moved_one_bucket; /* of moved_M: strings of segments that all fell into
                                  one bucket (moved only to advance their depth) */
} s5_stats;

/* Sort n strings.  perm and lcp as described above.  Uses the internal
 * workspace pool of the current device (grown on demand).
 * Returns S5_OK, S5_ERR_INVALID, S5_ERR_NOMEM, S5_ERR_HIP or S5_ERR_DEVICE. */
int s5_sort(const uint8_t* chars, const uint64_t* offsets, uint32_t n, uint32_t* out_perm,
            uint32_t* out_lcp, hipStream_t stream);

/* As s5_sort with explicit tuning and, optionally, a caller workspace of
 * workspace_bytes >= s5_workspace_bytes(n, cfg) (NULL = internal pool).
 * chars_len: bytes in the arena, or 0 = unknown.  When it is given, the device
 * checks that every offsets[i] < chars_len and that chars[chars_len - 1] is a
 * terminator (so every string ends inside the arena); a failed check stops
 * the sort before anything is written to out_perm or out_lcp beyond what a
 * set's first slot receives, and returns S5_ERR_INVALID. */
int s5_sort_ex(const uint8_t* chars, uint64_t chars_len, const uint64_t* offsets, uint32_t n,
               uint32_t* out_perm, uint32_t* out_lcp, const s5_config* cfg, void* workspace,
               size_t workspace_bytes, hipStream_t stream);

/* Device workspace bytes that a sort of n strings with cfg needs. */
size_t s5_workspace_bytes(uint32_t n, const s5_config* cfg);

/* Bytes of the static scratch array of s5_sort_static (per device). */
#define S5_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate (tight serving loops, harnesses that forbid
 * hipMalloc or pinned host allocations): s5_sort_ex with its workspace taken
 * from a fixed device array of S5_STATIC_SCRATCH_BYTES that the library
 * reserves on every device it runs on until the process ends.  Allocates no
 * device or pinned host memory (counters are read back into static host
 * memory) and takes no profiling events.  The caller passes the inputs and
 * the outputs as for s5_sort_ex.
 *
 * Limit: s5_workspace_bytes(n, cfg) <= S5_STATIC_SCRATCH_BYTES (at the
 * defaults about 1.1M strings); a larger sort returns S5_ERR_TOO_LARGE before
 * any device work.  All calls on one device share its array, which keeps the
 * last call's contents (a sort clears its counters with a kernel and writes
 * every other value before reading it).  Two sorts using the array at once
 * would race; here every call holds the library's lock and finishes on the
 * device before it returns, so calls from one process never overlap.
 * Returns what s5_sort_ex returns, or S5_ERR_TOO_LARGE. */
int s5_sort_static(const uint8_t* chars, uint64_t chars_len, const uint64_t* offsets, uint32_t n,
                   uint32_t* out_perm, uint32_t* out_lcp, const s5_config* cfg,
                   hipStream_t stream);

/* Sort num_sets independent sets in one call.  Set s holds the strings
 * offsets[set_begin[s] .. set_begin[s+1]); set_begin (num_sets+1 entries,
 * DEVICE memory, non-decreasing, set_begin[0] = 0) fixes where each set's
 * results go: out_perm holds set-local indices and out_lcp is 0 at every
 * set's first slot.  n = set_begin[num_sets] < 2^32.  The device checks the
 * table (set_begin[s] <= set_begin[s+1] <= n for every s); a set that fails
 * is not sorted or written, and the call returns S5_ERR_INVALID.  chars_len
 * is checked as for s5_sort_ex.
 *
 * All sets are sorted together: every distribution pass covers the segments
 * of every set (the segmented form of the level-by-level recursion of
 * Section 3.1), and the first cfg->graph_levels passes, the base case and the
 * boundary LCPs are one hipGraph, captured on the first call and replayed by
 * later calls with the same pointers, sizes and cfg (kernels only; work
 * counts are read on the device).  Reads set_begin[0] and set_begin[num_sets]
 * back (synchronizes the stream) and synchronizes again at the end. */
int s5_sort_batched(const uint8_t* chars, uint64_t chars_len, const uint64_t* offsets,
                    const uint64_t* set_begin, uint32_t num_sets, uint32_t* out_perm,
                    uint32_t* out_lcp, const s5_config* cfg, hipStream_t stream);

/* Per-set parameters of s5_sort_batched_tuned (the entries of an autotuned
 * table; 0 = the value from cfg).  The paper tunes such thresholds by hand
 * (Section 3.1 "Implementation Details"). */
typedef struct s5_set_tuning {
    uint16_t splitters;       /* most splitters per pass in this set, 2^d - 1, 7..1023 */
    uint16_t base_threshold;  /* base-case threshold T of this set, 64..2048 */
    uint32_t tile;            /* minimum strings per tile, multiple of 64, <= 2^20 */
} s5_set_tuning;

/* s5_sort_batched with per-set parameters: set_tuning is a HOST array of
 * num_sets entries (NULL = cfg for every set), validated and copied before
 * the call returns.  The launch-wide limits (largest T and tree depth) are
 * the maxima over the sets and cfg; cfg->unroll applies to every set.
 * Returns S5_ERR_INVALID for an entry out of range. */
int s5_sort_batched_tuned(const uint8_t* chars, uint64_t chars_len, const uint64_t* offsets,
                          const uint64_t* set_begin, uint32_t num_sets,
                          const s5_set_tuning* set_tuning, uint32_t* out_perm, uint32_t* out_lcp,
                          const s5_config* cfg, hipStream_t stream);

/* Copy the counters of the last sort finished on `stream` to host_out.
 * Synchronizes `stream`; returns S5_ERR_DEVICE if that sort's device status
 * word reported a failure. */
int s5_stats_get(hipStream_t stream, s5_stats* host_out);

/* Human-readable text for a status code (static storage). */
const char* s5_strerror(int status);

/* Free the internal workspace pools of every device. */
void s5_release(void);


/* ---- building blocks ------------------------------------------------------
 * The two primitives below are the first steps of every distribution pass,
 * exported for callers that drive their own recursion and for step-level
 * checks.  Same conventions as above. */

/* out_keys[i] = the 8 bytes of string i that start at byte `depth`, packed
 * big-endian (first byte most significant) and zero from the terminator on,
 * so unsigned key order is lexicographic order of those bytes (Section 2.2,
 * caching of characters and super-alphabets; Section 3.1, w = 8 characters per
 * machine word).  Requires depth <= length of every string. */
int s5_prefix_keys(const uint8_t* chars, const uint64_t* offsets, uint32_t n, uint32_t depth,
                   uint64_t* out_keys, hipStream_t stream);

/* Ternary classification against v = 2^d - 1 splitters, 1 <= v <= 1023,
 * given in sorted (non-decreasing) order in DEVICE memory (Section 3.1 and
 * Figure 1): with j = number of splitters smaller than the key, the bucket is
 * 2j + 1 if splitter j equals the key, else 2j.  Buckets 0..2v. */
int s5_classify(const uint64_t* keys, uint32_t n, const uint64_t* splitters, uint32_t v,
                uint16_t* out_bucket, hipStream_t stream);

/* s5_classify with the descent `variant` (S5_CLASSIFY_UNROLL, S5_CLASSIFY_EQUAL
 * or S5_CLASSIFY_JUMP; Jump gives exactly the Unroll buckets).  With repeated splitters the Equal variant may name a
 * different one of the equal splitters' equality buckets than 2j + 1 (j the
 * first equal splitter): every key equal to a splitter x_j still lands in an
 * equality bucket of a splitter equal to it, and every other key in the range
 * bucket between its neighbouring splitters, so the partition and its order
 * are the same.  With distinct splitters both variants agree. */
int s5_classify_ex(const uint64_t* keys, uint32_t n, const uint64_t* splitters, uint32_t v,
                   uint32_t variant, uint16_t* out_bucket, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* S5_H */
