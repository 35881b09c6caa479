/*
 * Plain sequential CPU oracle for string sorting with an LCP array.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or helper with
 * the HIP library.
 *
 * What it computes (Bingmann & Sanders, "Parallel String Sample Sort",
 * Section 2 "Preliminaries"):
 *   - strings are zero-terminated byte arrays over the alphabet {1..sigma};
 *     the terminator 0 is not part of the alphabet;
 *   - the output is the permutation that lists the strings in lexicographic
 *     order of their unsigned bytes; equal strings are listed by ascending
 *     input index (the paper leaves ties open; this makes the output unique);
 *   - lcp[i] = lcp(x[i-1], x[i]) over the sorted sequence x, lcp[0] = 0,
 *     counting the equal bytes before the first mismatch or terminator;
 *   - D, the distinguishing prefix size: every string contributes
 *     min(|s|, max(lcp with its sorted neighbours) + 1) where |s| counts the
 *     terminator.
 *
 * How: multikey quicksort (Section 2.1, Bentley-Sedgewick): partition on the
 * character at the common prefix depth into <, = and > parts around a
 * pseudo-median pivot character; the = part recurses one character deeper;
 * small parts use insertion sort.  An explicit stack replaces recursion.  When
 * the = part's character is the terminator, all its strings are identical and
 * it is ordered by input index.  The LCP array comes from a separate,
 * explicit byte-by-byte pass over the sorted order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t lo, hi;   /* half-open range of the index array */
    uint64_t depth;    /* all strings in [lo, hi) share this many leading bytes */
} task_t;

static int cmp_u32(const void* a, const void* b) {
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return (x > y) - (x < y);
}

/* compare strings a and b starting at byte `depth`, unsigned bytes, then by index */
static int str_less(const uint8_t* chars, const uint64_t* offsets, uint32_t a,
                    uint32_t b, uint64_t depth) {
    const uint8_t* s = chars + offsets[a] + depth;
    const uint8_t* t = chars + offsets[b] + depth;
    for (;;) {
        if (*s != *t) return *s < *t;
        if (*s == 0) return a < b;
        ++s;
        ++t;
    }
}

static uint8_t ch(const uint8_t* chars, const uint64_t* offsets, uint32_t i,
                  uint64_t depth) {
    return chars[offsets[i] + depth];
}

static uint8_t median3(uint8_t a, uint8_t b, uint8_t c) {
    if (a < b) {
        if (b < c) return b;
        return a < c ? c : a;
    }
    if (a < c) return a;
    return b < c ? c : b;
}

static void swap32(uint32_t* x, uint64_t i, uint64_t j) {
    uint32_t t = x[i];
    x[i] = x[j];
    x[j] = t;
}

/* Sort idx[0..n) by (string, index).  Returns 0, or -1 if memory runs out. */
int oracle_sort_idx(const uint8_t* chars, const uint64_t* offsets, uint32_t* idx,
                    uint64_t n) {
    uint64_t cap = 1024, top = 0;
    task_t* st;
    if (n <= 1) return 0;
    st = (task_t*)malloc(cap * sizeof(task_t));
    if (!st) return -1;
    st[top++] = (task_t){0, n, 0};
    while (top) {
        task_t t = st[--top];
        uint64_t size = t.hi - t.lo;
        if (size <= 1) continue;
        if (size < 16) {
            /* insertion sort on (bytes from depth, index) */
            for (uint64_t i = t.lo + 1; i < t.hi; ++i) {
                uint32_t v = idx[i];
                uint64_t j = i;
                while (j > t.lo && str_less(chars, offsets, v, idx[j - 1], t.depth)) {
                    idx[j] = idx[j - 1];
                    --j;
                }
                idx[j] = v;
            }
            continue;
        }
        uint8_t c = median3(ch(chars, offsets, idx[t.lo], t.depth),
                            ch(chars, offsets, idx[t.lo + size / 2], t.depth),
                            ch(chars, offsets, idx[t.hi - 1], t.depth));
        /* three-way partition: [lo,lt) < c, [lt,gt) == c, [gt,hi) > c */
        uint64_t lt = t.lo, i = t.lo, gt = t.hi;
        while (i < gt) {
            uint8_t x = ch(chars, offsets, idx[i], t.depth);
            if (x < c)
                swap32(idx, lt++, i++);
            else if (x > c)
                swap32(idx, i, --gt);
            else
                ++i;
        }
        if (top + 3 > cap) {
            task_t* ns = (task_t*)realloc(st, 2 * cap * sizeof(task_t));
            if (!ns) {
                free(st);
                return -1;
            }
            st = ns;
            cap *= 2;
        }
        st[top++] = (task_t){t.lo, lt, t.depth};
        st[top++] = (task_t){gt, t.hi, t.depth};
        if (c == 0) {
            /* every string in the = part ends here: identical strings */
            qsort(idx + lt, gt - lt, sizeof(uint32_t), cmp_u32);
        } else {
            st[top++] = (task_t){lt, gt, t.depth + 1};
        }
    }
    free(st);
    return 0;
}

/* lcp of two zero-terminated strings: equal bytes before mismatch or terminator */
static uint64_t lcp2(const uint8_t* s, const uint8_t* t) {
    uint64_t k = 0;
    while (s[k] == t[k] && s[k] != 0) ++k;
    return k;
}

/* Explicit LCP pass over a sorted order (Section 2: lcp_x(i) = lcp(x_{i-1}, x_i)). */
void oracle_lcp(const uint8_t* chars, const uint64_t* offsets, const uint32_t* perm,
                uint64_t n, uint32_t* lcp) {
    if (n == 0) return;
    lcp[0] = 0;
    for (uint64_t i = 1; i < n; ++i)
        lcp[i] = (uint32_t)lcp2(chars + offsets[perm[i - 1]], chars + offsets[perm[i]]);
}

/* Whole result: perm (input index of the i-th smallest string) and lcp. */
int oracle_sort(const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                uint32_t* perm, uint32_t* lcp) {
    for (uint32_t i = 0; i < n; ++i) perm[i] = i;
    if (oracle_sort_idx(chars, offsets, perm, n) != 0) return -1;
    oracle_lcp(chars, offsets, perm, n, lcp);
    return 0;
}

/* Many independent sets: set s is strings [set_begin[s], set_begin[s+1]);
 * perm holds set-local indices and lcp restarts at 0 on every set. */
int oracle_sort_batched(const uint8_t* chars, const uint64_t* offsets,
                        const uint64_t* set_begin, uint32_t num_sets, uint32_t* perm,
                        uint32_t* lcp) {
    for (uint32_t s = 0; s < num_sets; ++s) {
        uint64_t b = set_begin[s], e = set_begin[s + 1];
        if (e < b) return -1;
        if (oracle_sort(chars, offsets + b, (uint32_t)(e - b), perm + b, lcp + b) != 0)
            return -1;
    }
    return 0;
}

/* Distinguishing prefix size D (Section 2) from a sorted order and its LCPs. */
uint64_t oracle_dist_prefix(const uint8_t* chars, const uint64_t* offsets,
                            const uint32_t* perm, const uint32_t* lcp, uint64_t n) {
    uint64_t d = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t len = strlen((const char*)(chars + offsets[perm[i]])) + 1;
        uint64_t l = lcp[i];
        uint64_t r = i + 1 < n ? lcp[i + 1] : 0;
        uint64_t m = (l > r ? l : r) + 1;
        d += m < len ? m : len;
    }
    return d;
}

/* ---- checks of results too large to recompute -------------------------------
 * Both follow the definition of the output (Section 2): perm lists every
 * input index of a set exactly once, neighbours are in non-descending string
 * order (equal strings by ascending index), and lcp[i] is the LCP of the
 * neighbours, 0 at a set's first slot. */

/* 1 if perm restricted to every set is a permutation of 0..|set|-1, else 0
 * (set_begin NULL: one set of n). */
int oracle_check_perm(const uint32_t* perm, const uint64_t* set_begin, uint32_t num_sets,
                      uint64_t n) {
    uint8_t* seen = (uint8_t*)calloc(n ? n : 1, 1);
    if (!seen) return -1;
    int ok = 1;
    uint32_t ns = set_begin ? num_sets : 1;
    for (uint32_t s = 0; s < ns && ok; ++s) {
        uint64_t b = set_begin ? set_begin[s] : 0, e = set_begin ? set_begin[s + 1] : n;
        for (uint64_t i = b; i < e; ++i) {
            uint64_t g = b + perm[i];
            if (perm[i] >= e - b || seen[g]) {
                ok = 0;
                break;
            }
            seen[g] = 1;
        }
    }
    free(seen);
    return ok;
}

/* 1 if the pair (perm[p-1], perm[p]) is out of order or lcp[p] is wrong
 * (lcp must be 0 at a set's first slot), else 0. */
static int pair_bad(const uint8_t* chars, const uint64_t* offsets, const uint64_t* set_begin,
                    uint32_t num_sets, uint64_t n, const uint32_t* perm, const uint32_t* lcp,
                    uint64_t p) {
    if (p >= n) return 1;
    uint64_t b = 0, e = n;
    if (set_begin) { /* last set starting at or before p */
        uint32_t lo = 0, hi = num_sets - 1;
        while (lo < hi) {
            uint32_t mid = (lo + hi + 1) / 2;
            if (set_begin[mid] <= p) lo = mid; else hi = mid - 1;
        }
        b = set_begin[lo];
        e = set_begin[lo + 1];
    }
    if (perm[p] >= e - b) return 1;
    if (p == b) return lcp[p] != 0;
    if (perm[p - 1] >= e - b) return 1;
    uint32_t x = (uint32_t)(b + perm[p - 1]), y = (uint32_t)(b + perm[p]);
    if (!str_less(chars, offsets, x, y, 0)) return 1;
    return lcp2(chars + offsets[x], chars + offsets[y]) != lcp[p];
}

/* Number of the given positions whose pair (perm[p-1], perm[p]) is out of
 * order or whose lcp[p] is wrong (lcp must be 0 at a set's first slot). */
uint64_t oracle_check_pairs(const uint8_t* chars, const uint64_t* offsets,
                            const uint64_t* set_begin, uint32_t num_sets, uint64_t n,
                            const uint32_t* perm, const uint32_t* lcp,
                            const uint64_t* positions, uint64_t count) {
    uint64_t bad = 0;
    for (uint64_t q = 0; q < count; ++q)
        bad += (uint64_t)pair_bad(chars, offsets, set_begin, num_sets, n, perm, lcp, positions[q]);
    return bad;
}

/* The same check at every position 0..n-1.  Positions are independent, so
 * disjoint ranges of them are checked by `threads` OpenMP threads (a checker
 * only: the sorting oracle above stays sequential). */
uint64_t oracle_check_all_pairs(const uint8_t* chars, const uint64_t* offsets,
                                const uint64_t* set_begin, uint32_t num_sets, uint64_t n,
                                const uint32_t* perm, const uint32_t* lcp, int threads) {
    uint64_t bad = 0;
    int64_t nn = (int64_t)n;
#pragma omp parallel for num_threads(threads) reduction(+ : bad) schedule(static, 65536)
    for (int64_t p = 0; p < nn; ++p)
        bad += (uint64_t)pair_bad(chars, offsets, set_begin, num_sets, n, perm, lcp, (uint64_t)p);
    return bad;
}
