// Word-level helpers of S^5, usable on the device and on the host (the host
// side serves CPU checks of these helpers).  Keys are the next w = 8 bytes of
// a string packed big-endian, zero from the terminator on (Section 2.2,
// caching of characters and super-alphabets; Section 3.1, w characters per
// machine word), so unsigned 64-bit order is lexicographic byte order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace s5 {

#define S5_HD __host__ __device__ __forceinline__

// High bit of each byte set iff that byte of x is zero (exact, no false hits).
S5_HD uint64_t zero_byte_mask(uint64_t x) {
    const uint64_t L7 = 0x7F7F7F7F7F7F7F7Full;
    uint64_t t = ((x & L7) + L7) | x;
    return ~(t | L7);
}
S5_HD bool has_zero(uint64_t x) { return zero_byte_mask(x) != 0; }
// number of leading (most significant) nonzero bytes
S5_HD uint32_t nz_bytes(uint64_t x) {
    uint64_t z = zero_byte_mask(x);
    return z ? (uint32_t)(__builtin_clzll((unsigned long long)z) >> 3) : 8u;
}
// zero every byte from the first zero byte (most significant first) on
S5_HD uint64_t clip_at_zero(uint64_t k) {
    uint64_t z = zero_byte_mask(k);
    if (z == 0) return k;
    uint32_t q = (uint32_t)__builtin_clzll((unsigned long long)z) >> 3;
    return q == 0 ? 0ull : (k & (~0ull << (64 - 8 * q)));
}
// common leading bytes of two keys that are zero from their terminator on
S5_HD uint32_t lcp8(uint64_t a, uint64_t b) {
    return a == b ? nz_bytes(a) : (uint32_t)(__builtin_clzll((unsigned long long)(a ^ b)) >> 3);
}

// The 8 bytes at chars[pos..pos+8) as a big-endian key, zero from the first
// 0 byte on.  Reads the aligned word holding chars[pos] and, only when the
// string continues past that word, the next aligned word; both hold at least
// one byte of the string, so no read leaves the string's own words.
S5_HD uint64_t load_key(const uint8_t* chars, uint64_t pos) {
    uintptr_t a = (uintptr_t)(chars + pos);
    const uint64_t* w = (const uint64_t*)(a & ~(uintptr_t)7);
    uint32_t sh = (uint32_t)(a & 7) * 8;
    uint64_t k = __builtin_bswap64(w[0]) << sh;
    if (sh) {
        uint64_t valid = ~0ull << sh;
        if ((zero_byte_mask(k) & valid) == 0) k |= __builtin_bswap64(w[1]) >> (64 - sh);
    }
    return clip_at_zero(k);
}

// Second key word of a string whose next 8 bytes after the first key are not
// known (a word of 8 bytes 0xFF, which a string may also hold, only costs a
// gather).
constexpr uint64_t kKeyUnknown = ~0ull;

// The 16 bytes at chars[pos..pos+16) as two keys: *k0 = bytes pos..pos+8,
// *k1 = bytes pos+8..pos+16, both big-endian and zero from the first 0 byte
// on.  The (up to three) aligned words holding those bytes are read at once
// when they lie in the 4 KiB page of chars[pos]; otherwise in order, stopping
// after the first word that holds the terminator.  Either way every word read
// lies in a page that holds a byte of the string.
S5_HD void load_key16(const uint8_t* chars, uint64_t pos, uint64_t* k0, uint64_t* k1) {
    uintptr_t a = (uintptr_t)(chars + pos);
    const uint64_t* w = (const uint64_t*)(a & ~(uintptr_t)7);
    uint32_t sh = (uint32_t)(a & 7) * 8;
    uint64_t x, y, z = 0;
    if ((a & 4095) < 4080) {
        // all three words lie in the 4 KiB page of the first byte: read them at once
        x = __builtin_bswap64(w[0]) << sh;
        y = __builtin_bswap64(w[1]);
        z = __builtin_bswap64(w[2]);
        if (zero_byte_mask(x) & (~0ull << sh)) {
            *k0 = clip_at_zero(x);
            *k1 = 0;
            return;
        }
    } else {
        x = __builtin_bswap64(w[0]) << sh;
        if (zero_byte_mask(x) & (~0ull << sh)) {  // ends inside the first word
            *k0 = clip_at_zero(x);
            *k1 = 0;
            return;
        }
        y = __builtin_bswap64(w[1]);
        if (sh && !has_zero(y)) z = __builtin_bswap64(w[2]);
    }
    const uint64_t hi = sh ? x | (y >> (64 - sh)) : x;
    const uint64_t lo = sh ? (y << sh) | (z >> (64 - sh)) : y;
    *k0 = clip_at_zero(hi);
    *k1 = has_zero(*k0) ? 0ull : clip_at_zero(lo);
}

// The keys at chars[pos], chars[pos + 8], ..., chars[pos + 8 (N - 1)] (each as
// load_key gives it; all zero past the terminator).  The N + 1 aligned words
// holding those bytes are read at once when they lie in the 4 KiB page of
// chars[pos]; otherwise in order, stopping after the word that holds the
// terminator.  Every word read lies in a page that holds a byte of the string.
template <int N>
S5_HD void load_key_run(const uint8_t* chars, uint64_t pos, uint64_t (&out)[N]) {
    const uintptr_t a = (uintptr_t)(chars + pos);
    const uint64_t* w = (const uint64_t*)(a & ~(uintptr_t)7);
    const uint32_t sh = (uint32_t)(a & 7) * 8;
    uint64_t x[N + 1];
    if ((a & 4088) + 8 * (N + 1) <= 4096) {
#pragma unroll
        for (int i = 0; i <= N; ++i) x[i] = __builtin_bswap64(w[i]);
    } else {
        bool end = false;
#pragma unroll
        for (int i = 0; i <= N; ++i) {
            x[i] = end ? 0ull : __builtin_bswap64(w[i]);
            end = end || (i == 0 ? (zero_byte_mask(x[0] << sh) & (~0ull << sh)) != 0
                                 : has_zero(x[i]));
        }
    }
    bool dead = false;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const uint64_t k = sh ? (x[i] << sh) | (x[i + 1] >> (64 - sh)) : x[i];
        out[i] = dead ? 0ull : clip_at_zero(k);
        dead = dead || has_zero(k);
    }
}

// Both key words of a string advanced by `delta` bytes (1..8), from what is
// known: the first word k0 is exact, the second k1 exact or kKeyUnknown.
// Returns false when the bytes are not all known (then a gather is needed).
S5_HD bool advance_key16(uint64_t* k0, uint64_t* k1, uint32_t delta) {
    const uint64_t x = *k0, y = *k1;
    if (has_zero(x)) {  // the string ends inside k0: everything after is zero
        *k0 = delta < 8 ? x << (8 * delta) : 0ull;
        *k1 = 0;
        return true;
    }
    if (y == kKeyUnknown) return false;
    const bool ends = has_zero(y);
    *k0 = delta < 8 ? (x << (8 * delta)) | (y >> (64 - 8 * delta)) : y;
    *k1 = ends ? (delta < 8 ? y << (8 * delta) : 0ull) : kKeyUnknown;
    return true;
}

// The two key words of a string advanced by `delta` bytes (1..8) when the
// 24 bytes k0, k1, k2 that follow the current depth are all known (zero past
// the terminator): both new words are exact.
S5_HD void advance_key24(uint64_t* k0, uint64_t* k1, uint64_t k2, uint32_t delta) {
    const uint64_t x = *k0, y = *k1;
    if (delta >= 8) {
        *k0 = y;
        *k1 = k2;
        return;
    }
    const uint32_t s = 8 * delta;
    *k0 = (x << s) | (y >> (64 - s));
    *k1 = (y << s) | (k2 >> (64 - s));
}

// ---------------------------------------------------------------------------
// Alphabet compression (appendix A, "Alphabet compression"): when only sigma'
// byte values occur, each character becomes an order-preserving code of b
// bits (code 0 is the terminator, the alphabet's bytes get 1..sigma' in byte
// order), and one 64-bit key holds w = floor(64 / b) characters, packed from
// the most significant bit down; the 64 - b w lowest bits stay zero.  Unsigned
// key order is again the lexicographic order of the characters, and a zero
// field is the end of the string (every field after it is zero too).  Bytes
// are the case b = 8, w = 8.  Depths and LCPs count characters (= bytes of
// the string) either way.
struct KeyCodec {
    uint32_t b;            // bits per character (8: plain bytes)
    uint32_t w;            // characters per key
    uint64_t hi;           // top bit of every character field
    uint64_t lo;           // the other bits of every character field
    uint32_t inv_b;        // ceil(2^16 / b): q / b = (q * inv_b) >> 16 for q <= 64
    uint32_t pad;
    const uint8_t* table;  // packed: byte -> code, 0xFF for a byte outside the alphabet
    uint32_t* status;      // packed: status word that a byte outside the alphabet sets
};

S5_HD KeyCodec make_codec(uint32_t b, const uint8_t* table, uint32_t* status) {
    KeyCodec c;
    c.b = b;
    c.w = 64 / b;
    c.hi = 0;
    c.lo = 0;
    for (uint32_t f = 0; f < c.w; ++f) {
        const uint32_t top = 63 - f * b;  // field f occupies bits [top, top - b + 1]
        c.hi |= 1ull << top;
        c.lo |= ((1ull << (b - 1)) - 1) << (top - b + 1);
    }
    c.inv_b = (65536u + b - 1) / b;
    c.pad = 0;
    c.table = table;
    c.status = status;
    return c;
}
S5_HD uint32_t codec_div(const KeyCodec& c, uint32_t q) { return (q * c.inv_b) >> 16; }
// top bit of every zero field of x (exact, as zero_byte_mask)
S5_HD uint64_t codec_zero_mask(const KeyCodec& c, uint64_t x) {
    const uint64_t t = ((x & c.lo) + c.lo) | x;
    return ~(t | c.lo) & c.hi;
}
S5_HD bool codec_has_end(const KeyCodec& c, uint64_t x) { return codec_zero_mask(c, x) != 0; }
// characters before the end of the string inside the key (w if it does not end)
S5_HD uint32_t codec_before_end(const KeyCodec& c, uint64_t x) {
    const uint64_t z = codec_zero_mask(c, x);
    return z ? codec_div(c, (uint32_t)__builtin_clzll((unsigned long long)z)) : c.w;
}
// common leading characters of two keys (for two distinct keys: the fields
// before the first that differs)
S5_HD uint32_t codec_lcp(const KeyCodec& c, uint64_t a, uint64_t b) {
    return a == b ? codec_before_end(c, a)
                  : codec_div(c, (uint32_t)__builtin_clzll((unsigned long long)(a ^ b)));
}
// the key `delta` characters (1 <= delta <= w) further on, from the key x and
// the key y that follows it
S5_HD uint64_t codec_shift_in(const KeyCodec& c, uint64_t x, uint64_t y, uint32_t delta) {
    if (delta >= c.w) return y;
    const uint32_t s = c.b * delta, spare = 64 - c.b * c.w;
    return (x << s) | ((y >> (c.b * (c.w - delta))) & ~((1ull << spare) - 1ull));
}
// advance_key16 for the codec: both key words advanced by delta characters
// from what is known (k1 exact or kKeyUnknown); false when a gather is needed
S5_HD bool codec_advance2(const KeyCodec& c, uint64_t* k0, uint64_t* k1, uint32_t delta) {
    const uint64_t x = *k0, y = *k1;
    if (codec_has_end(c, x)) {
        *k0 = delta < c.w ? x << (c.b * delta) : 0ull;
        *k1 = 0;
        return true;
    }
    if (y == kKeyUnknown) return false;
    *k0 = codec_shift_in(c, x, y, delta);
    *k1 = codec_has_end(c, y) ? (delta < c.w ? y << (c.b * delta) : 0ull) : kKeyUnknown;
    return true;
}
// advance_key24 for the codec (k0, k1, k2 all known)
S5_HD void codec_advance3(const KeyCodec& c, uint64_t* k0, uint64_t* k1, uint64_t k2,
                          uint32_t delta) {
    const uint64_t x = *k0, y = *k1;
    *k0 = codec_shift_in(c, x, y, delta);
    *k1 = codec_shift_in(c, y, k2, delta);
}
// Packed keys are 3-bit codes (alphabets of at most 7 byte values, such as
// DNA), 21 characters per key: field f of a key occupies bits 63-3f..61-3f.
constexpr uint32_t kPackBits = 3, kPackChars = 21;

// NK packed keys (21 characters each) from the raw big-endian words of a
// string (bytes zero from the terminator on), each byte mapped through
// `table`.  Returns true if some byte is outside the alphabet (table 0xFF).
// `fence()` runs after every raw word's eight lookups (on the device a
// scheduling barrier, so that only one word's lookups are in flight).
struct NoFence {
    S5_HD void operator()() const {}
};
template <int NR, int NK, class F = NoFence>
S5_HD bool pack3(const uint8_t* table, const uint64_t (&raw)[NR], uint64_t (&key)[NK],
                 F fence = F()) {
    static_assert(8 * NR >= (int)kPackChars * NK, "not enough raw bytes");
    uint32_t bad = 0;
#pragma unroll
    for (int k = 0; k < NK; ++k) key[k] = 0;
#pragma unroll
    for (int i = 0; i < (int)kPackChars * NK; ++i) {
        const uint32_t ch = (uint32_t)(raw[i >> 3] >> (56 - 8 * (i & 7))) & 0xFFu;
        const uint32_t code = table[ch];
        bad |= code & 0x80u;
        key[i / kPackChars] |= (uint64_t)(code & 7u) << (61 - 3 * (i % kPackChars));
        if ((i & 7) == 7) fence();
    }
    return bad != 0;
}

S5_HD uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// heap index (1-based level order) of the in-order splitter j in a tree of depth d
S5_HD uint32_t inorder_node(uint32_t j, uint32_t d) {
    uint32_t t = j + 1;
    uint32_t L = d - 1 - (uint32_t)__builtin_ctz(t);
    return (1u << L) + (t >> (d - L));
}

// in-order index of the splitter at level-order node i (1-based heap index,
// 1 <= i < 2^d) of a perfect tree of depth d: the inverse of inorder_node
S5_HD uint32_t node_inorder(uint32_t i, uint32_t d) {
    const uint32_t L = 31u - (uint32_t)__builtin_clz(i);
    return ((2u * (i - (1u << L)) + 1u) << (d - 1u - L)) - 1u;
}

// One level of the "Equal" descent (Section 3.1, the variant that tests for
// equality at every node and leaves the tree at the first splitter equal to
// the key): at node i, a key equal to its splitter is done, in the equality
// bucket 2j + 1 of the node's in-order index j (bit operations on i, no
// in-order array); otherwise i = 2i + [key > x_i].  Branch-free: a finished
// descent keeps its node.  After d levels, an unfinished descent sits at leaf
// i and its bucket is equal_leaf_bucket(i, d).
S5_HD void equal_step(const uint64_t* t, uint32_t d, uint64_t key, uint32_t& i, bool& done,
                      uint32_t& b) {
    const uint64_t x = t[i];
    const bool eq = !done && key == x;
    b = eq ? 2u * node_inorder(i, d) + 1u : b;
    done = done || eq;
    i = done ? i : 2u * i + (key > x ? 1u : 0u);
}
S5_HD uint32_t equal_leaf_bucket(uint32_t i, uint32_t d) { return 2u * (i - (1u << d)); }

// Two-pass distribution (appendix A, "Multipass data distribution"): a
// level's strings are moved twice, stably, by the two digits of their bucket
// id, the low digit first -- a least-significant-digit radix sort on the ids,
// so each pass has few destinations.  Ids of a tree of depth d have d + 1
// bits; the low digit takes the lower half, rounded up.
constexpr uint32_t kDigitLow = 1, kDigitHigh = 2;
// values of a digit: k for the whole id (dig 0), else 2^bits of that digit
// (the high digit only up to the largest id k - 1)
S5_HD uint32_t digit_low_bits(uint32_t d) { return (d + 2u) / 2u; }
S5_HD uint32_t digit_values(uint32_t k, uint32_t d, uint32_t dig) {
    const uint32_t r = digit_low_bits(d);
    return dig == 0 ? k : dig == kDigitLow ? (1u << r) : ((k - 1u) >> r) + 1u;
}
S5_HD uint32_t digit_of(uint32_t b, uint32_t d, uint32_t dig) {
    const uint32_t r = digit_low_bits(d);
    return dig == 0 ? b : dig == kDigitLow ? (b & ((1u << r) - 1u)) : (b >> r);
}
// bits of a digit's values (for the ballot match of equal digits)
S5_HD uint32_t digit_bits(uint32_t d, uint32_t dig) {
    const uint32_t r = digit_low_bits(d);
    return dig == 0 ? d + 1u : dig == kDigitLow ? r : d + 1u - r;
}

// The dispatcher hands workgroups to the chip's 8 XCDs in turn (workgroup b
// runs on XCD b mod 8), and every XCD has an L2 of its own.  xcd_unit(b, n)
// renumbers the n workgroups of a launch so that runs of kXcdRun consecutive
// units go to one XCD (a bijection of [0, n)): neighbouring units then share
// an L2, while every XCD still takes its turn along the whole launch.  In the
// last, partial group of 8 runs each XCD takes one contiguous range.
constexpr uint32_t kXcds = 8, kXcdRun = 16;
S5_HD uint32_t xcd_unit(uint32_t b, uint32_t n) {
    constexpr uint32_t S = kXcds * kXcdRun;
    const uint32_t g0 = b / S * S;
    if (g0 + S <= n) return g0 + (b % kXcds) * kXcdRun + (b % S) / kXcds;
    const uint32_t c = b - g0, m = n - g0;
    const uint32_t x = c % kXcds, j = c / kXcds, q = m / kXcds, r = m % kXcds;
    return g0 + x * q + (x < r ? x : r) + j;
}

// Jump table over the top key bits (appendix A, "Jump tables").  All keys
// between the first and the last splitter share the top `sh` bits of those
// two splitters; the next `a` bits index a table whose entry is the node at
// which the descent (i = 2i + [key > x_i]) stops being the same for every key
// with those bits.  The descent starts there, so its result is the plain
// descent's.  Keys below the first or above the last splitter take buckets 0
// and 2v directly.
struct JumpShape {
    uint32_t sh, a;  // common top bits of the splitter range; index bits (a = 0: no table)
};
S5_HD JumpShape jump_shape(uint64_t first, uint64_t last, uint32_t d) {
    JumpShape j;
    j.sh = first == last ? 64u : (uint32_t)__builtin_clzll((unsigned long long)(first ^ last));
    uint32_t a = d + 2 < 12 ? d + 2 : 12u;
    j.a = 64 - j.sh < a ? 64 - j.sh : a;
    return j;
}
S5_HD uint32_t jump_index(uint64_t key, JumpShape j) {
    return j.a ? (uint32_t)((key << j.sh) >> (64 - j.a)) : 0u;
}
// table entry for index p (t: level order, t[1..v], d levels; first is the
// smallest splitter)
S5_HD uint32_t jump_entry(const uint64_t* t, uint32_t d, uint64_t first, JumpShape j,
                          uint32_t p) {
    const uint64_t top = j.sh >= 64 ? first : (j.sh ? first & ~(~0ull >> j.sh) : 0ull);
    const uint32_t rest = 64 - j.sh - j.a;  // bits below the index
    const uint64_t lo = j.a ? top | ((uint64_t)p << rest) : top;
    const uint64_t hi = lo | (rest >= 64 ? ~0ull : ((1ull << rest) - 1));
    uint32_t i = 1;
    for (uint32_t L = 0; L < d; ++L) {
        const uint64_t x = t[i];
        if (x < lo) i = 2 * i + 1;       // every key with index p is greater
        else if (x >= hi) i = 2 * i;     // every key with index p is smaller or equal
        else break;
    }
    return i;
}

// The jump table of a tree (level order t[1..v]) into jt: entries p0,
// p0 + step, ... (a workgroup passes its thread index and size).
S5_HD void build_jump_table(const uint64_t* t, uint32_t d, uint32_t v, uint16_t* jt,
                            uint32_t p0, uint32_t step) {
    const uint64_t first = t[inorder_node(0, d)], last = t[inorder_node(v - 1, d)];
    const JumpShape js = jump_shape(first, last, d);
    for (uint32_t p = p0; p < (1u << js.a); p += step)
        jt[p] = (uint16_t)jump_entry(t, d, first, js, p);
}

// U interleaved branch-free descents followed by one equality test each
// (Section 3.1: the "unrolled" variant that only uses <= comparisons on the
// way down).  t: level order, t[1..v]; tin: in order, tin[0..v).
template <int U>
S5_HD void classify_u(const uint64_t* t, const uint64_t* tin, uint32_t d,
                                           uint32_t v, const uint64_t (&key)[U],
                                           uint32_t (&b)[U]) {
    uint32_t i[U];
#pragma unroll
    for (int q = 0; q < U; ++q) i[q] = 1;
    for (uint32_t L = 0; L < d; ++L) {
#pragma unroll
        for (int q = 0; q < U; ++q) i[q] = 2 * i[q] + (key[q] > t[i[q]] ? 1u : 0u);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
        uint32_t j = i[q] - (v + 1);
        bool eq = (j < v) && (tin[j] == key[q]);
        b[q] = 2 * j + (eq ? 1u : 0u);
    }
}

// One step of the recursive splitter selection (Section 3.1): for the sorted
// sample range smp[a..b), a < b, the node takes the middle sample x; its left
// child recurses on smp[a..lo) and its right child on smp[hi..b), where
// [lo, hi) is the run of samples equal to x.
S5_HD void select_node(const uint64_t* smp, uint32_t a, uint32_t b, uint64_t* x, uint32_t* lo,
                       uint32_t* hi) {
    uint32_t mid = (a + b) >> 1;
    uint64_t m = smp[mid];
    uint32_t l = a, h = mid;  // first index in [a, mid] with smp >= m
    while (l < h) {
        uint32_t md = (l + h) >> 1;
        if (smp[md] < m) l = md + 1; else h = md;
    }
    *lo = l;
    l = mid + 1;
    h = b;  // first index in (mid, b] with smp > m
    while (l < h) {
        uint32_t md = (l + h) >> 1;
        if (smp[md] <= m) l = md + 1; else h = md;
    }
    *hi = l;
    *x = m;
}

// Keys at chars[pos[c]] for every c with need[c], like load_key, for N
// strings at once: all first words are loaded before any is inspected, then
// all second words, so a thread has N gathers in flight instead of one.  Lanes
// with need[c] == false read the aligned word holding chars[0] instead (always
// a word of the arena) and leave out[c] unchanged.
template <int N>
S5_HD void load_keys(const uint8_t* chars, const uint64_t (&pos)[N], const bool (&need)[N],
                     uint64_t (&out)[N]) {
    const uint64_t* safe = (const uint64_t*)((uintptr_t)chars & ~(uintptr_t)7);
    const uint64_t* w[N];
    uint32_t sh[N];
    uint64_t k[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
        const uintptr_t a = (uintptr_t)(chars + pos[c]);
        w[c] = need[c] ? (const uint64_t*)(a & ~(uintptr_t)7) : safe;
        sh[c] = need[c] ? (uint32_t)(a & 7) * 8 : 0u;
    }
#pragma unroll
    for (int c = 0; c < N; ++c) k[c] = __builtin_bswap64(*w[c]) << sh[c];
    bool more[N];
#pragma unroll
    for (int c = 0; c < N; ++c)
        more[c] = sh[c] != 0 && (zero_byte_mask(k[c]) & (~0ull << sh[c])) == 0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
        const uint64_t w1 = *(more[c] ? w[c] + 1 : w[c]);
        if (more[c]) k[c] |= __builtin_bswap64(w1) >> (64 - sh[c]);
    }
#pragma unroll
    for (int c = 0; c < N; ++c)
        if (need[c]) out[c] = clip_at_zero(k[c]);
}

#undef S5_HD

}  // namespace s5
