// CPU checks of the library's word-level helpers (s5_word.h), compiled for the
// host.  Every check compares a helper with a plain byte-level definition.
// Usage: word_helpers_test <fig1 golden file>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/mman.h>
#include <unistd.h>

#include <algorithm>
#include <random>
#include <string>
#include <vector>

#include "s5_word.h"

using namespace s5;

static int failures = 0;
#define CHECK(cond, ...)                                \
    do {                                                \
        if (!(cond)) {                                  \
            if (failures < 20) {                        \
                printf("FAIL %s:%d: ", __FILE__, __LINE__); \
                printf(__VA_ARGS__);                    \
                printf("\n");                           \
            }                                           \
            ++failures;                                 \
        }                                               \
    } while (0)

// byte-level definition of the key of s at depth
static uint64_t ref_key(const uint8_t* s) {
    uint64_t k = 0;
    bool ended = false;
    for (int i = 0; i < 8; ++i) {
        uint8_t c = ended ? 0 : s[i];
        if (c == 0) ended = true;
        k = (k << 8) | c;
    }
    return k;
}
static uint32_t ref_lcp(const uint8_t* a, const uint8_t* b) {
    uint32_t k = 0;
    while (k < 8 && a[k] == b[k] && a[k] != 0) ++k;
    return k;
}

static void test_load_key_guarded(std::mt19937_64& rng) {
    // strings that end right before an inaccessible page: any read past the
    // string's last aligned word would fault
    long pg = sysconf(_SC_PAGESIZE);
    uint8_t* mem = (uint8_t*)mmap(nullptr, 2 * pg, PROT_READ | PROT_WRITE,
                                  MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
    CHECK(mem != MAP_FAILED, "mmap");
    mprotect(mem + pg, pg, PROT_NONE);
    for (int len = 0; len <= 40; ++len) {
        uint8_t* s = mem + pg - (len + 1);
        for (int i = 0; i < len; ++i) s[i] = (uint8_t)(1 + rng() % 255);
        s[len] = 0;
        for (int dep = 0; dep <= len; ++dep) {
            uint64_t got = load_key(mem, (uint64_t)(s - mem) + dep);
            uint8_t tmp[8];
            for (int i = 0; i < 8; ++i) tmp[i] = dep + i <= len ? s[dep + i] : 0;
            CHECK(got == ref_key(tmp), "guarded len %d depth %d", len, dep);
            // batched form: mixed need flags, untouched outputs where not needed
            uint64_t pos[4], out[4] = {1, 2, 3, 4};
            bool need[4] = {true, false, true, false};
            for (int c = 0; c < 4; ++c) pos[c] = (uint64_t)(s - mem) + dep;
            load_keys<4>(mem, pos, need, out);
            CHECK(out[0] == ref_key(tmp) && out[2] == ref_key(tmp) && out[1] == 2 && out[3] == 4,
                  "load_keys len %d depth %d", len, dep);
            // two words at once: the second is the key 8 bytes deeper
            uint64_t k0 = 0, k1 = 0;
            load_key16(mem, (uint64_t)(s - mem) + dep, &k0, &k1);
            uint8_t tmp2[8];
            for (int i = 0; i < 8; ++i) tmp2[i] = dep + 8 + i <= len ? s[dep + 8 + i] : 0;
            CHECK(k0 == ref_key(tmp) && k1 == ref_key(tmp2), "load_key16 len %d depth %d", len,
                  dep);
            // four keys in a run
            uint64_t run[4];
            load_key_run<4>(mem, (uint64_t)(s - mem) + dep, run);
            for (int j = 0; j < 4; ++j) {
                uint8_t t[8];
                for (int i = 0; i < 8; ++i) t[i] = dep + 8 * j + i <= len ? s[dep + 8 * j + i] : 0;
                CHECK(run[j] == ref_key(t), "load_key_run len %d depth %d word %d", len, dep, j);
            }
        }
    }
    munmap(mem, 2 * pg);
}

// Walk strings deeper by random steps of 1..8 bytes keeping (k0, k1) as the
// redistribution does: advance from what is known, gather when it is not;
// both words must always equal the keys at the current depth (k1 may also be
// unknown).  Strings of 0xFF bytes check that a real all-0xFF word is harmless.
static void test_advance_key16(std::mt19937_64& rng) {
    std::vector<uint8_t> s(80);
    int gathers = 0, steps = 0;
    for (int t = 0; t < 4000; ++t) {
        const int len = (int)(rng() % 70);
        const bool ff = t % 7 == 0;
        for (int i = 0; i < len; ++i) s[i] = ff ? 0xFF : (uint8_t)(1 + rng() % 255);
        for (int i = len; i < 80; ++i) s[i] = 0;
        int dep = 0;
        uint64_t k0, k1;
        load_key16(s.data(), 0, &k0, &k1);
        while (dep < len) {
            const uint32_t delta = 1 + (uint32_t)(rng() % 8);
            if (dep + (int)delta > len) break;
            dep += (int)delta;
            ++steps;
            if (!advance_key16(&k0, &k1, delta)) {
                load_key16(s.data(), (uint64_t)dep, &k0, &k1);
                ++gathers;
            }
            CHECK(k0 == ref_key(&s[dep]), "advance k0 len %d depth %d", len, dep);
            CHECK(k1 == kKeyUnknown || k1 == ref_key(&s[dep + 8]), "advance k1 len %d depth %d",
                  len, dep);
        }
        // past the terminator everything is known to be zero
        if (len < 8) {
            uint64_t a = ref_key(&s[0]), b = ref_key(&s[8]);
            CHECK(advance_key16(&a, &b, 3) && a == ref_key(&s[3]) && b == 0, "ended len %d", len);
        }
    }
    CHECK(gathers < steps, "some steps need no gather (%d of %d)", gathers, steps);
    // three known words: both advanced words exact, for every step 1..8
    for (int t = 0; t < 2000; ++t) {
        const int len = (int)(rng() % 40);
        for (int i = 0; i < len; ++i) s[i] = (uint8_t)(1 + rng() % 255);
        for (int i = len; i < 80; ++i) s[i] = 0;
        uint64_t w[3];
        load_key_run<3>(s.data(), 0, w);
        for (uint32_t delta = 1; delta <= 8; ++delta) {
            uint64_t a0 = w[0], a1 = w[1];
            advance_key24(&a0, &a1, w[2], delta);
            CHECK(a0 == ref_key(&s[delta]) && a1 == ref_key(&s[delta + 8]),
                  "advance_key24 len %d delta %u", len, delta);
        }
    }
}

static void test_load_key_random(std::mt19937_64& rng) {
    std::vector<uint8_t> arena(1 << 16, 0);
    size_t p = 3;  // deliberately unaligned start
    std::vector<std::pair<size_t, int>> strs;
    while (p + 40 < arena.size()) {
        int len = rng() % 30;
        for (int i = 0; i < len; ++i) {
            uint8_t c = (rng() % 4 == 0) ? (uint8_t)(0x80 + rng() % 128) : (uint8_t)(1 + rng() % 127);
            arena[p + i] = c;
        }
        arena[p + len] = 0;
        strs.push_back({p, len});
        p += len + 1;
    }
    for (auto& sl : strs)
        for (int dep = 0; dep <= sl.second; ++dep) {
            const uint8_t* s = arena.data() + sl.first + dep;
            uint64_t got = load_key(arena.data(), sl.first + dep);
            CHECK(got == ref_key(s), "random key at %zu depth %d", sl.first, dep);
            uint64_t run[4];
            load_key_run<4>(arena.data(), sl.first + dep, run);
            for (int j = 0; j < 4; ++j) {
                const uint64_t want = dep + 8 * j <= sl.second ? ref_key(s + 8 * j) : 0ull;
                CHECK(run[j] == want, "random run at %zu depth %d word %d", sl.first, dep, j);
            }
        }
    // lcp8 and nz_bytes against byte loops
    for (size_t t = 1; t < strs.size(); ++t) {
        const uint8_t* a = arena.data() + strs[t - 1].first;
        const uint8_t* b = arena.data() + strs[t].first;
        CHECK(lcp8(ref_key(a), ref_key(b)) == ref_lcp(a, b), "lcp8 %zu", t);
        CHECK(lcp8(ref_key(a), ref_key(a)) == ref_lcp(a, a), "lcp8 self %zu", t);
        CHECK(nz_bytes(ref_key(a)) == std::min<uint32_t>(8, (uint32_t)strlen((const char*)a)),
              "nz %zu", t);
    }
    // key order equals byte order (memcmp on the zero-padded 8 bytes)
    for (int t = 0; t < 20000; ++t) {
        uint8_t a[8], b[8];
        for (int i = 0; i < 8; ++i) {
            a[i] = (uint8_t)(rng() % 3 == 0 ? 0 : rng());
            b[i] = (uint8_t)(rng() % 3 == 0 ? 0 : rng());
        }
        for (int i = 0; i < 8; ++i) if (a[i] == 0) for (int j = i; j < 8; ++j) a[j] = 0;
        for (int i = 0; i < 8; ++i) if (b[i] == 0) for (int j = i; j < 8; ++j) b[j] = 0;
        int c = memcmp(a, b, 8);
        uint64_t ka = ref_key(a), kb = ref_key(b);
        CHECK((c < 0) == (ka < kb) && (c == 0) == (ka == kb), "order");
        CHECK(clip_at_zero(ka) == ka, "clip idempotent");
    }
}

// in-order traversal of a perfect tree with heap indices 1..2^d-1
static void inorder(uint32_t i, uint32_t v, std::vector<uint32_t>& out) {
    if (i > v) return;
    inorder(2 * i, v, out);
    out.push_back(i);
    inorder(2 * i + 1, v, out);
}

static void test_inorder_map() {
    for (uint32_t d = 1; d <= 10; ++d) {
        uint32_t v = (1u << d) - 1;
        std::vector<uint32_t> ord;
        inorder(1, v, ord);
        for (uint32_t j = 0; j < v; ++j) CHECK(inorder_node(j, d) == ord[j], "d %u j %u", d, j);
    }
}

// Build a tree from a sorted sample exactly as the device does, level by level.
static void build_tree(const std::vector<uint64_t>& smp, uint32_t d, std::vector<uint64_t>& t,
                       std::vector<uint64_t>& tin) {
    uint32_t v = (1u << d) - 1;
    t.assign(v + 1, 0);
    std::vector<uint32_t> ra(v + 1), rb(v + 1);
    ra[1] = 0;
    rb[1] = (uint32_t)smp.size();
    for (uint32_t L = 0; L < d; ++L)
        for (uint32_t i = 1u << L; i < (2u << L); ++i) {
            uint32_t a = ra[i], b = rb[i], lo = 0, hi = 0;
            uint64_t x;
            if (a < b) select_node(smp.data(), a, b, &x, &lo, &hi);
            else x = t[i >> 1];
            t[i] = x;
            if (L + 1 < d) {
                ra[2 * i] = a < b ? a : 0; rb[2 * i] = a < b ? lo : 0;
                ra[2 * i + 1] = a < b ? hi : 0; rb[2 * i + 1] = a < b ? b : 0;
            }
        }
    tin.assign(v + 1, 0);
    for (uint32_t j = 0; j < v; ++j) tin[j] = t[inorder_node(j, d)];
}

// select_node against its definition by linear scans: the middle sample of
// [a, b) and the run [lo, hi) of samples equal to it, clipped to [a, b).
static void test_select_node(std::mt19937_64& rng) {
    for (int rep = 0; rep < 400; ++rep) {
        const uint32_t n = 1 + (uint32_t)(rng() % 600);
        const uint32_t distinct = 1 + (uint32_t)(rng() % (rep % 3 == 0 ? 4 : 2 * n));
        std::vector<uint64_t> smp(n);
        for (auto& x : smp) x = (rng() % distinct) * 0x0100000001ull;
        std::sort(smp.begin(), smp.end());
        for (int q = 0; q < 40; ++q) {
            uint32_t a = (uint32_t)(rng() % n), b = (uint32_t)(rng() % n);
            if (a > b) std::swap(a, b);
            ++b;
            uint64_t x;
            uint32_t lo, hi;
            select_node(smp.data(), a, b, &x, &lo, &hi);
            const uint32_t mid = (a + b) / 2;
            uint32_t rlo = mid, rhi = mid + 1;
            while (rlo > a && smp[rlo - 1] == smp[mid]) --rlo;
            while (rhi < b && smp[rhi] == smp[mid]) ++rhi;
            CHECK(x == smp[mid] && lo == rlo && hi == rhi, "n %u [%u, %u): %u %u vs %u %u", n, a,
                  b, lo, hi, rlo, rhi);
        }
    }
}

static void test_tree_and_classify(std::mt19937_64& rng) {
    for (int rep = 0; rep < 300; ++rep) {
        uint32_t d = 1 + rng() % 10, v = (1u << d) - 1;
        uint32_t m = 1 + rng() % (4 * (v + 1));
        uint32_t distinct = 1 + rng() % (2 * m);
        std::vector<uint64_t> pool(distinct);
        for (auto& x : pool) x = rng() >> (rng() % 64);
        std::vector<uint64_t> smp(m);
        for (auto& x : smp) x = pool[rng() % distinct];
        std::sort(smp.begin(), smp.end());
        std::vector<uint64_t> t, tin;
        build_tree(smp, d, t, tin);
        for (uint32_t j = 1; j < v; ++j) CHECK(tin[j - 1] <= tin[j], "in-order sorted d %u", d);
        for (int probe = 0; probe < 200; ++probe) {
            uint64_t key[4];
            for (auto& k : key) k = (rng() % 2) ? pool[rng() % distinct] + (rng() % 3) - 1 : rng();
            uint32_t b[4];
            classify_u<4>(t.data(), tin.data(), d, v, key, b);
            for (int q = 0; q < 4; ++q) {
                uint32_t j = (uint32_t)(std::lower_bound(tin.begin(), tin.begin() + v, key[q]) -
                                        tin.begin());
                uint32_t want = 2 * j + (j < v && tin[j] == key[q]);
                CHECK(b[q] == want, "classify d %u key %llx got %u want %u", d,
                      (unsigned long long)key[q], b[q], want);
            }
        }
    }
}

// the Equal descent run to the end on the host (no early exit: a finished
// descent keeps its node and its bucket)
static uint32_t equal_classify(const std::vector<uint64_t>& t, uint32_t d, uint64_t key) {
    uint32_t i = 1, b = 0;
    bool done = false;
    for (uint32_t L = 0; L < d; ++L) equal_step(t.data(), d, key, i, done, b);
    return done ? b : equal_leaf_bucket(i, d);
}

static void test_node_inorder() {
    for (uint32_t d = 1; d <= 10; ++d)
        for (uint32_t j = 0; j < (1u << d) - 1; ++j)
            CHECK(node_inorder(inorder_node(j, d), d) == j, "node_inorder d %u j %u", d, j);
}

static void test_equal_variant(std::mt19937_64& rng) {
    for (int rep = 0; rep < 300; ++rep) {
        uint32_t d = 1 + rng() % 10, v = (1u << d) - 1;
        uint32_t m = 1 + rng() % (4 * (v + 1));
        uint32_t distinct = 1 + rng() % (2 * m);
        std::vector<uint64_t> pool(distinct);
        for (auto& x : pool) x = rng() >> (rng() % 64);
        std::vector<uint64_t> smp(m);
        for (auto& x : smp) x = pool[rng() % distinct];
        std::sort(smp.begin(), smp.end());
        std::vector<uint64_t> t, tin;
        build_tree(smp, d, t, tin);
        const bool unique = std::adjacent_find(tin.begin(), tin.begin() + v) == tin.begin() + v;
        for (int probe = 0; probe < 200; ++probe) {
            const uint64_t key = (rng() % 2) ? pool[rng() % distinct] + (rng() % 3) - 1 : rng();
            const uint32_t b = equal_classify(t, d, key);
            const uint32_t j = (uint32_t)(std::lower_bound(tin.begin(), tin.begin() + v, key) -
                                          tin.begin());
            const bool eq = j < v && tin[j] == key;
            if (unique) {  // distinct splitters: exactly 2 lower_bound + [equal]
                CHECK(b == 2 * j + (eq ? 1u : 0u), "equal d %u got %u want %u", d, b, 2 * j + eq);
            } else if (eq) {  // an equality bucket of a splitter equal to the key
                CHECK((b & 1u) && b / 2 < v && tin[b / 2] == key, "equal dup d %u b %u", d, b);
            } else {  // the range bucket between the neighbouring splitters
                CHECK(b == 2 * j, "equal range d %u got %u want %u", d, b, 2 * j);
            }
        }
    }
}

// the Jump variant on the host: table, start node, descent, leaf test
static uint32_t jump_classify(const std::vector<uint64_t>& t, const std::vector<uint64_t>& tin,
                              const std::vector<uint16_t>& jt, uint32_t d, uint32_t v,
                              uint64_t key) {
    const uint64_t first = tin[0], last = tin[v - 1];
    const JumpShape js = jump_shape(first, last, d);
    uint32_t i = key < first ? (1u << d) : (key > last ? (1u << d) + v : jt[jump_index(key, js)]);
    while (i < (1u << d)) i = 2 * i + (key > t[i] ? 1u : 0u);
    const uint32_t j = i - (1u << d);
    return 2 * j + ((j < v && tin[j] == key) ? 1u : 0u);
}

static void test_jump_table(std::mt19937_64& rng) {
    for (int rep = 0; rep < 400; ++rep) {
        uint32_t d = 1 + rng() % 10, v = (1u << d) - 1;
        uint32_t m = 1 + rng() % (4 * (v + 1));
        uint32_t distinct = 1 + rng() % (2 * m);
        // pools near one value (long common prefixes) or spread over all 64 bits
        const uint64_t base = rng(), spread = rng() % 3 == 0 ? (1ull << (rng() % 40)) : ~0ull;
        std::vector<uint64_t> pool(distinct);
        for (auto& x : pool) x = spread == ~0ull ? rng() >> (rng() % 64) : base + rng() % spread;
        std::vector<uint64_t> smp(m);
        for (auto& x : smp) x = pool[rng() % distinct];
        std::sort(smp.begin(), smp.end());
        std::vector<uint64_t> t, tin;
        build_tree(smp, d, t, tin);
        const JumpShape js = jump_shape(tin[0], tin[v - 1], d);
        CHECK(js.a <= 12 && js.a <= d + 2 && js.sh + js.a <= 64, "jump shape d %u", d);
        std::vector<uint16_t> jt(1u << js.a);
        build_jump_table(t.data(), d, v, jt.data(), 0, 1);
        for (uint32_t p = 0; p < jt.size(); ++p) CHECK(jt[p] >= 1 && jt[p] < (2u << d), "entry");
        for (int probe = 0; probe < 300; ++probe) {
            uint64_t key;
            switch (rng() % 4) {
                case 0: key = pool[rng() % distinct]; break;
                case 1: key = pool[rng() % distinct] + (rng() % 5) - 2; break;
                case 2: key = tin[rng() % v] + (rng() % 3) - 1; break;
                default: key = rng(); break;
            }
            uint64_t kk[1] = {key};
            uint32_t want[1];
            classify_u<1>(t.data(), tin.data(), d, v, kk, want);
            const uint32_t got = jump_classify(t, tin, jt, d, v, key);
            CHECK(got == want[0], "jump d %u key %llx got %u want %u", d, (unsigned long long)key,
                  got, want[0]);
        }
    }
}

// ---- alphabet compression --------------------------------------------------
// reference: the codes of the characters of s from depth on (0 from the
// terminator on), one per character
static std::vector<uint32_t> ref_codes(const uint8_t* s, const uint8_t* table, int count) {
    std::vector<uint32_t> c(count, 0);
    bool ended = false;
    for (int i = 0; i < count; ++i) {
        if (!ended && s[i] == 0) ended = true;
        c[i] = ended ? 0 : table[s[i]];
    }
    return c;
}
static uint64_t ref_pack(const std::vector<uint32_t>& codes, int first) {
    uint64_t k = 0;
    for (int f = 0; f < 21; ++f) k |= (uint64_t)(codes[first + f] & 7) << (61 - 3 * f);
    return k;
}

static void test_codec(std::mt19937_64& rng) {
    // b = 8 is the byte codec exactly
    const KeyCodec b8 = make_codec(8, nullptr, nullptr);
    CHECK(b8.w == 8 && b8.hi == 0x8080808080808080ull && b8.lo == 0x7F7F7F7F7F7F7F7Full, "b8");
    for (int rep = 0; rep < 20000; ++rep) {
        uint64_t x = rng(), y = rng();
        if (rng() % 3 == 0) x &= ~(0xFFull << (8 * (rng() % 8)));
        if (rng() % 3 == 0) y = x ^ (1ull << (rng() % 64));
        x = clip_at_zero(x);
        y = clip_at_zero(y);
        CHECK(codec_has_end(b8, x) == has_zero(x), "b8 has_end");
        CHECK(codec_before_end(b8, x) == nz_bytes(x), "b8 before_end");
        CHECK(codec_lcp(b8, x, y) == lcp8(x, y), "b8 lcp");
        const uint32_t d = 1 + rng() % 8;
        uint64_t a0 = x, a1 = y, c0 = x, c1 = y;
        const bool ra = advance_key16(&a0, &a1, d), rc = codec_advance2(b8, &c0, &c1, d);
        CHECK(ra == rc && (!ra || (a0 == c0 && a1 == c1)), "b8 advance2");
    }
    for (uint32_t b = 3; b <= 8; ++b) {
        const KeyCodec c = make_codec(b, nullptr, nullptr);
        for (uint32_t q = 0; q <= 64; ++q) CHECK(codec_div(c, q) == q / b, "div b %u q %u", b, q);
    }
    // 3-bit codes against the reference: pack3, end test, lcp, advances
    const KeyCodec c3 = make_codec(3, nullptr, nullptr);
    CHECK(c3.w == 21 && kPackChars == 21, "w");
    uint8_t table[256];
    for (int rep = 0; rep < 3000; ++rep) {
        const int sigma = 1 + (int)(rng() % 7);
        std::vector<uint8_t> alpha;
        while ((int)alpha.size() < sigma) {
            const uint8_t ch = (uint8_t)(1 + rng() % 255);
            if (std::find(alpha.begin(), alpha.end(), ch) == alpha.end()) alpha.push_back(ch);
        }
        std::sort(alpha.begin(), alpha.end());
        for (int ch = 0; ch < 256; ++ch) table[ch] = 0xFF;
        table[0] = 0;
        for (int i = 0; i < sigma; ++i) table[alpha[i]] = (uint8_t)(i + 1);
        // two strings sharing a random prefix, lengths up to 80
        const int la = (int)(rng() % 80), lb = (int)(rng() % 80), common = (int)(rng() % 80);
        uint8_t sa[160] = {0}, sb[160] = {0};
        for (int i = 0; i < la; ++i) sa[i] = alpha[rng() % sigma];
        for (int i = 0; i < lb; ++i) sb[i] = i < common && i < la ? sa[i] : alpha[rng() % sigma];
        const bool plant = rng() % 10 == 0;  // a byte outside the alphabet
        if (plant && la > 0) sa[rng() % la] = 0xFF == table[1] ? 1 : (uint8_t)1;
        const bool bad_expected = plant && la > 0 && table[1] == 0xFF;
        uint64_t rawa[8], rawb[8];
        load_key_run<8>(sa, 0, rawa);
        load_key_run<8>(sb, 0, rawb);
        uint64_t ka[3], kb[3];
        const bool bad = pack3<8, 3>(table, rawa, ka);
        pack3<8, 3>(table, rawb, kb);
        const auto ca = ref_codes(sa, table, 64), cb = ref_codes(sb, table, 64);
        bool planted_in_range = false;
        for (int i = 0; i < 63 && i < la; ++i) planted_in_range |= table[sa[i]] == 0xFF;
        CHECK(bad == planted_in_range, "pack3 bad flag %d %d", bad, planted_in_range);
        if (bad_expected) continue;
        for (int k = 0; k < 3; ++k) {
            CHECK(ka[k] == ref_pack(ca, 21 * k), "pack3 key %d", k);
            // order of packed keys = order of the code sequences
            const auto ea = std::vector<uint32_t>(ca.begin() + 21 * k, ca.begin() + 21 * k + 21);
            const auto eb = std::vector<uint32_t>(cb.begin() + 21 * k, cb.begin() + 21 * k + 21);
            CHECK((ka[k] < kb[k]) == (ea < eb), "packed order");
            int end = 0;
            while (end < 21 && ea[end]) ++end;
            CHECK(codec_has_end(c3, ka[k]) == (end < 21), "has_end");
            CHECK(codec_before_end(c3, ka[k]) == (uint32_t)end, "before_end");
            int l = 0;
            while (l < 21 && ea[l] == eb[l] && ea[l]) ++l;
            CHECK(codec_lcp(c3, ka[k], kb[k]) == (uint32_t)l, "lcp %d", l);
        }
        // advancing by delta characters equals packing at depth delta
        const uint32_t d = 1 + rng() % 21;
        uint64_t s0 = ka[0], s1 = ka[1], t0 = ka[0], t1 = ka[1];
        codec_advance3(c3, &s0, &s1, ka[2], d);
        const bool known = codec_advance2(c3, &t0, &t1, d);
        const uint64_t want0 = ref_pack(ca, (int)d), want1 = d + 42 <= 64 ? ref_pack(ca, (int)d + 21) : 0;
        CHECK(s0 == want0 && (d + 42 > 64 || s1 == want1), "advance3 d %u", d);
        CHECK(known && t0 == want0, "advance2 d %u", d);
        CHECK(t1 == (codec_has_end(c3, ka[1]) ? (d < 21 ? ka[1] << (3 * d) : 0ull) : kKeyUnknown),
              "advance2 second word");
    }
}

static void test_fig1(const char* path) {
    FILE* f = fopen(path, "r");
    CHECK(f != nullptr, "open %s", path);
    if (!f) return;
    char line[256];
    std::vector<uint64_t> spl, lvl;
    std::vector<std::pair<uint64_t, uint32_t>> probes;
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        char tag[32];
        if (sscanf(line, "%31s", tag) != 1) continue;
        const char* p = line + strlen(tag);
        if (!strcmp(tag, "splitters") || !strcmp(tag, "level_order")) {
            unsigned long long x;
            int used;
            while (sscanf(p, " %llx%n", &x, &used) == 1) {
                (!strcmp(tag, "splitters") ? spl : lvl).push_back(x);
                p += used;
            }
        } else if (!strcmp(tag, "probe")) {
            unsigned long long x;
            unsigned b;
            if (sscanf(p, " %llx %u", &x, &b) == 2) probes.push_back({x, b});
        }
    }
    fclose(f);
    CHECK(spl.size() == 3 && lvl.size() == 3 && probes.size() >= 7, "fixture shape");
    if (spl.size() != 3 || lvl.size() != 3) return;
    std::vector<uint64_t> t, tin;
    build_tree(spl, 2, t, tin);
    for (int i = 0; i < 3; ++i) CHECK(t[i + 1] == lvl[i], "fig1 level order %d", i);
    for (auto& pr : probes) {
        uint64_t key[1] = {pr.first};
        uint32_t b[1];
        classify_u<1>(t.data(), tin.data(), 2, 3, key, b);
        CHECK(b[0] == pr.second, "fig1 probe %llx got %u want %u", (unsigned long long)pr.first,
              b[0], pr.second);
        CHECK(equal_classify(t, 2, pr.first) == pr.second, "fig1 equal probe %llx",
              (unsigned long long)pr.first);
    }
}

// Two digits of the bucket ids: every id is its digits put back together,
// both digits stay below their value counts (at most 64), and a stable sort by
// the low digit and then the high digit (the two moves) orders ids exactly as
// a stable sort by the id does.
static void test_bucket_digits(std::mt19937_64& rng) {
    for (uint32_t d = 1; d <= 10; ++d) {
        const uint32_t k = (2u << d) - 1u, r = digit_low_bits(d);
        const uint32_t nlo = digit_values(k, d, kDigitLow), nhi = digit_values(k, d, kDigitHigh);
        CHECK(digit_values(k, d, 0) == k && nlo <= 64 && nhi <= 64 && nlo * nhi >= k, "d %u", d);
        CHECK(nlo <= (1u << digit_bits(d, kDigitLow)) && nhi <= (1u << digit_bits(d, kDigitHigh)) &&
                  digit_bits(d, 0) == d + 1,
              "bits d %u", d);
        for (uint32_t b = 0; b < k; ++b) {
            const uint32_t lo = digit_of(b, d, kDigitLow), hi = digit_of(b, d, kDigitHigh);
            CHECK(lo < nlo && hi < nhi && ((hi << r) | lo) == b && digit_of(b, d, 0) == b,
                  "d %u b %u", d, b);
        }
        std::vector<std::pair<uint32_t, uint32_t>> ids(3000);  // (bucket, input position)
        for (uint32_t i = 0; i < ids.size(); ++i) ids[i] = {(uint32_t)(rng() % k), i};
        std::vector<std::pair<uint32_t, uint32_t>> two = ids, one = ids;
        for (uint32_t dig : {kDigitLow, kDigitHigh})
            std::stable_sort(two.begin(), two.end(), [&](const auto& a, const auto& b) {
                return digit_of(a.first, d, dig) < digit_of(b.first, d, dig);
            });
        std::stable_sort(one.begin(), one.end(),
                         [](const auto& a, const auto& b) { return a.first < b.first; });
        CHECK(two == one, "two moves d %u", d);
    }
}

// xcd_unit renumbers a launch's workgroups: a bijection of [0, n); inside
// every full group of 8 runs, workgroups b and b + 8 (same XCD) take
// neighbouring units, and the 8 XCDs take the group's 8 runs.
static void test_xcd_unit() {
    const uint32_t S = kXcds * kXcdRun;
    for (uint32_t n : {0u, 1u, 7u, 8u, 9u, S - 1, S, S + 1, 3 * S + 5, 4883u, 65536u, 100003u}) {
        std::vector<uint32_t> seen(n, 0);
        bool ok = true;
        for (uint32_t b = 0; b < n; ++b) {
            const uint32_t u = xcd_unit(b, n);
            if (u >= n || seen[u]++) ok = false;
        }
        CHECK(ok, "xcd_unit not a bijection of [0, %u)", n);
        for (uint32_t b = 0; b + kXcds < n / S * S; ++b)
            if ((b + kXcds) / S == b / S)
                CHECK(xcd_unit(b + kXcds, n) == xcd_unit(b, n) + 1, "n %u b %u", n, b);
        for (uint32_t g = 0; g + S <= n; g += S)
            for (uint32_t x = 0; x < kXcds; ++x)
                CHECK(xcd_unit(g + x, n) == g + x * kXcdRun, "n %u run %u", n, x);
    }
}

int main(int argc, char** argv) {
    std::mt19937_64 rng(12345);
    test_load_key_guarded(rng);
    test_load_key_random(rng);
    test_advance_key16(rng);
    test_inorder_map();
    test_select_node(rng);
    test_tree_and_classify(rng);
    test_node_inorder();
    test_equal_variant(rng);
    test_jump_table(rng);
    test_codec(rng);
    test_bucket_digits(rng);
    test_xcd_unit();
    if (argc > 1) test_fig1(argv[1]);
    if (failures) {
        printf("%d failures\n", failures);
        return 1;
    }
    printf("OK\n");
    return 0;
}
