/*
 * Seeded synthetic string sets.  Each generator writes null-terminated strings
 * back to back into one arena and the start of every string into `offsets`.
 * These generators stand in for the paper's real datasets (Section 4 and the
 * appendix on the experimental setup: random strings, URLs, DNA reads and
 * word lists), none of which are used or reproduced here.
 *
 * Pseudo-random numbers come from splitmix64 (Steele, Lea, Flood: "Fast
 * splittable pseudorandom number generators", 2014).  This file holds no part
 * of the sorting method itself; it only makes inputs.
 *
 * kinds:
 *   1 random: length uniform in [8,20], bytes uniform over 'a'..'z'
 *   2 url:    "http://" + host + ".com" + 1..6 segments "/" + 3..12 chars of
 *             [a-z0-9]; 50,000 hosts of 6..20 lowercase letters; the host is
 *             drawn Zipf(s=1.1) by rank
 *   3 dna:    reads of 100 bases over ACGT from an order-3 Markov chain whose
 *             64 rows are Dirichlet(1,1,1,1); first 3 bases uniform; 90% of
 *             the reads generated, 10% exact copies of uniformly chosen
 *             generated reads, then the order is shuffled
 *   4 words:  tokens drawn Zipf(s=1.0) from a 1,000,000-word vocabulary; word
 *             length 1+Poisson(6) (capped at 40); letters i.i.d. with
 *             probability proportional to 1/r over a seeded letter order
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s; } rng_t;

static uint64_t next64(rng_t* r) {
    uint64_t z = (r->s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
/* uniform double in [0,1) */
static double unif(rng_t* r) { return (double)(next64(r) >> 11) * (1.0 / 9007199254740992.0); }
/* uniform integer in [a,b] (multiply-shift, 32-bit range) */
static uint64_t uint_in(rng_t* r, uint64_t a, uint64_t b) {
    uint64_t span = b - a + 1;
    return a + (((next64(r) >> 32) * span) >> 32);
}
static rng_t rng_make(uint64_t seed, uint64_t stream) {
    rng_t r = {seed ^ (0xD1B54A32D192ED03ull * (stream + 1))};
    next64(&r);
    return r;
}

uint64_t s5gen_max_len(int kind) {
    switch (kind) {
        case 1: return 21;                    /* 20 chars + terminator */
        case 2: return 7 + 20 + 4 + 6 * 13 + 1; /* 110 */
        case 3: return 101;
        case 4: return 41;
        default: return 0;
    }
}

/* cumulative Zipf(s) distribution over ranks 1..m */
static double* zipf_cdf(uint64_t m, double s) {
    double* c = (double*)malloc(m * sizeof(double));
    double acc = 0;
    if (!c) return 0;
    for (uint64_t r = 0; r < m; ++r) {
        acc += pow((double)(r + 1), -s);
        c[r] = acc;
    }
    for (uint64_t r = 0; r < m; ++r) c[r] /= acc;
    c[m - 1] = 1.0;
    return c;
}
/* index of the first cdf entry >= u */
static uint64_t draw_cdf(const double* c, uint64_t m, double u) {
    uint64_t lo = 0, hi = m - 1;
    while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        if (c[mid] < u) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static int64_t gen_random(uint64_t n, uint64_t seed, uint8_t* chars, uint64_t cap,
                          uint64_t* off) {
    rng_t r = rng_make(seed, 1);
    uint64_t p = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t len = uint_in(&r, 8, 20);
        if (p + len + 1 > cap) return -1;
        off[i] = p;
        for (uint64_t j = 0; j < len; ++j) chars[p++] = (uint8_t)uint_in(&r, 'a', 'z');
        chars[p++] = 0;
    }
    return (int64_t)p;
}

static const char ALNUM[] = "abcdefghijklmnopqrstuvwxyz0123456789";

static int64_t gen_url(uint64_t n, uint64_t seed, uint8_t* chars, uint64_t cap,
                       uint64_t* off) {
    const uint64_t H = 50000;
    rng_t hr = rng_make(seed, 2), r = rng_make(seed, 3);
    uint8_t* host = (uint8_t*)malloc(H * 21);
    uint8_t* hlen = (uint8_t*)malloc(H);
    double* cdf = zipf_cdf(H, 1.1);
    uint64_t p = 0;
    int64_t ret = 0;
    if (!host || !hlen || !cdf) { ret = -2; goto done; }
    for (uint64_t h = 0; h < H; ++h) {
        hlen[h] = (uint8_t)uint_in(&hr, 6, 20);
        for (uint64_t j = 0; j < hlen[h]; ++j) host[h * 21 + j] = (uint8_t)uint_in(&hr, 'a', 'z');
    }
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t h = draw_cdf(cdf, H, unif(&r));
        if (p + s5gen_max_len(2) > cap) { ret = -1; goto done; }
        off[i] = p;
        memcpy(chars + p, "http://", 7); p += 7;
        memcpy(chars + p, host + h * 21, hlen[h]); p += hlen[h];
        memcpy(chars + p, ".com", 4); p += 4;
        uint64_t k = uint_in(&r, 1, 6);
        for (uint64_t s = 0; s < k; ++s) {
            uint64_t len = uint_in(&r, 3, 12);
            chars[p++] = '/';
            for (uint64_t j = 0; j < len; ++j) chars[p++] = (uint8_t)ALNUM[uint_in(&r, 0, 35)];
        }
        chars[p++] = 0;
    }
    ret = (int64_t)p;
done:
    free(host); free(hlen); free(cdf);
    return ret;
}

static int64_t gen_dna(uint64_t n, uint64_t seed, uint8_t* chars, uint64_t cap,
                       uint64_t* off) {
    static const uint8_t BASE[4] = {'A', 'C', 'G', 'T'};
    const uint64_t L = 100;
    rng_t tr = rng_make(seed, 4), r = rng_make(seed, 5);
    double cum[64][4];
    uint64_t ngen = n - n / 10;
    uint8_t* reads = 0;
    uint64_t* order = 0;
    int64_t ret = 0;
    if (n == 0) return 0;
    if (ngen == 0) ngen = n;
    if (n * (L + 1) > cap) return -1;
    for (int c = 0; c < 64; ++c) {           /* Dirichlet(1,1,1,1) row = normalised Exp(1) draws */
        double e[4], s = 0;
        for (int b = 0; b < 4; ++b) { e[b] = -log(1.0 - unif(&tr)); s += e[b]; }
        double acc = 0;
        for (int b = 0; b < 4; ++b) { acc += e[b] / s; cum[c][b] = acc; }
        cum[c][3] = 1.0;
    }
    reads = (uint8_t*)malloc(ngen * L);
    order = (uint64_t*)malloc(n * sizeof(uint64_t));
    if (!reads || !order) { ret = -2; goto done; }
    for (uint64_t i = 0; i < ngen; ++i) {
        uint8_t* s = reads + i * L;
        for (uint64_t j = 0; j < 3; ++j) s[j] = (uint8_t)uint_in(&r, 0, 3);
        for (uint64_t j = 3; j < L; ++j) {
            int ctx = s[j - 3] * 16 + s[j - 2] * 4 + s[j - 1];
            double u = unif(&r);
            int b = 0;
            while (b < 3 && cum[ctx][b] < u) ++b;
            s[j] = (uint8_t)b;
        }
    }
    /* string ids: 0..ngen-1 generated, ngen..n-1 copies; then Fisher-Yates shuffle */
    for (uint64_t i = 0; i < n; ++i) order[i] = i < ngen ? i : uint_in(&r, 0, ngen - 1);
    for (uint64_t i = n - 1; i > 0; --i) {
        uint64_t j = uint_in(&r, 0, i);
        uint64_t t = order[i]; order[i] = order[j]; order[j] = t;
    }
    for (uint64_t i = 0; i < n; ++i) {
        const uint8_t* s = reads + order[i] * L;
        off[i] = i * (L + 1);
        for (uint64_t j = 0; j < L; ++j) chars[i * (L + 1) + j] = BASE[s[j]];
        chars[i * (L + 1) + L] = 0;
    }
    ret = (int64_t)(n * (L + 1));
done:
    free(reads); free(order);
    return ret;
}

static uint64_t poisson(rng_t* r, double lambda) {
    double lim = exp(-lambda), prod = unif(r);
    uint64_t k = 0;
    while (prod > lim) { ++k; prod *= unif(r); }
    return k;
}

static int64_t gen_words(uint64_t n, uint64_t seed, uint8_t* chars, uint64_t cap,
                         uint64_t* off) {
    const uint64_t V = 1000000, MAXW = 40;
    rng_t vr = rng_make(seed, 6), r = rng_make(seed, 7);
    uint8_t letters[26];
    double lcum[26], acc = 0;
    uint64_t* woff = (uint64_t*)malloc((V + 1) * sizeof(uint64_t));
    uint8_t* vocab = (uint8_t*)malloc(V * MAXW);
    double* cdf = zipf_cdf(V, 1.0);
    uint64_t p = 0, q = 0;
    int64_t ret = 0;
    if (!woff || !vocab || !cdf) { ret = -2; goto done; }
    for (int i = 0; i < 26; ++i) letters[i] = (uint8_t)('a' + i);
    for (int i = 25; i > 0; --i) {
        int j = (int)uint_in(&vr, 0, (uint64_t)i);
        uint8_t t = letters[i]; letters[i] = letters[j]; letters[j] = t;
    }
    for (int i = 0; i < 26; ++i) { acc += 1.0 / (i + 1); lcum[i] = acc; }
    for (int i = 0; i < 26; ++i) lcum[i] /= acc;
    lcum[25] = 1.0;
    for (uint64_t w = 0; w < V; ++w) {
        uint64_t len = 1 + poisson(&vr, 6.0);
        if (len > MAXW) len = MAXW;
        woff[w] = q;
        for (uint64_t j = 0; j < len; ++j) {
            double u = unif(&vr);
            int b = 0;
            while (b < 25 && lcum[b] < u) ++b;
            vocab[q++] = letters[b];
        }
    }
    woff[V] = q;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t w = draw_cdf(cdf, V, unif(&r));
        uint64_t len = woff[w + 1] - woff[w];
        if (p + len + 1 > cap) { ret = -1; goto done; }
        off[i] = p;
        memcpy(chars + p, vocab + woff[w], len);
        p += len;
        chars[p++] = 0;
    }
    ret = (int64_t)p;
done:
    free(woff); free(vocab); free(cdf);
    return ret;
}

/* Generate n strings of `kind`; returns arena bytes used, -1 if `cap` is too
 * small, -2 on allocation failure, -3 for an unknown kind. */
int64_t s5gen_generate(int kind, uint64_t n, uint64_t seed, uint8_t* chars, uint64_t cap,
                       uint64_t* offsets) {
    switch (kind) {
        case 1: return gen_random(n, seed, chars, cap, offsets);
        case 2: return gen_url(n, seed, chars, cap, offsets);
        case 3: return gen_dna(n, seed, chars, cap, offsets);
        case 4: return gen_words(n, seed, chars, cap, offsets);
        default: return -3;
    }
}

/* Plan of a batched workload: for every set its size, log-uniform in
 * [min_size, max_size], and its generator kind, uniform over `kinds`. */
void s5gen_batched_plan(uint32_t num_sets, uint64_t seed, uint64_t min_size,
                        uint64_t max_size, const int* kinds, int num_kinds,
                        uint64_t* set_size, int* set_kind) {
    rng_t r = rng_make(seed, 8);
    double a = log((double)min_size), b = log((double)max_size);
    for (uint32_t s = 0; s < num_sets; ++s) {
        uint64_t sz = (uint64_t)floor(exp(a + (b - a) * unif(&r)));
        if (sz < min_size) sz = min_size;
        if (sz > max_size) sz = max_size;
        set_size[s] = sz;
        set_kind[s] = kinds[uint_in(&r, 0, (uint64_t)num_kinds - 1)];
    }
}

/* Generate every set of a plan into one arena.  Set s uses seed ^ (s+1)
 * mixed through splitmix64; its strings follow those of set s-1.  Offsets
 * are global (into the one arena).  Sets are generated in parallel when the
 * library is built with OpenMP.  Returns arena bytes used or a negative code
 * as s5gen_generate. */
int64_t s5gen_batched(uint32_t num_sets, uint64_t seed, const uint64_t* set_size,
                      const int* set_kind, uint8_t* chars, uint64_t cap,
                      uint64_t* offsets) {
    uint64_t* region = (uint64_t*)malloc((num_sets + 1) * sizeof(uint64_t));
    uint64_t* first = (uint64_t*)malloc((num_sets + 1) * sizeof(uint64_t));
    int64_t* used = (int64_t*)malloc((num_sets + 1) * sizeof(int64_t));
    int64_t ret = 0;
    if (!region || !first || !used) { ret = -2; goto done; }
    region[0] = 0;
    first[0] = 0;
    for (uint32_t s = 0; s < num_sets; ++s) {
        region[s + 1] = region[s] + set_size[s] * s5gen_max_len(set_kind[s]);
        first[s + 1] = first[s] + set_size[s];
    }
    if (region[num_sets] > cap) { ret = -1; goto done; }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < (int64_t)num_sets; ++s) {
        rng_t m = {seed ^ ((uint64_t)s + 1)};
        uint64_t sseed = next64(&m);
        used[s] = s5gen_generate(set_kind[s], set_size[s], sseed, chars + region[s],
                                 set_size[s] * s5gen_max_len(set_kind[s]), offsets + first[s]);
    }
    /* compact the regions and rebase offsets, in order */
    {
        uint64_t p = 0;
        for (uint32_t s = 0; s < num_sets; ++s) {
            if (used[s] < 0) { ret = used[s]; goto done; }
            if (p != region[s]) memmove(chars + p, chars + region[s], (size_t)used[s]);
            for (uint64_t i = first[s]; i < first[s + 1]; ++i) offsets[i] += p;
            p += (uint64_t)used[s];
        }
        ret = (int64_t)p;
    }
done:
    free(region); free(first); free(used);
    return ret;
}
