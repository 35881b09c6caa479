// Learned splitter proposal for S^5 (gfx950, FP32, no MFMA).
//
// The paper proposes adapting the algorithm to the input by inspecting the
// sample and measures what a set of splitters gains by the entropy of the
// bucket sizes (appendix A, "Adaptivity").  Here a small network models the
// distribution function of a segment's 8-byte keys and its quantiles become
// the splitters.  Classification is still the exact key comparison of
// Section 3.1, so the sort's output never depends on the model.  A proposal
// is rejected, and the segment gets sampled splitters, if a range bucket holds
// more than beta times its ideal share: first counted on the training sample
// itself (before any classification), then on the exact bucket histogram.
//
// Model: one feature per key byte (most significant first), scaled by the
// range that byte takes over the sample, (c - lo) / max(hi - lo, 1); two
// hidden layers of 32 ReLU units; sigmoid output.  1377 parameters:
// W1 (32x8), b1, W2 (32x32), b2, w3 (32), b3.  Weights start from splitmix64
// used as a counter-based generator; training is full-batch mean squared
// error against the sample's empirical CDF, optimised with Adam.  One step is
// one launch: 256-sample workgroups compute partial gradients in parallel;
// every workgroup of the next step sums the previous partials in the same
// fixed order and applies the identical Adam update, so the result is
// deterministic.
#include "s5_internal.h"
#include "s5_launch.h"
#include "s5_word.h"

namespace s5 {

constexpr uint32_t kGrp = kLearnGrp;  // samples per training workgroup (one per thread)
constexpr int kH = 32;                // hidden units per layer
constexpr uint32_t kNP = 1377;        // parameters
constexpr uint32_t kNPS = 1408;       // stride of one parameter vector
constexpr uint32_t oW1 = 0, oB1 = 256, oW2 = 288, oB2 = 1312, oW3 = 1344, oB3 = 1376;
constexpr float kB1 = 0.9f, kB2 = 0.999f, kEps = 1e-8f;
constexpr uint32_t kS = kH + 1;       // LDS row stride of per-sample vectors
constexpr uint32_t kS1 = kH + 8;      // first hidden layer and features, 16-byte aligned rows

__device__ __forceinline__ float* wbuf(const LearnCtx& c, uint32_t slot, uint32_t b) {
    return c.W + ((size_t)slot * 2 + b) * kNPS;
}
__device__ __forceinline__ float* m1buf(const LearnCtx& c, uint32_t slot, uint32_t b) {
    return c.M1 + ((size_t)slot * 2 + b) * kNPS;
}
__device__ __forceinline__ float* m2buf(const LearnCtx& c, uint32_t slot, uint32_t b) {
    return c.M2 + ((size_t)slot * 2 + b) * kNPS;
}
__device__ __forceinline__ float* pbuf(const LearnCtx& c, uint32_t slot, uint32_t b,
                                       uint32_t grp) {
    return c.part + (((size_t)slot * 2 + b) * c.groups + grp) * kNPS;
}

__device__ __forceinline__ float init_weight(uint64_t seed, uint32_t i) {
    float a;
    if (i < oB1) a = 0.8660254037844386f;             // sqrt(6 / 8)
    else if (i >= oW2 && i < oB2) a = 0.4330127018922193f;  // sqrt(6 / 32)
    else if (i >= oW3 && i < oB3) a = 0.04330127018922193f; // 0.1 * sqrt(6 / 32)
    else return 0.0f;
    const uint64_t r = mix64(seed + i + 1 + 0x9E3779B97F4A7C15ull);  // splitmix64(seed + i + 1)
    const float u = (float)(uint32_t)(r >> 40) * (1.0f / 16777216.0f);
    return (2.0f * u - 1.0f) * a;
}

__device__ __forceinline__ uint32_t byte_at(uint64_t k, int b) {
    return (uint32_t)(k >> (56 - 8 * b)) & 0xFFu;
}

// byte b of k minus byte b of lo, over max(byte b of hi - byte b of lo, 1)
__device__ __forceinline__ void key_features(uint64_t k, uint64_t lo, uint64_t hi, float (&x)[8]) {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int l = (int)byte_at(lo, b), w = (int)byte_at(hi, b) - l;
        x[b] = (float)((int)byte_at(k, b) - l) / (float)(w > 1 ? w : 1);
    }
}

__device__ __forceinline__ uint64_t bytes_minmax(uint64_t a, uint64_t b, bool take_max) {
    uint64_t r = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t x = byte_at(a, i), y = byte_at(b, i);
        r |= (uint64_t)(take_max ? (x > y ? x : y) : (x < y ? x : y)) << (56 - 8 * i);
    }
    return r;
}

// byte-wise minimum and maximum of m keys into out[0], out[1] (256 threads)
__device__ void sample_range(const uint64_t* smp, uint32_t m, uint64_t* out) {
    __shared__ uint64_t rlo[256], rhi[256];
    const uint32_t tid = threadIdx.x;
    uint64_t lo = ~0ull, hi = 0;
    for (uint32_t i = tid; i < m; i += 256) {
        lo = bytes_minmax(lo, smp[i], false);
        hi = bytes_minmax(hi, smp[i], true);
    }
    rlo[tid] = lo;
    rhi[tid] = hi;
    __syncthreads();
    for (uint32_t off = 128; off > 0; off >>= 1) {
        if (tid < off) {
            rlo[tid] = bytes_minmax(rlo[tid], rlo[tid + off], false);
            rhi[tid] = bytes_minmax(rhi[tid], rhi[tid + off], true);
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[0] = rlo[0];
        out[1] = rhi[0];
    }
}

// forward pass for one key with weights w (LDS or global); optional activations
__device__ __forceinline__ float mlp_forward(const float* w, const float (&x)[8], float* h1o,
                                             float* h2o) {
    float h1[kH];
#pragma unroll
    for (int i = 0; i < kH; ++i) {
        float z = w[oB1 + i];
#pragma unroll
        for (int j = 0; j < 8; ++j) z = fmaf(w[oW1 + i * 8 + j], x[j], z);
        h1[i] = z > 0.0f ? z : 0.0f;
    }
    float z3 = w[oB3];
#pragma unroll 4
    for (int i = 0; i < kH; ++i) {
        float z = w[oB2 + i];
#pragma unroll
        for (int j = 0; j < kH; ++j) z = fmaf(w[oW2 + i * kH + j], h1[j], z);
        const float h = z > 0.0f ? z : 0.0f;
        if (h2o) h2o[i] = h;
        z3 = fmaf(w[oW3 + i], h, z3);
    }
    if (h1o) {
#pragma unroll
        for (int i = 0; i < kH; ++i) h1o[i] = h1[i];
    }
    return 1.0f / (1.0f + __expf(-z3));
}

// Adam update of parameter p from the summed gradient g (step t >= 1).
__device__ __forceinline__ float adam(float w, float g, float& m1, float& m2, uint32_t t,
                                      float lr) {
    m1 = kB1 * m1 + (1.0f - kB1) * g;
    m2 = kB2 * m2 + (1.0f - kB2) * g * g;
    const float mh = m1 / (1.0f - __powf(kB1, (float)t));
    const float vh = m2 / (1.0f - __powf(kB2, (float)t));
    return w - lr * mh / (sqrtf(vh) + kEps);
}

// sum of the previous step's partial gradients for parameter p, fixed order
__device__ __forceinline__ float summed_grad(const LearnCtx& c, uint32_t slot, uint32_t b,
                                             uint32_t p) {
    float g = 0.0f;
#pragma unroll 8
    for (uint32_t q = 0; q < c.groups; ++q) g += pbuf(c, slot, b, q)[p];
    return g;
}

// ---------------------------------------------------------------------------
// one training step: update from the previous partial gradients, then the
// partial gradients of this step's weights over this group's 256 samples.

__device__ __forceinline__ void learn_step_body(const LearnCtx& c, uint32_t slot, uint32_t step,
                                                float lr) {
    // 80 KB in all, so that two workgroups fit on one compute unit
    __shared__ float w[kNPS];
    __shared__ __align__(16) float sh1[kGrp * kS1];  // per sample: h1, then the 8 features
    __shared__ float sv[kGrp * kS];  // per sample: h2 and d3, then d2, then d1
    const uint32_t grp = blockIdx.x, tid = threadIdx.x;
    const uint32_t prev = (step + 1) & 1u, cur = step & 1u;
    const float* wp = wbuf(c, slot, prev);
    for (uint32_t p = tid; p < kNP; p += kGrp) {
        float wv = wp[p];
        float m1 = 0.0f, m2 = 0.0f;
        if (step > 0) {
            const float g = summed_grad(c, slot, prev, p);
            m1 = m1buf(c, slot, prev)[p];
            m2 = m2buf(c, slot, prev)[p];
            wv = adam(wv, g, m1, m2, step, lr);
        }
        w[p] = wv;
        if (grp == 0) {
            wbuf(c, slot, cur)[p] = wv;
            m1buf(c, slot, cur)[p] = m1;
            m2buf(c, slot, cur)[p] = m2;
        }
    }
    __syncthreads();
    // forward and backward for this thread's sample
    const uint32_t i = grp * kGrp + tid;
    const uint64_t lo = c.range[2 * slot], hi = c.range[2 * slot + 1];
    float x[8];
    key_features(c.samples[(size_t)slot * kLearnM + i], lo, hi, x);
    float h1[kH], h2[kH];
    const float y = mlp_forward(w, x, h1, h2);
    const float t = ((float)i + 0.5f) / (float)c.m;
    const float d3 = (2.0f / (float)c.m) * (y - t) * y * (1.0f - y);
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        sv[tid * kS + j] = h2[j];
        sh1[tid * kS1 + j] = h1[j];
    }
    sv[tid * kS + kH] = d3;
#pragma unroll
    for (int j = 0; j < 8; ++j) sh1[tid * kS1 + kH + j] = x[j];
    __syncthreads();
    float* out = pbuf(c, slot, cur, grp);
    // third layer (every sample's h2 and d3, read before d2 replaces them):
    // thread 32 + j owns w3[j], thread 64 owns b3
    if (tid >= 32 && tid < 64) {
        float g = 0.0f;
#pragma unroll 8
        for (uint32_t b = 0; b < kGrp; ++b) g = fmaf(sv[b * kS + kH], sv[b * kS + tid - 32], g);
        out[oW3 + tid - 32] = g;
    } else if (tid == 64) {
        float g = 0.0f;
#pragma unroll 8
        for (uint32_t b = 0; b < kGrp; ++b) g += sv[b * kS + kH];
        out[oB3] = g;
    }
    // back-propagation to both hidden layers, in registers (d2 is formed
    // again from h2 once the third layer's sums are done with h2)
    float d1[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) d1[j] = 0.0f;
#pragma unroll 4
    for (int r = 0; r < kH; ++r) {
        const float d2 = h2[r] > 0.0f ? d3 * w[oW3 + r] : 0.0f;
#pragma unroll
        for (int j = 0; j < kH; ++j) d1[j] = fmaf(d2, w[oW2 + r * kH + j], d1[j]);
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) d1[j] = h1[j] > 0.0f ? d1[j] : 0.0f;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kH; ++r) sv[tid * kS + r] = h2[r] > 0.0f ? d3 * w[oW3 + r] : 0.0f;
    __syncthreads();
    // second layer: thread t owns W2[t / 8][4 (t % 8) .. +3], and b2[t] for t < 32
    {
        const uint32_t r = tid >> 3, jq = (tid & 7u) << 2;
        float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, g3 = 0.0f;
#pragma unroll 8
        for (uint32_t b = 0; b < kGrp; ++b) {
            const float d = sv[b * kS + r];
            const float4 h = *reinterpret_cast<const float4*>(&sh1[b * kS1 + jq]);
            g0 = fmaf(d, h.x, g0);
            g1 = fmaf(d, h.y, g1);
            g2 = fmaf(d, h.z, g2);
            g3 = fmaf(d, h.w, g3);
        }
        float* o = out + oW2 + r * kH + jq;
        o[0] = g0;
        o[1] = g1;
        o[2] = g2;
        o[3] = g3;
        if (tid < 32) {
            float g = 0.0f;
#pragma unroll 8
            for (uint32_t b = 0; b < kGrp; ++b) g += sv[b * kS + tid];
            out[oB2 + tid] = g;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kH; ++j) sv[tid * kS + j] = d1[j];
    __syncthreads();
    // first layer: thread t owns W1[t / 8][t % 8], and b1[t] for t < 32
    {
        const uint32_t r = tid >> 3, j = tid & 7u;
        float g = 0.0f;
#pragma unroll 8
        for (uint32_t b = 0; b < kGrp; ++b) g = fmaf(sv[b * kS + r], sh1[b * kS1 + kH + j], g);
        out[oW1 + tid] = g;
        if (tid < 32) {
            float gb = 0.0f;
#pragma unroll 8
            for (uint32_t b = 0; b < kGrp; ++b) gb += sv[b * kS + tid];
            out[oB1 + tid] = gb;
        }
    }
}

// grid (groups, slots); graph mode strides over the learned segments of the pass
__global__ __launch_bounds__(256) void k_learn_step(LearnCtx c, uint32_t step, float lr,
                                                    const uint32_t* wcnt, uint32_t cap,
                                                    const Globals* glob) {
    const uint32_t units = block_work_count(wcnt, cap, glob, gridDim.y);
    for (uint32_t slot = blockIdx.y; slot < units; slot += gridDim.y) {
        learn_step_body(c, slot, step, lr);
        __syncthreads();
    }
}

// Final Adam update after `steps` steps: weights land in buffer (steps & 1).
__device__ void learn_final_update(const LearnCtx& c, uint32_t slot, uint32_t steps, float lr,
                                   float* w_lds) {
    const uint32_t prev = (steps + 1) & 1u, cur = steps & 1u;
    for (uint32_t p = threadIdx.x; p < kNP; p += blockDim.x) {
        const float g = summed_grad(c, slot, prev, p);
        float m1 = m1buf(c, slot, prev)[p], m2 = m2buf(c, slot, prev)[p];
        const float wv = adam(wbuf(c, slot, prev)[p], g, m1, m2, steps, lr);
        if (w_lds) w_lds[p] = wv;
        wbuf(c, slot, cur)[p] = wv;
    }
}

// initial weights into buffer 1 (read by step 0 as "previous") and the
// feature range of the caller's sample
__global__ __launch_bounds__(256) void k_learn_init(LearnCtx c, uint64_t seed) {
    const uint32_t slot = blockIdx.x;
    for (uint32_t p = threadIdx.x; p < kNP; p += blockDim.x) wbuf(c, slot, 1)[p] = init_weight(seed, p);
    sample_range(c.samples + (size_t)slot * kLearnM, c.m, c.range + 2 * slot);
}

__global__ __launch_bounds__(256) void k_learn_final(LearnCtx c, uint32_t steps, float lr) {
    learn_final_update(c, blockIdx.x, steps, lr, nullptr);
}

// ---------------------------------------------------------------------------
// in-sort path: sample + sort, then propose splitters and build the tree

__device__ __forceinline__ void learn_prep_body(const LearnCtx& c, uint32_t slot,
                                                const LSeg* lseg, const uint32_t* learn_seg,
                                                const uint64_t* key_in, uint64_t seed) {
    __shared__ uint64_t smp[kLearnM];
    const LSeg g = lseg[learn_seg[slot]];
    const uint64_t sseed = mix64(seed ^ 0x5A5A5A5A5A5A5A5Aull ^ mix64(((uint64_t)g.begin << 32) | g.depth));
    for (uint32_t r = threadIdx.x; r < kLearnM; r += blockDim.x) {
        const uint64_t h = mix64(sseed + 0x9E3779B97F4A7C15ull * (r + 1));
        smp[r] = key_in[g.begin + (uint32_t)(((h >> 32) * (uint64_t)g.size) >> 32)];
    }
    __syncthreads();
    for (uint32_t kk = 2; kk <= kLearnM; kk <<= 1) {
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < kLearnM / 2; i += blockDim.x) {
                const uint32_t lo = 2 * i - (i & (j - 1)), hi = lo + j;
                const bool up = (lo & kk) == 0;
                const uint64_t a = smp[lo], b = smp[hi];
                if ((a > b) == up) {
                    smp[lo] = b;
                    smp[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t r = threadIdx.x; r < kLearnM; r += blockDim.x) c.samples[(size_t)slot * kLearnM + r] = smp[r];
    for (uint32_t p = threadIdx.x; p < kNP; p += blockDim.x) wbuf(c, slot, 1)[p] = init_weight(seed, p);
    sample_range(smp, kLearnM, c.range + 2 * slot);
}

__global__ __launch_bounds__(256) void k_learn_prep(LearnCtx c, const LSeg* lseg,
                                                    const uint32_t* learn_seg,
                                                    const uint64_t* key_in, uint64_t seed,
                                                    const uint32_t* wcnt, uint32_t cap,
                                                    const Globals* glob) {
    const uint32_t units = block_work_count(wcnt, cap, glob, gridDim.x);
    for (uint32_t slot = blockIdx.x; slot < units; slot += gridDim.x) {
        learn_prep_body(c, slot, lseg, learn_seg, key_in, seed);
        __syncthreads();
    }
}

// first index of sorted a[0..m) holding a value >= x (strict: > x)
__device__ __forceinline__ uint32_t bound(const uint64_t* a, uint32_t m, uint64_t x, bool strict) {
    uint32_t lo = 0, hi = m;
    while (lo < hi) {
        const uint32_t md = (lo + hi) >> 1;
        if (strict ? a[md] <= x : a[md] < x) lo = md + 1; else hi = md;
    }
    return lo;
}

// LDS of one proposal (one workgroup of 256 threads).
struct ProposeLds {
    uint64_t S[kLearnM];           // the sorted sample
    float F[kLearnM];              // model outputs made monotone by a running maximum
    uint64_t Hk[1u << (kDMax - 1)];  // heavy-hitter keys, ascending
    uint64_t Qk[1u << kDMax];      // quantile splitters, non-decreasing
    uint64_t spl[1u << kDMax];     // the proposal: both lists merged
    float tmx[256];
    uint32_t tsum[256];
    uint32_t cnt, gmax;
};

// block-wide sum of one value per thread (256 threads)
__device__ __forceinline__ uint32_t block_sum256(uint32_t x, ProposeLds& L) {
    for (uint32_t o = 32; o > 0; o >>= 1) x += __shfl_xor(x, (int)o);
    __syncthreads();
    if (threadIdx.x == 0) L.cnt = 0;
    __syncthreads();
    if ((threadIdx.x & 63u) == 0) atomicAdd(&L.cnt, x);
    __syncthreads();
    return L.cnt;
}

// Splitter proposal of the model with weights w (LDS) for its sorted sample
// smp[0..m) (m a multiple of 256, <= kLearnM), feature range (flo, fhi):
//  1. F_i = running maximum of the model outputs (a monotone CDF); y_out[i]
//     receives the outputs themselves when given;
//  2. heavy hitters: the keys of runs of >= L* equal sample keys, L* the
//     smallest L >= 2 with at most v/2 such runs, get splitters of their own,
//     so each becomes an equality bucket (Section 3.1);
//  3. the other vq = v - |heavy| splitters are model quantiles: splitter j
//     (1 <= j <= vq) is the sample key at the first i with
//     F_i >= j / (vq + 1) (in float32), or the last sample key;
//  4. L.spl = both lists merged (sorted, repeats allowed);
//  5. the check on the sample: the largest number of sample keys strictly
//     between neighbouring splitters (or outside them) against
//     beta * m / (v + 1).
// Returns true (in every thread) if the proposal is rejected.
__device__ __forceinline__ bool propose_body(const float* w, const uint64_t* smp, uint32_t m, uint32_t v,
                             float beta, uint64_t flo, uint64_t fhi, float* y_out,
                             ProposeLds& L) {
    const uint32_t tid = threadIdx.x;
    const uint32_t per = m / 256u;  // consecutive samples per thread
    for (uint32_t i = tid; i < m; i += 256) L.S[i] = smp[i];
    if (tid == 0) L.gmax = 0;
    __syncthreads();
    float run = 0.0f;
    for (uint32_t e = 0; e < per; ++e) {
        float x[8];
        key_features(L.S[tid * per + e], flo, fhi, x);
        const float y = mlp_forward(w, x, nullptr, nullptr);
        if (y_out) y_out[tid * per + e] = y;
        run = y > run ? y : run;
        L.F[tid * per + e] = run;
    }
    L.tmx[tid] = run;
    __syncthreads();
    for (uint32_t off = 1; off < 256; off <<= 1) {
        const float o = tid >= off ? L.tmx[tid - off] : 0.0f;
        __syncthreads();
        if (o > L.tmx[tid]) L.tmx[tid] = o;
        __syncthreads();
    }
    const float before = tid ? L.tmx[tid - 1] : 0.0f;
    for (uint32_t e = 0; e < per; ++e)
        if (L.F[tid * per + e] < before) L.F[tid * per + e] = before;
    __syncthreads();
    // run lengths, recorded at the last key of every run (0 elsewhere)
    constexpr uint32_t kPer = kLearnM / 256;
    uint32_t rl[kPer];
#pragma unroll
    for (uint32_t e = 0; e < kPer; ++e) {
        const uint32_t i = tid * per + e;
        const bool last = e < per && (i + 1 == m || L.S[i + 1] != L.S[i]);
        rl[e] = last ? i + 1 - bound(L.S, m, L.S[i], false) : 0u;
    }
    // L* by bisection: the count of runs of length >= L falls as L grows
    const uint32_t cap = v / 2;
    uint32_t lo = 2, hi = m + 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        uint32_t c = 0;
#pragma unroll
        for (uint32_t e = 0; e < kPer; ++e) c += rl[e] >= mid ? 1u : 0u;
        if (block_sum256(c, L) <= cap) hi = mid; else lo = mid + 1;
    }
    // heavy keys in sample order: exclusive scan of the flags over the threads
    uint32_t mine = 0;
#pragma unroll
    for (uint32_t e = 0; e < kPer; ++e) mine += rl[e] >= lo ? 1u : 0u;
    L.tsum[tid] = mine;
    __syncthreads();
    for (uint32_t off = 1; off < 256; off <<= 1) {
        const uint32_t o = tid >= off ? L.tsum[tid - off] : 0u;
        __syncthreads();
        L.tsum[tid] += o;
        __syncthreads();
    }
    const uint32_t nh = L.tsum[255];
    uint32_t pos = L.tsum[tid] - mine;
#pragma unroll
    for (uint32_t e = 0; e < kPer; ++e)
        if (rl[e] >= lo) L.Hk[pos++] = L.S[tid * per + e];
    // quantile splitters; j / (vq + 1) is formed in double and rounded once to
    // float, which equals the correctly rounded float quotient (a quotient of
    // integers below 2^11 is never within 2^-53 relative of a float midpoint)
    const uint32_t vq = v - nh;
    for (uint32_t j = tid + 1; j <= vq; j += 256) {
        const float q = (float)((double)j / (double)(vq + 1));
        uint32_t a = 0, b = m;
        while (a < b) {
            const uint32_t md = (a + b) >> 1;
            if (L.F[md] < q) a = md + 1; else b = md;
        }
        L.Qk[j - 1] = L.S[a < m ? a : m - 1];
    }
    __syncthreads();
    // merge: a heavy key goes before equal quantile keys
    for (uint32_t a = tid; a < nh; a += 256) L.spl[a + bound(L.Qk, vq, L.Hk[a], false)] = L.Hk[a];
    for (uint32_t b = tid; b < vq; b += 256) L.spl[b + bound(L.Hk, nh, L.Qk[b], true)] = L.Qk[b];
    __syncthreads();
    // range bucket j (between splitters j-1 and j) counted on the sample
    uint32_t mx = 0;
    for (uint32_t j = tid; j <= v; j += 256) {
        const uint32_t a = j ? bound(L.S, m, L.spl[j - 1], true) : 0u;
        const uint32_t b = j < v ? bound(L.S, m, L.spl[j], false) : m;
        const uint32_t n = b > a ? b - a : 0u;
        mx = n > mx ? n : mx;
    }
    atomicMax(&L.gmax, mx);
    __syncthreads();
    return (double)L.gmax > (double)beta * (double)m / (double)(v + 1);
}

// Final update, the proposal, the check on the sample, and the splitter tree.
__device__ __forceinline__ void learn_finish_body(const LearnCtx& c, uint32_t slot, LSeg* lseg,
                                                  const uint32_t* learn_seg, uint32_t steps,
                                                  float lr, float beta, Globals* glob,
                                                  uint64_t* tree_lo, uint64_t* tree_in,
                                                  uint8_t* tree_lcp, uint16_t* jump,
                                                  const KeyCodec& kc) {
    __shared__ float w[kNPS];
    __shared__ ProposeLds L;
    const uint32_t tid = threadIdx.x;
    const uint32_t si = learn_seg[slot];
    const LSeg g = lseg[si];
    learn_final_update(c, slot, steps, lr, w);
    __syncthreads();
    const uint64_t* smp = c.samples + (size_t)slot * kLearnM;
    const bool reject = propose_body(w, smp, kLearnM, g.v, beta, c.range[2 * slot],
                                     c.range[2 * slot + 1], nullptr, L);
    if (tid == 0) {  // the proposal's sample imbalance, for the statistics
        const uint32_t milli =
            (uint32_t)((1000.0 * L.gmax * (g.v + 1)) / (double)kLearnM + 0.5);
        atomicAdd(&glob->learned_props, 1u);
        atomicMax(&glob->imb_max_milli, milli);
        atomicAdd(&glob->imb_sum_milli, (unsigned long long)milli);
    }
    if (reject) {
        if (tid == 0) {
            lseg[si].pad0 = 0xFFFFFFFFu;  // the sampled tree is built instead
            atomicAdd(&glob->fallbacks, 1u);
        }
        return;
    }
    uint64_t* lo_out = tree_lo + g.tree_base;
    uint64_t* in_out = tree_in + g.tree_base;
    uint8_t* lcp_out = tree_lcp + g.tree_base;
    for (uint32_t j = tid; j <= g.v; j += 256) {
        if (j < g.v) {
            const uint64_t x = L.spl[j];
            lo_out[inorder_node(j, g.d)] = x;
            in_out[j] = x;
            uint8_t l = 0;
            if (j > 0 && L.spl[j - 1] != x) l = (uint8_t)codec_lcp(kc, L.spl[j - 1], x);
            lcp_out[j] = l;
        } else {
            lo_out[0] = 0;
            in_out[j] = 0;
            lcp_out[j] = 0;
        }
    }
    if (jump) {  // the level-order tree in LDS (the quantile list is done with), then the table
        uint64_t* t = L.Qk;
        __syncthreads();
        for (uint32_t j = tid; j < g.v; j += 256) t[inorder_node(j, g.d)] = L.spl[j];
        __syncthreads();
        build_jump_table(t, g.d, g.v, jump + (uint64_t)g.tree_base * kJumpPerTreeSlot, tid, 256);
    }
}

__global__ __launch_bounds__(256) void k_learn_finish(LearnCtx c, LSeg* lseg,
                                                      const uint32_t* learn_seg, uint32_t steps,
                                                      float lr, float beta, Globals* glob,
                                                      uint64_t* tree_lo, uint64_t* tree_in,
                                                      uint8_t* tree_lcp, uint16_t* jump,
                                                      const uint32_t* wcnt, uint32_t cap,
                                                      KeyCodec kc) {
    const uint32_t units = block_work_count(wcnt, cap, glob, gridDim.x);
    for (uint32_t slot = blockIdx.x; slot < units; slot += gridDim.x) {
        learn_finish_body(c, slot, lseg, learn_seg, steps, lr, beta, glob, tree_lo, tree_in,
                          tree_lcp, jump, kc);
        __syncthreads();
    }
}

// Largest range bucket of every segment still on learned splitters against
// beta * |S| / (v + 1); an imbalanced segment is switched back to sampled
// splitters.
__device__ __forceinline__ void learn_check_body(uint32_t slot, LSeg* lseg,
                                                 const uint32_t* learn_seg, const uint32_t* cs,
                                                 float beta, Globals* glob) {
    __shared__ uint32_t smax;
    const uint32_t si = learn_seg[slot];
    const LSeg g = lseg[si];
    if (g.pad0 == 0xFFFFFFFFu) return;  // rejected on its sample already
    if (threadIdx.x == 0) smax = 0;
    __syncthreads();
    uint32_t mx = 0;
    for (uint32_t b = threadIdx.x * 2; b < g.k; b += 2 * 256) {
        uint32_t t = 0;
        for (uint32_t q = 0; q < g.chunks; ++q) t += cs[g.cs_base + (uint64_t)q * g.k + b];
        mx = t > mx ? t : mx;
    }
    atomicMax(&smax, mx);
    __syncthreads();
    if (threadIdx.x == 0 && (double)smax > (double)beta * g.size / (g.v + 1)) {
        lseg[si].pad0 = 0xFFFFFFFFu;
        lseg[si].redo_tune |= kRedoBit;  // redo: sampled tree, classification and column scan
        atomicAdd(&glob->fallbacks, 1u);
        atomicAdd(&glob->late_fallbacks, 1u);
    }
}

__global__ __launch_bounds__(256) void k_learn_check(LSeg* lseg, const uint32_t* learn_seg,
                                                     const uint32_t* cs, float beta,
                                                     Globals* glob, const uint32_t* wcnt,
                                                     uint32_t cap) {
    const uint32_t units = block_work_count(wcnt, cap, glob, gridDim.x);
    for (uint32_t slot = blockIdx.x; slot < units; slot += gridDim.x) {
        learn_check_body(slot, lseg, learn_seg, cs, beta, glob);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// building blocks for callers and step-level checks

__global__ __launch_bounds__(256) void k_mlp_eval(const float* w, const uint64_t* keys, uint32_t n,
                                                  uint64_t lo, uint64_t hi, float* out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[8];
    key_features(keys[i], lo, hi, x);
    out[i] = mlp_forward(w, x, nullptr, nullptr);
}

// the proposal for a caller's model and sorted sample (one workgroup)
__global__ __launch_bounds__(256) void k_mlp_propose(const float* params, const uint64_t* keys,
                                                     uint32_t m, uint32_t v, float beta,
                                                     uint64_t* out_spl, float* out_y,
                                                     uint32_t* out_reject) {
    __shared__ float w[kNPS];
    __shared__ uint64_t range[2];
    __shared__ ProposeLds L;
    for (uint32_t p = threadIdx.x; p < kNP; p += 256) w[p] = params[p];
    sample_range(keys, m, range);
    __syncthreads();
    const bool reject = propose_body(w, keys, m, v, beta, range[0], range[1], out_y, L);
    for (uint32_t j = threadIdx.x; j < v; j += 256) out_spl[j] = L.spl[j];
    if (threadIdx.x == 0) *out_reject = reject ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_learn_sum(LearnCtx c, uint32_t b, float* out) {
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < kNP; p += gridDim.x * blockDim.x)
        out[p] = summed_grad(c, 0, b, p);
}

// ---------------------------------------------------------------------------
// host-side launchers

size_t learn_bytes(uint32_t slots, uint32_t m) {
    const size_t groups = m / kGrp;
    return (size_t)slots * kLearnM * 8 + (size_t)slots * 2 * kNPS * 4 * 3 +
           (size_t)slots * 2 * groups * kNPS * 4 + (size_t)slots * 16;
}

LearnCtx learn_ctx(void* mem, uint32_t slots, uint32_t m) {
    LearnCtx c;
    char* p = (char*)mem;
    c.samples = (uint64_t*)p;
    p += (size_t)slots * kLearnM * 8;
    c.range = (uint64_t*)p;
    p += (size_t)slots * 16;
    c.W = (float*)p;
    p += (size_t)slots * 2 * kNPS * 4;
    c.M1 = (float*)p;
    p += (size_t)slots * 2 * kNPS * 4;
    c.M2 = (float*)p;
    p += (size_t)slots * 2 * kNPS * 4;
    c.part = (float*)p;
    c.m = m;
    c.groups = m / kGrp;
    return c;
}

void launch_learn_sort_trees(const LearnCtx& c, uint32_t slots, LSeg* lseg,
                             const uint32_t* learn_seg, const uint64_t* key_in, uint64_t seed,
                             uint32_t steps, float lr, float beta, Globals* glob,
                             uint64_t* tree_lo, uint64_t* tree_in, uint8_t* tree_lcp,
                             uint16_t* jump, const KeyCodec& kc, const Dyn& dy, hipStream_t st) {
    const uint32_t g = dy.cnt ? dy.grid : slots;
    hipLaunchKernelGGL(k_learn_prep, dim3(g), dim3(256), 0, st, c, lseg, learn_seg, key_in, seed,
                       dy.cnt, dy.cap, glob);
    for (uint32_t s = 0; s < steps; ++s)
        hipLaunchKernelGGL(k_learn_step, dim3(c.groups, g), dim3(kGrp), 0, st, c, s, lr, dy.cnt,
                           dy.cap, glob);
    hipLaunchKernelGGL(k_learn_finish, dim3(g), dim3(256), 0, st, c, lseg, learn_seg, steps, lr,
                       beta, glob, tree_lo, tree_in, tree_lcp, jump, dy.cnt, dy.cap, kc);
}

void launch_learn_check(uint32_t slots, LSeg* lseg, const uint32_t* learn_seg, const uint32_t* cs,
                        float beta, Globals* glob, const Dyn& dy, hipStream_t st) {
    hipLaunchKernelGGL(k_learn_check, dim3(dy.cnt ? dy.grid : slots), dim3(256), 0, st, lseg,
                       learn_seg, cs, beta, glob, dy.cnt, dy.cap);
}

// train on caller-sorted keys (slot 0); final weights copied to out
void launch_mlp_train(const LearnCtx& c, const uint64_t* sorted_keys, uint32_t m, uint32_t steps,
                      float lr, uint64_t seed, float* out, hipStream_t st) {
    (void)hipMemcpyAsync(c.samples, sorted_keys, (size_t)m * 8, hipMemcpyDeviceToDevice, st);
    hipLaunchKernelGGL(k_learn_init, dim3(1), dim3(256), 0, st, c, seed);
    for (uint32_t s = 0; s < steps; ++s)
        hipLaunchKernelGGL(k_learn_step, dim3(c.groups, 1), dim3(kGrp), 0, st, c, s, lr,
                           (const uint32_t*)nullptr, 0u, (const Globals*)nullptr);
    if (steps) {
        hipLaunchKernelGGL(k_learn_final, dim3(1), dim3(256), 0, st, c, steps, lr);
        (void)hipMemcpyAsync(out, c.W + (size_t)(steps & 1u) * kNPS, kNP * 4, hipMemcpyDeviceToDevice, st);
    } else {
        (void)hipMemcpyAsync(out, c.W + kNPS, kNP * 4, hipMemcpyDeviceToDevice, st);
    }
}

// gradient at `params` over caller-sorted keys (slot 0)
void launch_mlp_grad(const LearnCtx& c, const float* params, const uint64_t* sorted_keys,
                     uint32_t m, float* out, hipStream_t st) {
    (void)hipMemcpyAsync(c.samples, sorted_keys, (size_t)m * 8, hipMemcpyDeviceToDevice, st);
    hipLaunchKernelGGL(k_learn_init, dim3(1), dim3(256), 0, st, c, 0ull);
    (void)hipMemcpyAsync(c.W + kNPS, params, kNP * 4, hipMemcpyDeviceToDevice, st);
    hipLaunchKernelGGL(k_learn_step, dim3(c.groups, 1), dim3(kGrp), 0, st, c, 0u, 0.0f,
                       (const uint32_t*)nullptr, 0u, (const Globals*)nullptr);
    hipLaunchKernelGGL(k_learn_sum, dim3(8), dim3(256), 0, st, c, 0u, out);
}

void launch_mlp_propose(const float* params, const uint64_t* sorted_keys, uint32_t m, uint32_t v,
                        float beta, uint64_t* out_spl, float* out_y, uint32_t* out_reject,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_propose, dim3(1), dim3(256), 0, st, params, sorted_keys, m, v, beta,
                       out_spl, out_y, out_reject);
}

void launch_mlp_eval(const float* params, const uint64_t* keys, uint32_t n, uint64_t lo,
                     uint64_t hi, float* out, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_mlp_eval, dim3((n + 255) / 256), dim3(256), 0, st, params, keys, n, lo, hi,
                       out);
}

}  // namespace s5
