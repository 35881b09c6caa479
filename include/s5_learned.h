/*
 * s5_learned.h -- the learned splitter model of the S^5 library as building
 * blocks (device pointers, stream-ordered, same conventions as s5.h).
 *
 * The paper proposes adapting string sample sort to its input by inspecting
 * the sample (appendix A, "Adaptivity").  With splitter_mode =
 * S5_SPLIT_LEARNED, s5_sort_ex models the distribution function of every
 * segment of >= 65536 strings with a small network trained on 4096 sampled
 * keys and places the splitters at its quantiles; classification remains the
 * exact comparison of Section 3.1, so the output never depends on the model.
 * A proposal is replaced by sampled splitters if a range bucket holds more
 * than imbalance_bound times its ideal share |S|/(v+1), counted first on the
 * training sample and then on the exact bucket histogram (s5_stats.fallbacks
 * counts both).  The calls below expose the same model, training and
 * evaluation code.
 *
 * Model: one feature per key byte b (most significant first),
 * (c_b - lo_b) / max(hi_b - lo_b, 1), where lo and hi hold the byte-wise
 * minimum and maximum over the training keys (packed like the keys; lo = 0,
 * hi = ~0 gives plain c_b / 255); two hidden layers of 32 ReLU units; sigmoid
 * output.  Parameters (1377 floats):
 * W1 (32x8, row major), b1 (32), W2 (32x32), b2 (32), w3 (32), b3 (1).
 * Initial weights: splitmix64 as a counter-based generator, parameter i gets
 * (2u - 1) * a with u = top 24 bits of splitmix64(seed + i + 1) / 2^24 and
 * a = sqrt(6/8) (W1), sqrt(6/32) (W2), 0.1 sqrt(6/32) (w3), biases 0.
 * Training: full-batch mean squared error against the empirical CDF
 * t_i = (i + 0.5)/m of the sorted keys, Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8), one update per step.
 */
#ifndef S5_LEARNED_H
#define S5_LEARNED_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Train from the initial weights of `seed` on m sorted keys (256 <= m <= 4096,
 * m a multiple of 256; features scaled by the keys' own byte-wise range) for
 * `steps` Adam steps of learning rate lr; the 1377 final parameters go to
 * out_params.  Synchronizes the stream.  Returns S5_OK, S5_ERR_INVALID (bad m,
 * NULL pointer, steps > 100000), S5_ERR_NOMEM or S5_ERR_HIP. */
int s5_mlp_train(const uint64_t* sorted_keys, uint32_t m, uint32_t steps, float lr,
                 uint64_t seed, float* out_params, hipStream_t stream);

/* Gradient of the mean squared error at `params` over m sorted keys (same
 * constraints on m, features scaled as in training) into out_grad (1377
 * floats).  Synchronizes the stream; same return codes. */
int s5_mlp_grad(const float* params, const uint64_t* sorted_keys, uint32_t m, float* out_grad,
                hipStream_t stream);

/* Model output (estimated CDF) for n keys into out (n floats), features
 * scaled by the byte-wise range (lo, hi).  Asynchronous; returns S5_OK,
 * S5_ERR_INVALID (NULL pointer with n > 0) or S5_ERR_HIP. */
int s5_mlp_eval(const float* params, const uint64_t* keys, uint32_t n, uint64_t lo, uint64_t hi,
                float* out, hipStream_t stream);

/* The splitter proposal of model `params` for its own sorted training sample
 * (256 <= m <= 4096, m a multiple of 256; 1 <= v <= 1023; features scaled by
 * the sample's byte-wise range as in training), the code the sort runs on
 * every learned segment:
 *   1. F_i = running maximum of the model outputs over the sample (a monotone
 *      estimate of the distribution function); out_cdf[i] receives the
 *      outputs themselves (before the running maximum), m floats;
 *   2. heavy hitters: the keys of runs of >= L* equal sample keys, L* the
 *      smallest L >= 2 with at most v/2 such runs, are splitters of their own,
 *      so each becomes an equality bucket (Section 3.1, equality buckets;
 *      appendix A, "Adaptivity": inspecting the sample);
 *   3. the other vq = v - (number of heavy keys) splitters are quantiles:
 *      splitter j (1 <= j <= vq) is the sample key at the first i with
 *      F_i >= j / (vq + 1), compared in float32, else the last sample key;
 *   4. out_splitters (v uint64) = both lists merged in ascending order
 *      (repeats allowed: equal splitters leave empty range buckets);
 *   5. *out_reject (one uint32) = 1 if some range bucket of the sample itself
 *      (keys strictly between neighbouring splitters, or outside them) holds
 *      more than beta * m / (v + 1) keys, else 0; the sort then uses sampled
 *      splitters for that segment.
 * Asynchronous; returns S5_OK, S5_ERR_INVALID (bad m or v, NULL pointer,
 * beta <= 0) or S5_ERR_HIP. */
int s5_mlp_propose(const float* params, const uint64_t* sorted_keys, uint32_t m, uint32_t v,
                   float beta, uint64_t* out_splitters, float* out_cdf, uint32_t* out_reject,
                   hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* S5_LEARNED_H */
