// Host-side launchers of the S^5 kernels (defined in s5_kernels.hip and
// s5_learn.hip, called by s5_host.cpp).  Not part of the public ABI.
//
// Pass kernels take a Dyn: host-driven launches (Dyn{}) size the grid to the
// work the host read back; graph-captured launches use a fixed grid that
// strides over a device-side count.
#pragma once

#include "s5_internal.h"

namespace s5 {

void launch_init_keys(const uint8_t* chars, uint64_t chars_len, const uint64_t* offsets,
                      uint32_t n, uint64_t* key, uint64_t* key2, uint64_t* key3, uint32_t* idx,
                      Globals* glob, const KeyCodec& kc, hipStream_t st);
void launch_alphabet(const uint8_t* chars, uint64_t chars_len, const uint64_t* offsets,
                     uint32_t n, uint32_t samples, uint32_t* bitmap, hipStream_t st);
void launch_prefix_keys(const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                        uint32_t depth, uint64_t* key, hipStream_t st);
void launch_plan_roots(const uint64_t* set_begin, uint32_t num_sets, uint32_t n,
                       uint32_t* out_perm, uint32_t* out_lcp, const PlanCtx& ctx, hipStream_t st);
void launch_pass_stats(const Counters* cur, const Counters* next, Globals* glob, uint32_t level,
                       hipStream_t st);
void launch_zero_words(void* p, size_t bytes, hipStream_t st);
// copy `bytes` (a multiple of 4) from device memory into pinned host memory
// (its device address `dst`), then store `seq` into the host word `flag`
void launch_publish(const void* src, size_t bytes, void* dst, uint32_t* flag, uint32_t seq,
                    hipStream_t st);

void launch_sample_tree(uint32_t n_large, const LSeg* lseg, const uint64_t* key_in,
                        uint32_t alpha, uint32_t vmax, uint64_t seed, uint64_t* tree_lo,
                        uint64_t* tree_in, uint8_t* tree_lcp, uint16_t* jump, uint32_t* tile_tab,
                        uint32_t* chunk_tab, Counters* next_cnt, const Globals* glob,
                        const Dyn& dy, uint32_t redo, const KeyCodec& kc, hipStream_t st);
void launch_classify(uint32_t tiles, uint32_t unroll, uint32_t variant, const LSeg* lseg,
                     const uint32_t* tile_tab, const uint64_t* key_in, const uint64_t* tree_lo,
                     const uint64_t* tree_in, const uint16_t* jump, uint16_t* bid, uint32_t* cm,
                     uint32_t vmax, uint32_t kmax, const Globals* glob, const Dyn& dy,
                     uint32_t redo, hipStream_t st);
// dig != 0: the columns of a digit of the bucket ids (two-pass distribution)
void launch_colscan(uint32_t chunks, uint32_t kmax, const LSeg* lseg, const uint32_t* chunk_tab,
                    uint32_t* cm, uint32_t* cs, const Globals* glob, const Dyn& dy, uint32_t redo,
                    hipStream_t st, uint32_t dig = 0);
// Two-pass distribution (host-driven): per-tile histograms of digit `dig`
// (kDigitLow / kDigitHigh) of the bucket ids in `bid`, and after the column
// scan the digits' starts added into the chunk prefixes.
void launch_digit_count(uint32_t tiles, const LSeg* lseg, const uint32_t* tile_tab,
                        const uint16_t* bid, uint32_t* cm, uint32_t dig, hipStream_t st);
void launch_digit_starts(uint32_t n_large, const LSeg* lseg, uint32_t* cs, uint32_t dig,
                         hipStream_t st);
// kmax: the most buckets of any segment of the pass (sizes the LDS)
void launch_bucket_plan(uint32_t n_large, const LSeg* lseg, uint32_t* cs, uint32_t* bstart,
                        const uint64_t* tree_in, const uint8_t* tree_lcp, const PlanCtx& ctx,
                        uint32_t next_buf, uint32_t kmax, const Dyn& dy, hipStream_t st);
void launch_scatter(uint32_t tiles, uint32_t unroll, const LSeg* lseg, const uint32_t* tile_tab,
                    const uint16_t* bid, const uint64_t* key_in, const uint64_t* key2_in,
                    const uint32_t* idx_in, uint64_t* key_out, uint64_t* key2_out,
                    uint32_t* idx_out, const uint32_t* cm, const uint32_t* cs,
                    const uint32_t* bstart, const uint64_t* tree_in, const uint8_t* tree_lcp,
                    const uint8_t* chars, const uint64_t* offsets, uint32_t* out_perm,
                    uint32_t* out_lcp, uint32_t vmax, uint32_t kmax, const Globals* glob,
                    const Dyn& dy, const uint64_t* key3, const KeyCodec& kc, hipStream_t st,
                    hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr,
                    uint32_t dig = 0, uint16_t* bid_out = nullptr);
// key2_0 / key2_1: the second key words of the two work buffers (exact or
// kKeyUnknown), which serve an item's first refinement round
void launch_base_sort(const uint32_t* n_items, Seg* const* items, const uint64_t* key0,
                      const uint64_t* key1, const uint64_t* key2_0, const uint64_t* key2_1,
                      const uint32_t* idx0, const uint32_t* idx1,
                      const uint8_t* chars, const uint64_t* offsets, uint32_t* out_perm,
                      uint32_t* out_lcp, uint32_t T, const Globals* glob, const Dyn* dy,
                      const uint32_t* guard, const KeyCodec& kc, hipStream_t st);
void launch_lcp_fix(const uint8_t* chars, const uint64_t* offsets, const uint64_t* set_begin,
                    uint32_t num_sets, uint32_t n, const uint32_t* out_perm, uint32_t* out_lcp,
                    const uint32_t* guard, const Globals* glob, hipStream_t st);
void launch_classify_plain(const uint64_t* keys, uint32_t n, const uint64_t* splitters,
                           uint32_t v, uint32_t d, uint32_t variant, uint64_t* tree_lo,
                           uint64_t* tree_in, uint16_t* jump, uint16_t* out, hipStream_t st);

// Counting of output writes for later sorts (the write-check build; returns
// false in the product build, where S5_OUT is a plain store).
bool set_write_count(const WriteCount& w);

size_t learn_bytes(uint32_t slots, uint32_t m);
LearnCtx learn_ctx(void* mem, uint32_t slots, uint32_t m);
void launch_learn_sort_trees(const LearnCtx& c, uint32_t slots, LSeg* lseg,
                             const uint32_t* learn_seg, const uint64_t* key_in, uint64_t seed,
                             uint32_t steps, float lr, float beta, Globals* glob,
                             uint64_t* tree_lo, uint64_t* tree_in, uint8_t* tree_lcp,
                             uint16_t* jump, const KeyCodec& kc, const Dyn& dy, hipStream_t st);
void launch_learn_check(uint32_t slots, LSeg* lseg, const uint32_t* learn_seg, const uint32_t* cs,
                        float beta, Globals* glob, const Dyn& dy, hipStream_t st);
void launch_mlp_train(const LearnCtx& c, const uint64_t* sorted_keys, uint32_t m, uint32_t steps,
                      float lr, uint64_t seed, float* out, hipStream_t st);
void launch_mlp_grad(const LearnCtx& c, const float* params, const uint64_t* sorted_keys,
                     uint32_t m, float* out, hipStream_t st);
void launch_mlp_propose(const float* params, const uint64_t* sorted_keys, uint32_t m, uint32_t v,
                        float beta, uint64_t* out_spl, float* out_y, uint32_t* out_reject,
                        hipStream_t st);
void launch_mlp_eval(const float* params, const uint64_t* keys, uint32_t n, uint64_t lo,
                     uint64_t hi, float* out, hipStream_t st);

}  // namespace s5
