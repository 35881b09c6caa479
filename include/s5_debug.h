/*
 * s5_debug.h -- test hooks of the S^5 library (same conventions as s5.h).
 * They exist so that tests can reach the library's error paths and check its
 * output writes; a production caller never needs them.
 */
#ifndef S5_DEBUG_H
#define S5_DEBUG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* device-side capacities that s5_debug_limit_capacity can shrink */
#define S5_CAP_LARGE 0u  /* segments distributed in one pass */
#define S5_CAP_BASE0 1u  /* base-case items of <= 64 strings */
#define S5_CAP_BASE3 4u  /* base-case items of 513..T strings */

/* Limit capacity `which` to at most `limit` entries for the sorts that follow
 * (limit 0 removes the limit).  The device's planner then finds the capacity
 * exhausted on inputs that need more, sets its status word and every later
 * kernel of the sort exits without work; the sort returns S5_ERR_DEVICE.
 * Drops the cached graphs of batched sorts.  Returns S5_OK or
 * S5_ERR_INVALID (unknown `which`). */
int s5_debug_limit_capacity(uint32_t which, uint32_t limit);

/* Count the writes of the sorts that follow into the output arrays perm and
 * lcp (DEVICE pointers of n entries each; the sort must be given these same
 * outputs): perm_counts[i] / lcp_counts[i] (DEVICE, n uint32 each, zeroed by
 * the caller) are incremented at every write of out_perm[i] / out_lcp[i], and
 * *stray (DEVICE, one uint32) at every output write that lands in neither
 * array.  perm_counts = NULL stops counting.  Only the write-check build of
 * the library (libs5_wcheck.so) counts; the product build returns
 * S5_ERR_INVALID.  Counting costs one atomic per output write. */
int s5_debug_count_writes(uint32_t* perm, uint32_t* lcp, uint64_t n, uint32_t* perm_counts,
                          uint32_t* lcp_counts, uint32_t* stray);

/* With on != 0, the sorts that follow publish their per-level counters into
 * a word next to the flag the host polls, so the flag never shows them: every
 * read-back then takes its fallback path (after 2 ms the host finds the
 * stream drained and copies the counters).  on = 0 restores publication.
 * Returns S5_OK. */
int s5_debug_miss_publish(int on);

#ifdef __cplusplus
}
#endif

#endif /* S5_DEBUG_H */
