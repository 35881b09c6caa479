/*
 * s5_profile.h -- per-kernel timing of the S^5 library's own launches.
 *
 * For roofline reporting: while profiling is enabled, every kernel launch of
 * a sort is bracketed by two HIP events recorded on the stream the kernel is
 * launched on (for the redistribution kernel the dispatch itself stamps the
 * two events, hipExtLaunchKernel, so their interval is the kernel's
 * execution; the device still idles a few microseconds around each timed
 * launch while the events are processed); after the sort completes the elapsed
 * times are accumulated per kernel together with the strings the launch
 * processed and the algorithmic bytes that implies (the per-string byte
 * counts of each step, e.g. 24 bytes of (key, index) read and written per
 * string by a redistribution pass, Section 3.1 "Parallelization":
 * out-of-place redistribution).
 * Instrumentation only: it changes no result.  Process-wide, not thread-safe
 * with respect to concurrent sorts.
 */
#ifndef S5_PROFILE_H
#define S5_PROFILE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct s5_kernel_profile {
    char name[32];      /* kernel name, e.g. "scatter" */
    uint64_t launches;  /* launches accumulated */
    double total_ms;    /* sum of launch durations (HIP events) */
    uint64_t items;     /* strings processed, summed over launches */
    double alg_bytes;   /* algorithmic bytes, summed over launches */
} s5_kernel_profile;

/* Enable (on != 0) or disable profiling; either way the accumulators are
 * cleared.  Returns S5_OK. */
int s5_profile_enable(int on);

/* Restrict the event timing to the launches of one kernel (a name as
 * reported by s5_profile_read, e.g. "scatter"), so that the events themselves
 * add little to a timed sort; NULL or "" times every kernel again.  Returns
 * S5_OK, or S5_ERR_INVALID for an unknown name. */
int s5_profile_only(const char* kernel);

/* Copy up to `max` kernel entries to `out` (host memory); *count receives the
 * number of kernels with at least one launch.  Returns S5_OK or
 * S5_ERR_INVALID for a NULL pointer. */
int s5_profile_read(s5_kernel_profile* out, uint32_t max, uint32_t* count);

#ifdef __cplusplus
}
#endif

#endif /* S5_PROFILE_H */
