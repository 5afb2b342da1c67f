/*
 * bgv_profile.h -- optional per-kernel timing of libbgv launches.
 *
 * When enabled, kernel launches of the library carry a start and a stop HIP event that
 * the launch itself records (hipExtLaunchKernelGGL on the kernel's stream), so the
 * events hold the kernel's own execution interval, and a caller can obtain the average
 * device duration of each kernel over a region of its own.  Disabled by default.  Not
 * thread-safe across concurrent callers of enable/reset.
 */
#ifndef BGV_PROFILE_H
#define BGV_PROFILE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Start (on != 0) or stop recording events around library kernel launches. */
void bgv_profile_enable(int on);
/* Record only launches of kernels whose name starts with prefix (e.g. "k_bh_force"),
 * so that a timed region carries the events of the kernel under study alone.  NULL or
 * "" records every kernel (the default).  Takes effect for later launches. */
void bgv_profile_filter(const char *prefix);
/* Record one in `every` of the launches that pass the filter (the first, then every
 * every-th), so long runs are sampled with a fraction of the event overhead; 1 or less
 * records all (the default).  Statistics count the recorded launches only. */
void bgv_profile_sample(int every);
/* Forget every recorded launch. */
void bgv_profile_reset(void);
/* Number of distinct kernels recorded since the last reset.  Waits for the recorded
 * events to complete (host synchronisation on them). */
int bgv_profile_count(void);
/* Kernel idx in [0, count): its name (static storage until the next reset), number
 * of launches and summed device time in milliseconds.  Returns 0, or -1 if idx is out
 * of range. */
int bgv_profile_get(int idx, const char **name, int64_t *launches, double *total_ms);
/* Device-side work counters accumulated while profiling is enabled (reset by
 * bgv_profile_reset).  "bh_interactions": number of Barnes-Hut force terms summed
 * (body-body pairs plus body-cell centre-of-mass terms) over all layout iterations.
 * "bh_redo_blocks": Barnes-Hut force workgroups (8 bodies each) whose walk outgrew
 * the short per-body stack of the first launch and were redone with the full one
 * (counted whether or not profiling is enabled).  Synchronises the device.  Returns 0, or -1 for an unknown name or a HIP error. */
int bgv_profile_counter(const char *name, uint64_t *value);

#ifdef __cplusplus
}
#endif
#endif /* BGV_PROFILE_H */
