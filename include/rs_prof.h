/*
 * rs_prof.h -- per-kernel timing of librs.so (diagnostics, not part of the
 * sort itself).
 *
 * While enabled, every kernel the library launches is bracketed by two HIP
 * events recorded on the stream the kernel is launched on, so the measured
 * durations are those of the kernels in the caller's own stream order.
 * Recording is per process; calls from several threads are serialised by
 * an internal lock.  Disabled by default: then no event is recorded.
 */
#ifndef RS_PROF_H
#define RS_PROF_H

#include <stdint.h>

#include "rs.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Starts (enable != 0) or stops recording.  Starting discards earlier
 * records. */
rs_status rs_prof_enable(int enable);

/* Waits for the recorded events and returns, for kernel `name` (for example
 * "rs_rank_scatter"), the number of launches and their summed duration in
 * milliseconds.  An unknown name gives 0 launches. */
rs_status rs_prof_query(const char *name, uint64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* RS_PROF_H */
