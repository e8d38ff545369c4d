/*
 * lbtp_probe.h -- measurement helper of liblbtp, not part of the method.
 *
 * lbtp_copy_probe copies `bytes` bytes (a multiple of 16, both pointers
 * 16-byte aligned device memory) from src to dst with a plain streaming
 * kernel on `stream` (hipStream_t, NULL = null stream), asynchronously.  Its
 * only use is as the known-size reference that calibrates the HBM byte
 * counters (FETCH_SIZE, WRITE_SIZE) of a profiler run: the counter value of
 * the probe divided into its true byte count gives the scale that converts
 * the counters of the sweep kernels into bytes.  Returns LBTP_EINVAL for a
 * bad size or alignment, LBTP_EHIP if the launch fails.
 */
#ifndef LBTP_PROBE_H
#define LBTP_PROBE_H

#include "lbtp.h"

#ifdef __cplusplus
extern "C" {
#endif

LBTP_API int lbtp_copy_probe(void *dst, const void *src, long long bytes, void *stream);

/* Timing aid for the dominant kernel: enqueue `launches` launches of the
 * plain pressure sweep on the context's stream, each running sweep_block
 * sweeps (eq. 3-1; one when blocking is off), continuing the current
 * pressure state without re-basing or evaluating the stopping rule, so the
 * launches can be timed back to back.  The state afterwards is that of
 * launches x sweep_block more plain sweeps.  Needs a pressure solve since the
 * last lbtp_set_state / lbtp_put_state (LBTP_ESTATE otherwise), launches >= 0
 * (LBTP_EINVAL otherwise).  Returns the sweeps per launch (> 0) or an error. */
LBTP_API int lbtp_probe_sweeps(lbtp_ctx *ctx, long long launches);

#ifdef __cplusplus
}
#endif
#endif /* LBTP_PROBE_H */
