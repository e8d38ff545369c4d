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

#ifdef __cplusplus
}
#endif
#endif /* LBTP_PROBE_H */
