/*
 * Measurement helper beside the solver's C ABI (not a step of the method):
 * the HBM bandwidth a plain streaming kernel reaches on the device, so that
 * the solver kernels' bandwidth can be reported against it as well as
 * against the device's peak.
 */
#ifndef JPCG_PROBE_H
#define JPCG_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * STREAM triad c[i] = a[i] + s * b[i] for i < n, FP64, on the given HIP
 * stream (NULL = the null stream), asynchronous.  a, b, c are device
 * pointers, 16-byte aligned; c may not overlap a or b.  grid = workgroups of
 * 256 threads (<= 0: 4096).  Moves 24 n bytes.  Returns 0, -1 for bad
 * arguments, -2 if the launch failed.
 */
int jpcg_stream_triad(const double *a, const double *b, double *c, double s, int64_t n, int32_t grid,
                      void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif
