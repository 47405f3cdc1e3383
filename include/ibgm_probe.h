/*
 * ibgm_probe.h -- measurement aid of libibgm.so: the streaming rate a plain
 * hand-written kernel reaches on this GPU, the practical ceiling against
 * which the bandwidth-bound kernels of the IB-GM step are read (the vendor's
 * peak is not reachable by streaming code).  Not part of the method.
 */
#ifndef IBGM_PROBE_H
#define IBGM_PROBE_H

#include <stdint.h>

#include "ibgm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Read the nsrc device arrays src[q] and write the ndst device arrays
 * dst[q] (FP32, n elements each, n a multiple of 4, 16-byte aligned, at most
 * 12 of each) `reps` times with one elementwise kernel (16-byte loads and
 * stores, grid-stride), on hip_stream, timed with HIP events after one
 * warm-up launch; *bytes_per_s (host) = (nsrc + ndst) 4 n reps / time.
 * Synchronises.  Arrays larger than the GPU's last-level cache (256 MB on
 * MI355X) give the HBM rate. */
ib_status ib_probe_stream_rate(const float *const *src, int32_t nsrc, float *const *dst,
                               int32_t ndst, int64_t n, int32_t reps, void *hip_stream,
                               double *bytes_per_s);

#ifdef __cplusplus
}
#endif
#endif
