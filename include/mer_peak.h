/*
 * mer_peak.h -- reference kernels for the rooflines of the micro-edge
 * library (libmer_peak.so, separate from libmer.so): the bandwidth a plain
 * streaming copy reaches, and the rate of device-scope float atomic adds.
 * The micro-edge method itself (Sec. 4.2, last paragraph) scatters its
 * per-pixel gradients to shared vertices, which on a GPU means float atomics
 * into the vertex and attribute gradient buffers; these kernels measure what
 * the chip does for that pattern without the method around it.
 *
 * Conventions: device pointers owned by the caller; work is enqueued on
 * `stream` (a hipStream_t, NULL = null stream) and the call returns without
 * waiting; 0 on success, -1 on a bad argument (nothing enqueued), -3 if the
 * launch failed.
 */
#ifndef MER_PEAK_H
#define MER_PEAK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* dst[i] = src[i] for i < n_floats; n_floats a positive multiple of 4, both
 * pointers 16-byte aligned.  Reads and writes 4 n_floats bytes each. */
int mer_peak_copy(const float *src, float *dst, int64_t n_floats, void *stream);

/* lanes * per_lane float atomic adds of 1.0f into buf[0, footprint): lane i
 * adds into element (i + r * lanes) mod footprint, r = 0 .. per_lane - 1, so
 * each wave adds to 64 consecutive floats at a time.  lanes a positive
 * multiple of 256 (one workgroup of 256 per 256 lanes).  buf is
 * accumulated; the caller clears it. */
int mer_peak_atomic_add(float *buf, int64_t footprint, int64_t lanes, int per_lane, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MER_PEAK_H */
