/*
 * bspline_probe.h - measurement helper exported by libbspline.so beside the
 * evaluator (bspline.h).  It is not part of the method: it measures the
 * memory ceiling that the evaluation kernels are set against, with the
 * read/write mix of their roofline (paper, section "Performance Summary and
 * Roofline analysis": 64 coefficient reads and 10 output writes per VGH
 * orbital-eval, i.e. 256 bytes read and 40 bytes written on an FP32 table).
 */
#ifndef BSPLINE_PROBE_H
#define BSPLINE_PROBE_H

#include <stdint.h>

#include "bspline.h"

#ifdef __cplusplus
extern "C" {
#endif

#define BSPL_PROBE_NT_STORES 0x1 /* non-temporal stores of the written words */
#define BSPL_PROBE_CHUNKED 0x2   /* the six words of a wavefront's 64 units form
                                    one contiguous 6 KiB span (else six planes) */
#define BSPL_PROBE_RANDOM 0x4    /* chunked, each wavefront's span drawn at random
                                    (counter hash of its index and salt; spans
                                    repeat and are skipped as random gathers do) */

/* Streaming kernel with 6 reads per write (85.7 % of the bytes read).
 *  src: device buffer of 6 * units 16-byte words (units a multiple of 64
 *       when chunked or random), read once each unless random;
 *  dst: device buffer of units 16-byte words, written once each (the sum of
 *       the six words of its unit, so no read can be skipped);
 *  per_lane: units in flight per lane, 1, 2 or 4;
 *  grid: persistent workgroups of 256 lanes, or 0 for units / per_lane
 *        lanes (each unit handled once, no striding);
 *  flags: any of BSPL_PROBE_NT_STORES, BSPL_PROBE_CHUNKED, BSPL_PROBE_RANDOM;
 *  salt: seeds the random spans (vary it between calls so that successive
 *        calls read different spans, as successive position batches do).
 * Moves 112 * units bytes (96 read, 16 written per unit, counted as requested
 * even where a random span repeats).  The caller owns
 * both buffers; asynchronous on the stream.  EINVAL for units < 0, grid < 0,
 * a bad per_lane or flags, a chunked units count not a multiple of 64, or
 * NULL buffers while units > 0; EUNSUPPORTED
 * when the byte count overflows; EDEVICE if the launch fails.             */
bspl_status spline_stream_probe(const void* src, void* dst, int64_t units, int32_t per_lane,
                                int32_t grid, int32_t flags, uint64_t salt, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* BSPLINE_PROBE_H */
