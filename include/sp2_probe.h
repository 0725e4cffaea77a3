/* sp2_probe.h — measurement helper beside the solver library (libsp2_probe.so).
 *
 * Not part of the density-matrix solver.  It runs the layer product's matrix
 * instruction sequence with no memory traffic, so that the rate the matrix
 * cores reach on this GPU under its power limit, for operands of given
 * statistics, can be measured next to the layer kernel's.
 */
#ifndef SP2_PROBE_H
#define SP2_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Every work-group (256 threads, one wave per SIMD, as in the layer kernel)
 * loads two K steps of hi/lo fragments of a 256 x 256 tile's row panels
 * from the K-tiled planes `hi`, `lo` (device, np x np, the layout sp2_split
 * writes for np a multiple of 256), then issues `iters` times, for each of
 * the two K steps, the layer kernel's 48 matrix instructions per wave
 * (hi*hi, hi*lo, lo*hi over a 4 x 4 block of 32 x 32 accumulators) on those
 * register-resident fragments: 2 * 48 * 32768 * 2 flop per wave and
 * iteration.  `precision`: SP2_BF16X3 (2) or SP2_FP16X3 (3).  Work-group b
 * reads panels b % (np / 256) and (b / (np / 256)) % (np / 256).
 *
 * sink: device, nblocks * 256 floats (one value per thread, so that the
 *   products are not optimised away).
 * clocks: device, 4 * nblocks uint64: per work-group the shader clock
 *   counter and the constant-rate wall clock at the start and at the end of
 *   its loop (clock0, wall0, clock1, wall1).
 * wall_hz: host, receives the wall clock's rate in Hz (may be NULL).
 * Returns 0, 1 for an invalid argument (nothing launched), 5 when the launch
 * fails.  Asynchronous on `stream` (a hipStream_t, NULL: the null stream). */
int32_t sp2_probe_mfma(const uint16_t* hi, const uint16_t* lo, int64_t np, int32_t precision,
                       int32_t iters, int32_t nblocks, float* sink, uint64_t* clocks,
                       double* wall_hz, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SP2_PROBE_H */
