/*
 * ag_probe.h -- measurement kernels used to calibrate the roofline of the
 * multirotor step (not part of the simulator's API).
 *
 * agp_valu_fma: every lane runs 8 independent FP32 FMA chains of `iters`
 *   steps (single, non-packed v_fma_f32), grid `blocks` x 256 threads; writes
 *   one float per thread to out (device, blocks*256 floats) so nothing is
 *   dead code.  FMA count = blocks * 256 * iters * 8.
 * agp_copy: plain vectorised device copy of `bytes` bytes (multiple of 16)
 *   from src to dst (device pointers, 16-byte aligned): reads and writes
 *   exactly `bytes` each; used to calibrate the HBM byte counters and to
 *   measure the achievable copy bandwidth.  `blocks` x 256 lanes walk the
 *   16-byte elements grid-stride; blocks = 0 launches one lane per element.
 * Both enqueue on `stream` (hipStream_t) and return 0, or a hipError_t code.
 */
#ifndef AG_PROBE_H
#define AG_PROBE_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif
int agp_valu_fma(void* stream, float* out, int32_t blocks, int32_t iters);
int agp_copy(void* stream, void* dst, const void* src, size_t bytes, int32_t blocks);
#ifdef __cplusplus
}
#endif
#endif
