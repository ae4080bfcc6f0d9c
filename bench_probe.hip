// bench_probe.hip -- calibration kernels for the benchmark's roofline (not
// part of the simulator library).
//
// agp_valu_fma: every lane runs 8 independent FP32 FMA chains of `iters`
//   steps (single, non-packed v_fma_f32), grid `blocks` x 256 threads; writes
//   one float per thread to out (device, blocks*256 floats) so nothing is
//   dead code.  FMA count = blocks * 256 * iters * 8.
// agp_copy: plain vectorised device copy of `bytes` bytes (multiple of 16)
//   from src to dst (device pointers, 16-byte aligned): reads and writes
//   exactly `bytes` each; used to calibrate the HBM byte counters and to
//   measure the achievable copy bandwidth.  `blocks` x 256 lanes walk the
//   16-byte elements grid-stride; blocks = 0 launches one lane per element.
// Both enqueue on `stream` (hipStream_t) and return 0, or a hipError_t code.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace {

__global__ __launch_bounds__(256) void k_valu_fma(float* out, int iters) {
    const float b = 0.999999f, c = 1.0e-7f;
    float a0 = threadIdx.x * 1e-3f, a1 = a0 + 1.0f, a2 = a0 + 2.0f, a3 = a0 + 3.0f;
    float a4 = a0 + 4.0f, a5 = a0 + 5.0f, a6 = a0 + 6.0f, a7 = a0 + 7.0f;
    for (int i = 0; i < iters; ++i) {
        a0 = __builtin_fmaf(a0, b, c); a1 = __builtin_fmaf(a1, b, c);
        a2 = __builtin_fmaf(a2, b, c); a3 = __builtin_fmaf(a3, b, c);
        a4 = __builtin_fmaf(a4, b, c); a5 = __builtin_fmaf(a5, b, c);
        a6 = __builtin_fmaf(a6, b, c); a7 = __builtin_fmaf(a7, b, c);
    }
    out[blockIdx.x * 256 + threadIdx.x] = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
}

// Plain copy, one 16-byte element per lane and grid-stride step.
__global__ __launch_bounds__(256) void k_copy(float4* __restrict__ dst, const float4* __restrict__ src, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

}  // namespace

extern "C" int agp_valu_fma(void* stream, float* out, int32_t blocks, int32_t iters) {
    if (!out || blocks < 1 || iters < 1) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_valu_fma, dim3(blocks), dim3(256), 0, (hipStream_t)stream, out, iters);
    return (int)hipGetLastError();
}

extern "C" int agp_copy(void* stream, void* dst, const void* src, size_t bytes, int32_t blocks_in) {
    if (!dst || !src || bytes % 16 || blocks_in < 0) return (int)hipErrorInvalidValue;
    const size_t n = bytes / 16;
    const size_t one_each = (n + 255) / 256;          // blocks for one element per lane
    size_t nb = blocks_in > 0 ? (size_t)blocks_in : one_each;
    if (nb > one_each) nb = one_each;
    if (nb < 1) nb = 1;
    if (nb > 0x7fffffffu) return (int)hipErrorInvalidValue;
    const unsigned blocks = (unsigned)nb;
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (float4*)dst, (const float4*)src, n);
    return (int)hipGetLastError();
}
