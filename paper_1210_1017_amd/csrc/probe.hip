// Machine probes: the vector-ALU and HBM ceilings that the interaction and
// the streaming kernels of the step are read against, measured on the GPU
// that runs them instead of taken from a datasheet alone.
#include "sph_internal.h"

namespace sph {

// 8 independent FP32 FMA chains per lane (enough in flight to hide the FMA
// latency with a few waves per SIMD). The build has packed FP32 switched
// off, so each is one v_fma_f32: 2 FLOP per lane per instruction.
__global__ __launch_bounds__(256) void k_probe_fma(float *__restrict__ out, int iters, float b,
                                                   float c) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    float a0 = 1e-3f * (float)threadIdx.x, a1 = a0 + 0.125f, a2 = a0 + 0.25f, a3 = a0 + 0.375f;
    float a4 = a0 + 0.5f, a5 = a0 + 0.625f, a6 = a0 + 0.75f, a7 = a0 + 0.875f;
#pragma unroll 4
    for (int i = 0; i < iters; i++) {
        a0 = fmaf(a0, b, c);
        a1 = fmaf(a1, b, c);
        a2 = fmaf(a2, b, c);
        a3 = fmaf(a3, b, c);
        a4 = fmaf(a4, b, c);
        a5 = fmaf(a5, b, c);
        a6 = fmaf(a6, b, c);
        a7 = fmaf(a7, b, c);
    }
    out[t] = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
}

// Streaming copy with 16-byte loads and stores: each lane moves 4 vectors
// per pass (all 4 loads issued before the stores), grid-stride over passes;
// the tail (fewer than 4 vectors per lane of a pass) takes the bounds test.
__global__ __launch_bounds__(256) void k_probe_copy(const float4 *__restrict__ src,
                                                    float4 *__restrict__ dst, uint64_t n16) {
    const uint64_t lanes = (uint64_t)gridDim.x * 256u;
    for (uint64_t k = (uint64_t)blockIdx.x * 256u + threadIdx.x; k < n16; k += 4 * lanes) {
        float4 v[4];
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (k + u * lanes < n16) v[u] = src[k + u * lanes];
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (k + u * lanes < n16) dst[k + u * lanes] = v[u];
    }
}

hipError_t launch_probe_fma(float *out, uint32_t blocks, int iters, hipStream_t s) {
    hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(256), 0, s, out, iters, 0.99999988f, 1e-7f);
    return hipGetLastError();
}

hipError_t launch_probe_copy(const void *src, void *dst, uint64_t bytes, uint32_t blocks,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, s, (const float4 *)src,
                       (float4 *)dst, bytes / 16);
    return hipGetLastError();
}

}  // namespace sph
