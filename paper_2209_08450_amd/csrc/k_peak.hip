// Measurement instruments for the roofline denominators (not part of the
// reconstruction): a device copy for the HBM rate and a chain of
// independent FP32 FMAs for the VALU issue rate, both built with the same
// flags as every other kernel here (packed FP32 disabled, so the FMA loop
// issues one v_fma_f32 per lane and instruction, as the backprojector does).
#include <algorithm>

#include "tp_internal.h"

namespace tp {
namespace {

// Grid-stride copy of n16 16-byte elements.
__global__ void __launch_bounds__(256) k_peak_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                   int64_t n16) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

// Each lane runs kChains independent FMA chains for `iters` steps (8 FMAs per
// step and chain group), then stores one sum so nothing is dead code.
constexpr int kChains = 8;
__global__ void __launch_bounds__(256) k_peak_fma(float* __restrict__ out, int iters, float a, float b) {
    float acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = static_cast<float>(threadIdx.x + c);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = __builtin_fmaf(acc[c], a, b);
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = __builtin_fmaf(acc[c], b, a);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c];
    out[static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

}  // namespace

hipError_t launch_peak_copy(const void* src, void* dst, int64_t bytes, hipStream_t st) {
    const int64_t n16 = bytes / 16;
    const int64_t blocks = std::min<int64_t>((n16 + 255) / 256, 256 * 64);
    hipLaunchKernelGGL(k_peak_copy, dim3(static_cast<unsigned>(std::max<int64_t>(blocks, 1))), dim3(256), 0, st,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
    return hipGetLastError();
}

int64_t peak_fma_flop(int blocks, int iters) {
    return static_cast<int64_t>(blocks) * 256 * iters * 2 * kChains * 2;
}

hipError_t launch_peak_fma(float* out, int blocks, int iters, hipStream_t st) {
    hipLaunchKernelGGL(k_peak_fma, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, out, iters, 0.999f,
                       1e-3f);
    return hipGetLastError();
}

}  // namespace tp
