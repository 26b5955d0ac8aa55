// Measurement instruments for the roofline denominators (not part of the
// reconstruction): a device copy for the HBM rate, independent FP32 FMAs and
// FP16 dot products for the VALU issue rates, and conflict-free 16-byte LDS
// reads for the LDS read rate, all built with the same flags as every other
// kernel here (packed FP32 disabled: one v_fma_f32 per lane and instruction).
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

// Each lane runs kChains independent multiply-add chains for `iters` steps;
// the chains' instructions of one step are independent of each other, so
// the issue is never held up by a result, only by the SIMD's rate.  One sum
// is stored so nothing is dead code.  Forms (tp_valu_form):
//   FMA_F32       v_fma_f32, all operands VGPRs (the backprojectors' form)
//   FMA_F32_SGPR  v_fma_f32 reading its coefficient from a scalar register
//   FMA_MIX_F16   v_fma_mix_f32: an FP16 operand widened inside the FMA
//   DOT2_F16      v_dot2_f32_f16: two FP16 products added to an FP32 sum
constexpr int kChains = 16;
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

template <int FORM>
__global__ void __launch_bounds__(256) k_peak_valu(float* __restrict__ out, int iters, float a, float b) {
    float acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = static_cast<float>(threadIdx.x + c);
    float va = a, vb = b;
    half2_t x = {static_cast<_Float16>(a), static_cast<_Float16>(b)};
    half2_t y = {static_cast<_Float16>(b), static_cast<_Float16>(a)};
    if constexpr (FORM != TP_VALU_FMA_F32_SGPR) asm volatile("" : "+v"(va), "+v"(vb), "+v"(x), "+v"(y));
#pragma unroll 8
    for (int it = 0; it < iters; ++it) {
        // an opaque FP16 operand each step, so its widening stays inside the FMA
        if constexpr (FORM == TP_VALU_FMA_MIX_F16) asm volatile("" : "+v"(x));
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if constexpr (FORM == TP_VALU_FMA_F32 || FORM == TP_VALU_FMA_F32_SGPR) {
                acc[c] = __builtin_fmaf(va, vb, acc[c]);
            } else if constexpr (FORM == TP_VALU_FMA_MIX_F16) {
                acc[c] = __builtin_fmaf(static_cast<float>(x.x), vb, acc[c]);
            } else {
                acc[c] = __builtin_amdgcn_fdot2(x, y, acc[c], false);
            }
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c];
    out[static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

// LDS read rate: each thread issues kLdsReads 16-byte reads per step from a
// 16 KiB buffer, lanes of a wave on consecutive 16-byte words (no bank
// conflicts), XOR-folding the words so the reads are live.
constexpr int kLdsWords = 1024;
constexpr int kLdsReads = 16;
__global__ void __launch_bounds__(256) k_peak_lds(uint32_t* __restrict__ out, int iters) {
    __shared__ uint4 buf[kLdsWords];
    const int t = threadIdx.x;
    for (int i = t; i < kLdsWords; i += 256) buf[i] = make_uint4(i, 3 * i, 5 * i, 7 * i);
    __syncthreads();
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    int idx = t;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kLdsReads; ++u) {
            const uint4 v = buf[(idx + 64 * u) & (kLdsWords - 1)];
            acc.x ^= v.x;
            acc.y ^= v.y;
            acc.z ^= v.z;
            acc.w ^= v.w;
        }
        idx = (idx + 7) & (kLdsWords - 1);
    }
    out[static_cast<int64_t>(blockIdx.x) * blockDim.x + t] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

}  // namespace

hipError_t launch_peak_copy(const void* src, void* dst, int64_t bytes, hipStream_t st) {
    const int64_t n16 = bytes / 16;
    const int64_t blocks = std::min<int64_t>((n16 + 255) / 256, 256 * 64);
    hipLaunchKernelGGL(k_peak_copy, dim3(static_cast<unsigned>(std::max<int64_t>(blocks, 1))), dim3(256), 0, st,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
    return hipGetLastError();
}

int64_t peak_valu_flop(int form, int blocks, int iters) {
    return static_cast<int64_t>(blocks) * 256 * iters * kChains * (form == TP_VALU_DOT2_F16 ? 4 : 2);
}

hipError_t launch_peak_valu(int form, float* out, int blocks, int iters, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>(blocks));
    switch (form) {
        case TP_VALU_FMA_F32:
            hipLaunchKernelGGL(k_peak_valu<TP_VALU_FMA_F32>, grid, dim3(256), 0, st, out, iters, 0.5f, 0.25f);
            break;
        case TP_VALU_FMA_F32_SGPR:
            hipLaunchKernelGGL(k_peak_valu<TP_VALU_FMA_F32_SGPR>, grid, dim3(256), 0, st, out, iters, 0.5f, 0.25f);
            break;
        case TP_VALU_FMA_MIX_F16:
            hipLaunchKernelGGL(k_peak_valu<TP_VALU_FMA_MIX_F16>, grid, dim3(256), 0, st, out, iters, 0.5f, 0.25f);
            break;
        case TP_VALU_DOT2_F16:
            hipLaunchKernelGGL(k_peak_valu<TP_VALU_DOT2_F16>, grid, dim3(256), 0, st, out, iters, 0.5f, 0.25f);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int64_t peak_lds_bytes(int blocks, int iters) {
    return static_cast<int64_t>(blocks) * 256 * iters * kLdsReads * 16;
}

hipError_t launch_peak_lds(uint32_t* out, int blocks, int iters, hipStream_t st) {
    hipLaunchKernelGGL(k_peak_lds, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, out, iters);
    return hipGetLastError();
}

}  // namespace tp
