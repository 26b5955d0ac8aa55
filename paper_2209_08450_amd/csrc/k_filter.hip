// Ramp filtering of detector rows by FFT (paper, Section 2.2: one-dimensional
// filtering with FFT plans built once and executed per chunk; padding to
// powers of two, Section 2.2 and the padding discussion of Section 3).
//
// One work-group filters two real rows at once as the real and imaginary parts
// of one complex sequence of length L held in LDS.  Because the ramp response
// H is real and even, IFFT(H . FFT(u1 + i u2)) = (h * u1) + i (h * u2): the two
// filtered rows come back in the real and imaginary parts with no unpacking.
// The inverse transform is a forward transform of the conjugate:
//   y = conj(FFT(conj(H . Z))) / L = conj(FFT(H . conj(Z))) / L   (H real),
// with 1/L folded into the H table.  The FFT is a Stockham radix-4 sweep
// (radix-2 first pass when log2 L is odd) with FP64-derived twiddles; every
// butterfly's four inputs are read into registers, the block synchronises,
// then the outputs are written in place.
//
// k_norm_filter fuses the dark/flat correction and -log: it reads raw uint16
// counts, normalises them in registers, filters in FP32 and writes only the
// filtered rows (storage precision); the -log sinogram never reaches HBM.
// Sign flips are written as 0 - x: the fneg form of a half-precision store
// trips an instruction-selection failure when packed FP32 is disabled.
#include "tp_internal.h"

namespace tp {
namespace {

constexpr float kMinTransmission = 1e-6f;
constexpr int kMaxPerThread4 = 4;  // radix-4 butterflies per thread (L / (4 B) with B = L / 16)
constexpr int kMaxPerThread2 = 8;  // radix-2 butterflies per thread

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// multiply by -i
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }

// In-place forward DFT X[k] = sum_m x[m] exp(-2 pi i k m / L) of buf[0..L).
// Caller must have synchronised after writing buf; returns synchronised.
__device__ void fft_forward_lds(float2* buf, int L, int log2L, const float2* __restrict__ tw) {
    const int tid = threadIdx.x;
    const int B = blockDim.x;
    int Ns = 1;
    if (log2L & 1) {
        const int h = L >> 1;
        float2 v0[kMaxPerThread2], v1[kMaxPerThread2];
#pragma unroll
        for (int c = 0; c < kMaxPerThread2; ++c) {
            const int j = tid + c * B;
            if (j < h) { v0[c] = buf[j]; v1[c] = buf[j + h]; }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < kMaxPerThread2; ++c) {
            const int j = tid + c * B;
            if (j < h) { buf[2 * j] = cadd(v0[c], v1[c]); buf[2 * j + 1] = csub(v0[c], v1[c]); }
        }
        __syncthreads();
        Ns = 2;
    }
    const int q = L >> 2;
    for (; Ns < L; Ns <<= 2) {
        const int tstride = L / (Ns << 2);
        float2 v[kMaxPerThread4][4];
#pragma unroll
        for (int c = 0; c < kMaxPerThread4; ++c) {
            const int j = tid + c * B;
            if (j < q) {
                const int k = j & (Ns - 1);
                const int t1 = k * tstride;
                float2 x0 = buf[j];
                float2 x1 = buf[j + q];
                float2 x2 = buf[j + 2 * q];
                float2 x3 = buf[j + 3 * q];
                if (Ns > 1) {
                    x1 = cmul(x1, tw[t1]);
                    x2 = cmul(x2, tw[(2 * t1) & (L - 1)]);
                    x3 = cmul(x3, tw[(3 * t1) & (L - 1)]);
                }
                const float2 a0 = cadd(x0, x2), a1 = csub(x0, x2);
                const float2 a2 = cadd(x1, x3), a3 = cmul_mi(csub(x1, x3));
                v[c][0] = cadd(a0, a2);
                v[c][1] = cadd(a1, a3);
                v[c][2] = csub(a0, a2);
                v[c][3] = csub(a1, a3);
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < kMaxPerThread4; ++c) {
            const int j = tid + c * B;
            if (j < q) {
                const int k = j & (Ns - 1);
                const int d = ((j - k) << 2) + k;
                buf[d] = v[c][0];
                buf[d + Ns] = v[c][1];
                buf[d + 2 * Ns] = v[c][2];
                buf[d + 3 * Ns] = v[c][3];
            }
        }
        __syncthreads();
    }
}

// Pad, filter, and leave y = IFFT(H . FFT(u)) in buf as (row0, row1) = (re, -im).
__device__ void filter_in_lds(float2* buf, int n, int off, const FilterTables& ft) {
    const int tid = threadIdx.x, B = blockDim.x, L = ft.L;
    // buf[off .. off+n) holds the rows; replicate the end values outward
    const float2 left = buf[off];
    const float2 right = buf[off + n - 1];
    for (int m = tid; m < L; m += B) {
        if (m < off) buf[m] = left;
        else if (m >= off + n) buf[m] = right;
    }
    __syncthreads();
    fft_forward_lds(buf, L, ft.log2L, ft.tw);
    for (int m = tid; m < L; m += B) {
        const float2 z = buf[m];
        const float h = ft.H[m];
        buf[m] = make_float2(z.x * h, -z.y * h);
    }
    __syncthreads();
    fft_forward_lds(buf, L, ft.log2L, ft.tw);
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(1024)
k_filter(const TI* in, TO* out, int64_t n_lines, int n, int off, FilterTables ft) {
    extern __shared__ float2 buf[];
    const int tid = threadIdx.x, B = blockDim.x;
    const int64_t l0 = 2 * static_cast<int64_t>(blockIdx.x);
    const bool has1 = l0 + 1 < n_lines;
    const int64_t b0 = l0 * n, b1 = (l0 + 1) * n;
    for (int j = tid; j < n; j += B) {
        const float a = load_as_float(in, b0 + j);
        const float b = has1 ? load_as_float(in, b1 + j) : 0.0f;
        buf[off + j] = make_float2(a, b);
    }
    __syncthreads();
    filter_in_lds(buf, n, off, ft);
    for (int j = tid; j < n; j += B) {
        const float2 y = buf[off + j];
        store_from_float(out, b0 + j, y.x);
        if (has1) store_from_float(out, b1 + j, 0.0f - y.y);
    }
}

// Rows (r, a) and (r, a + 1) of the chunk, a even; raw counts normalised in registers.
template <typename TO>
__global__ void __launch_bounds__(1024)
k_norm_filter(RawInput in, const float* __restrict__ dmean, const float* __restrict__ den, int n_angles,
              int n, int off, FilterTables ft, TO* out) {
    extern __shared__ float2 buf[];
    const int tid = threadIdx.x, B = blockDim.x;
    const int pairs = (n_angles + 1) >> 1;
    const int r = blockIdx.x / pairs;
    const int a0 = 2 * (blockIdx.x - r * pairs);
    const bool has1 = a0 + 1 < n_angles;
    const uint16_t* p0 = in.proj + a0 * in.proj_stride + static_cast<int64_t>(r) * n;
    const uint16_t* p1 = p0 + in.proj_stride;
    const float* dm = dmean + static_cast<int64_t>(r) * n;
    const float* dn = den + static_cast<int64_t>(r) * n;
    for (int j = tid; j < n; j += B) {
        const float d = dm[j], e = dn[j];
        const float t0 = fmaxf((static_cast<float>(p0[j]) - d) / e, kMinTransmission);
        float v1 = 0.0f;
        if (has1) v1 = 0.0f - logf(fmaxf((static_cast<float>(p1[j]) - d) / e, kMinTransmission));
        buf[off + j] = make_float2(0.0f - logf(t0), v1);
    }
    __syncthreads();
    filter_in_lds(buf, n, off, ft);
    TO* o0 = out + (static_cast<int64_t>(r) * n_angles + a0) * n;
    TO* o1 = o0 + n;
    for (int j = tid; j < n; j += B) {
        const float2 y = buf[off + j];
        store_from_float(o0, j, y.x);
        if (has1) store_from_float(o1, j, 0.0f - y.y);
    }
}

int filter_block(int L) {
    int b = L / 16;
    if (b < 64) b = 64;
    if (b > 1024) b = 1024;
    return b;
}

template <typename K>
hipError_t ensure_lds(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

template <typename TI, typename TO>
hipError_t launch_filter_t(const void* in, void* out, int64_t n_lines, int n, const FilterTables& ft,
                           hipStream_t st) {
    const size_t lds = static_cast<size_t>(ft.L) * sizeof(float2);
    hipError_t e = ensure_lds(k_filter<TI, TO>, lds);
    if (e != hipSuccess) return e;
    const int off = (ft.L - n) / 2;
    const int64_t blocks = (n_lines + 1) / 2;
    hipLaunchKernelGGL((k_filter<TI, TO>), dim3(static_cast<unsigned>(blocks)), dim3(filter_block(ft.L)),
                       lds, st, static_cast<const TI*>(in), static_cast<TO*>(out), n_lines, n, off, ft);
    return hipGetLastError();
}

template <typename TI>
hipError_t launch_filter_in(const void* in, tp_dtype out_dt, void* out, int64_t n_lines, int n,
                            const FilterTables& ft, hipStream_t st) {
    switch (out_dt) {
        case TP_F32: return launch_filter_t<TI, float>(in, out, n_lines, n, ft, st);
        case TP_F16: return launch_filter_t<TI, __half>(in, out, n_lines, n, ft, st);
        case TP_BF16: return launch_filter_t<TI, uint16_t>(in, out, n_lines, n, ft, st);
    }
    return hipErrorInvalidValue;
}

template <typename TO>
hipError_t launch_norm_filter_t(const RawInput& in, const float* dmean, const float* den, int n_angles,
                                int n_rows, int n, const FilterTables& ft, void* out, hipStream_t st) {
    const size_t lds = static_cast<size_t>(ft.L) * sizeof(float2);
    hipError_t e = ensure_lds(k_norm_filter<TO>, lds);
    if (e != hipSuccess) return e;
    const int off = (ft.L - n) / 2;
    const int64_t blocks = static_cast<int64_t>(n_rows) * ((n_angles + 1) / 2);
    hipLaunchKernelGGL((k_norm_filter<TO>), dim3(static_cast<unsigned>(blocks)), dim3(filter_block(ft.L)),
                       lds, st, in, dmean, den, n_angles, n, off, ft, static_cast<TO*>(out));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_filter(const void* in, tp_dtype in_dt, void* out, tp_dtype out_dt, int64_t n_lines,
                         int n_det, const FilterTables& ft, hipStream_t st) {
    switch (in_dt) {
        case TP_F32: return launch_filter_in<float>(in, out_dt, out, n_lines, n_det, ft, st);
        case TP_F16: return launch_filter_in<__half>(in, out_dt, out, n_lines, n_det, ft, st);
        case TP_BF16: return launch_filter_in<uint16_t>(in, out_dt, out, n_lines, n_det, ft, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_norm_filter(const RawInput& in, const float* dmean, const float* den, int n_angles,
                              int n_rows, int n_det, const FilterTables& ft, tp_dtype out_dt, void* out,
                              hipStream_t st) {
    switch (out_dt) {
        case TP_F32: return launch_norm_filter_t<float>(in, dmean, den, n_angles, n_rows, n_det, ft, out, st);
        case TP_F16: return launch_norm_filter_t<__half>(in, dmean, den, n_angles, n_rows, n_det, ft, out, st);
        case TP_BF16:
            return launch_norm_filter_t<uint16_t>(in, dmean, den, n_angles, n_rows, n_det, ft, out, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace tp
