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
#include "fft_device.h"

namespace tp {
namespace {

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
        const float v0 = neglog_counts(static_cast<float>(p0[j]), d, e);
        const float v1 = has1 ? neglog_counts(static_cast<float>(p1[j]), d, e) : 0.0f;
        buf[off + j] = make_float2(v0, v1);
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

// Multiply the spectrum by H/L and conjugate, transform again: slots then hold
// y = conj of (IFFT(H . FFT(u)) * L) / L, i.e. (row0, -row1).
template <int L>
__device__ __forceinline__ void reg_filter(float2 (&x)[kRegPts], float2* lds, const FilterTables& ft, int t) {
    constexpr int B = L / kRegPts;
    reg_fft<L>(x, lds, ft.tw, t);
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) {
        const float h = ft.H[t + B * s];
        x[s] = make_float2(x[s].x * h, 0.0f - x[s].y * h);
    }
    // no barrier needed: the forward transform's last LDS reads were followed
    // by one, and its last pass ran in registers
    reg_fft<L>(x, lds, ft.tw, t);
}

template <int L, typename TI, typename TO>
__global__ void __launch_bounds__(L / kRegPts)
k_filter_reg(const TI* in, TO* out, int64_t n_lines, int n, int off, FilterTables ft) {
    extern __shared__ float2 lds[];
    constexpr int B = L / kRegPts;
    const int t = threadIdx.x;
    const int64_t l0 = 2 * static_cast<int64_t>(blockIdx.x);
    const bool has1 = l0 + 1 < n_lines;
    const TI* r0 = in + l0 * n;
    const TI* r1 = r0 + n;
    const float e00 = load_as_float(r0, 0), e01 = load_as_float(r0, n - 1);
    const float e10 = has1 ? load_as_float(r1, 0) : 0.0f, e11 = has1 ? load_as_float(r1, n - 1) : 0.0f;
    float2 x[kRegPts];
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) {
        const int j = t + B * s - off;
        if (j < 0) x[s] = make_float2(e00, e10);
        else if (j >= n) x[s] = make_float2(e01, e11);
        else x[s] = make_float2(load_as_float(r0, j), has1 ? load_as_float(r1, j) : 0.0f);
    }
    reg_filter<L>(x, lds, ft, t);
    TO* o0 = out + l0 * n;
    TO* o1 = o0 + n;
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) {
        const int j = t + B * s - off;
        if (j >= 0 && j < n) {
            store_from_float(o0, j, x[s].x);
            if (has1) store_from_float(o1, j, 0.0f - x[s].y);
        }
    }
}


// Angle pairs per work-group of the fused kernel: each pair's raw counts are
// prefetched into registers while the previous pair is transformed.
constexpr int kPairsPerGroup = 8;

// HALF: the detector fills the middle half of the padded row (n = L/2, off =
// L/4, every power-of-two detector), so slots 0-3 are left padding, 4-11 data
// and 12-15 right padding at compile time: padding slots load nothing and
// hold no registers.  Otherwise the same tests run on the runtime offsets
// (each is uniform over the work-group).
template <int L, typename TO, bool HALF>
__global__ void __launch_bounds__(L / kRegPts)
k_norm_filter_reg(RawInput in, const float* __restrict__ dmean, const float* __restrict__ rden, int n_angles, int n,
                  int off, FilterTables ft, TO* out) {
    extern __shared__ float2 lds[];
    constexpr int B = L / kRegPts;
    const int pairs = (n_angles + 1) >> 1;
    const int groups = (pairs + kPairsPerGroup - 1) / kPairsPerGroup;
    const int r = blockIdx.x / groups;
    const int g0 = (blockIdx.x - r * groups) * kPairsPerGroup;
    const int g1 = min(pairs, g0 + kPairsPerGroup);
    const float* dm = dmean + static_cast<int64_t>(r) * n;
    const float* dn = rden + static_cast<int64_t>(r) * n;
    // the thread's FFT twiddles, the same for every transform of the group
    RegTw<L> w;
    reg_tw_load<L>(w, ft.tw, threadIdx.x);
    // slot s holds padded position t + B s; a slot whose B positions all lie
    // left (right) of the detector holds the edge value in every thread
    auto left_pad = [&](int s) { return HALF ? s < 4 : B * s + B - 1 - off < 0; };
    auto right_pad = [&](int s) { return HALF ? s >= 12 : B * s - off > n - 1; };
    auto column = [&](int t, int s) { return HALF ? t + B * s - off : min(max(t + B * s - off, 0), n - 1); };
    // raw counts of a pair: row 2g in the low half, row 2g + 1 (or 0) in the high half
    auto load_pair = [&](int g, int t, uint32_t (&raw)[kRegPts]) {
        const int a0 = 2 * g;
        const uint16_t* p0 = in.proj + a0 * in.proj_stride + static_cast<int64_t>(r) * n;
        const bool has1 = a0 + 1 < n_angles;
        const uint16_t* p1 = has1 ? p0 + in.proj_stride : p0;
#pragma unroll
        for (int s = 0; s < kRegPts; ++s) {
            if (left_pad(s) || right_pad(s)) continue;
            const int c = column(t, s);
            const uint32_t hi = p1[c];
            raw[s] = p0[c] | (has1 ? hi << 16 : 0u);
        }
    };
    uint32_t cur[kRegPts], nxt[kRegPts];
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) cur[s] = nxt[s] = 0u;
    load_pair(g0, threadIdx.x, cur);
    const float dL = dm[0], eL = dn[0], dR = dm[n - 1], eR = dn[n - 1];
#pragma unroll 1
    for (int g = g0; g < g1; ++g) {
        // an opaque thread index per pair: per-thread offsets (columns, LDS and
        // output positions) are recomputed in the loop instead of being
        // hoisted into registers held across it
        int t = threadIdx.x;
        asm volatile("" : "+v"(t));
        if (g + 1 < g1) load_pair(g + 1, t, nxt);
        const int a0 = 2 * g;
        const bool has1 = a0 + 1 < n_angles;
        const uint16_t* p0 = in.proj + a0 * in.proj_stride + static_cast<int64_t>(r) * n;
        const uint16_t* p1 = has1 ? p0 + in.proj_stride : p0;
        const float2 left = make_float2(neglog_counts(static_cast<float>(p0[0]), dL, eL),
                                        has1 ? neglog_counts(static_cast<float>(p1[0]), dL, eL) : 0.0f);
        const float2 right = make_float2(neglog_counts(static_cast<float>(p0[n - 1]), dR, eR),
                                         has1 ? neglog_counts(static_cast<float>(p1[n - 1]), dR, eR) : 0.0f);
        float2 x[kRegPts];
#pragma unroll
        for (int s = 0; s < kRegPts; ++s) {
            if (left_pad(s)) {
                x[s] = left;
            } else if (right_pad(s)) {
                x[s] = right;
            } else {
                const int c = column(t, s);
                const float d = dm[c], e = dn[c];
                x[s] = make_float2(neglog_counts(static_cast<float>(cur[s] & 0xffffu), d, e),
                                   has1 ? neglog_counts(static_cast<float>(cur[s] >> 16), d, e) : 0.0f);
            }
        }
        // y = conj of IFFT(H . FFT(u)) (H real and even, 1/L folded in)
        reg_fft_w<L>(x, lds, w, t);
#pragma unroll
        for (int s = 0; s < kRegPts; ++s) {
            const float h = ft.H[t + B * s];
            x[s] = make_float2(x[s].x * h, 0.0f - x[s].y * h);
        }
        reg_fft_w<L>(x, lds, w, t);
        TO* o0 = out + (static_cast<int64_t>(r) * n_angles + a0) * n;
        TO* o1 = o0 + n;
#pragma unroll
        for (int s = 0; s < kRegPts; ++s) {
            if (HALF && (s < 4 || s >= 12)) continue;
            const int j = t + B * s - off;
            if (HALF || (j >= 0 && j < n)) {
                store_from_float(o0, j, x[s].x);
                if (has1) store_from_float(o1, j, 0.0f - x[s].y);
            }
        }
#pragma unroll
        for (int s = 0; s < kRegPts; ++s) cur[s] = nxt[s];
    }
}

size_t reg_lds_bytes(int L) { return static_cast<size_t>(L + L / 16) * sizeof(float2); }

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

template <int L, typename K>
hipError_t launch_reg(K kernel, dim3 grid, hipStream_t st, size_t& lds) {
    lds = reg_lds_bytes(L);
    return ensure_lds(kernel, lds);
}

template <typename TI, typename TO>
hipError_t launch_filter_t(const void* in, void* out, int64_t n_lines, int n, const FilterTables& ft,
                           hipStream_t st) {
    const int off = (ft.L - n) / 2;
    const int64_t blocks = (n_lines + 1) / 2;
    const dim3 grid(static_cast<unsigned>(blocks));
    const TI* pin = static_cast<const TI*>(in);
    TO* pout = static_cast<TO*>(out);
    size_t lds = 0;
    hipError_t e = hipSuccess;
#define TP_REG_CASE(LL)                                                                                    \
    case LL:                                                                                              \
        e = launch_reg<LL>(k_filter_reg<LL, TI, TO>, grid, st, lds);                                      \
        if (e != hipSuccess) return e;                                                                    \
        hipLaunchKernelGGL((k_filter_reg<LL, TI, TO>), grid, dim3(LL / kRegPts), lds, st, pin, pout, n_lines, \
                           n, off, ft);                                                                   \
        return hipGetLastError();
    switch (ft.L) {
        TP_REG_CASE(1024)
        TP_REG_CASE(2048)
        TP_REG_CASE(4096)
        TP_REG_CASE(8192)
        default: break;
    }
#undef TP_REG_CASE
    lds = static_cast<size_t>(ft.L) * sizeof(float2);
    e = ensure_lds(k_filter<TI, TO>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_filter<TI, TO>), grid, dim3(filter_block(ft.L)), lds, st, pin, pout, n_lines, n, off, ft);
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
    const int off = (ft.L - n) / 2;
    const int64_t blocks = static_cast<int64_t>(n_rows) * ((n_angles + 1) / 2);
    const dim3 grid(static_cast<unsigned>(blocks));
    const int64_t reg_blocks =
        static_cast<int64_t>(n_rows) * ((((n_angles + 1) / 2) + kPairsPerGroup - 1) / kPairsPerGroup);
    const dim3 reg_grid(static_cast<unsigned>(reg_blocks));
    TO* pout = static_cast<TO*>(out);
    size_t lds = 0;
    hipError_t e = hipSuccess;
#define TP_REG_CASE(LL)                                                                                    \
    case LL:                                                                                              \
        if (2 * n == LL) {                                                                                \
            e = launch_reg<LL>(k_norm_filter_reg<LL, TO, true>, reg_grid, st, lds);                       \
            if (e != hipSuccess) return e;                                                                \
            hipLaunchKernelGGL((k_norm_filter_reg<LL, TO, true>), reg_grid, dim3(LL / kRegPts), lds, st, in, \
                               dmean, den, n_angles, n, off, ft, pout);                                   \
        } else {                                                                                          \
            e = launch_reg<LL>(k_norm_filter_reg<LL, TO, false>, reg_grid, st, lds);                      \
            if (e != hipSuccess) return e;                                                                \
            hipLaunchKernelGGL((k_norm_filter_reg<LL, TO, false>), reg_grid, dim3(LL / kRegPts), lds, st, in, \
                               dmean, den, n_angles, n, off, ft, pout);                                   \
        }                                                                                                 \
        return hipGetLastError();
    switch (ft.L) {
        TP_REG_CASE(1024)
        TP_REG_CASE(2048)
        TP_REG_CASE(4096)
        TP_REG_CASE(8192)
        default: break;
    }
#undef TP_REG_CASE
    lds = static_cast<size_t>(ft.L) * sizeof(float2);
    e = ensure_lds(k_norm_filter<TO>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_norm_filter<TO>), grid, dim3(filter_block(ft.L)), lds, st, in, dmean, den, n_angles, n,
                       off, ft, pout);
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
