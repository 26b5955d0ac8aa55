// Dark/flat-field correction and negative logarithm (paper, Section 2.2).
//
// k_darkflat: per detector pixel (row r, column j), the arithmetic means of the
//   dark and flat frames.  Frame values are summed as integers (<= 256 frames
//   of 16-bit counts stay below 2^24, exact in FP32), then divided once.
//   Stores D and rden = 1 / max(F - D, 1).
// k_normalize: sino[r][a][j] = -ln(max((P[a][r][j] - D) * rden, 1e-6)).
//   One work-group per (projection a, row r): it moves a whole detector row,
//   so both the projection-major read and the sinogram-major write are
//   contiguous; 8 counts per thread per 16-byte load where the row allows.
//
// The allocation-free variant keeps D and rden in `scratch`, a file-scope
// device array (one copy per GPU, held until the process ends); host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device.
#include <mutex>

#include "tp_internal.h"

namespace tp {

// D at [0, kNoAllocPixels), rden at [kNoAllocPixels, 2 kNoAllocPixels).
static __device__ __align__(256) float scratch[2 * kNoAllocPixels];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_addr[kMaxScratchDevices] = {};

__global__ void __launch_bounds__(256)
k_darkflat(RawInput in, int n_rows, int n_det, float* __restrict__ dmean, float* __restrict__ rden) {
    const int64_t npix = static_cast<int64_t>(n_rows) * n_det;
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const int64_t r = p / n_det, j = p - r * n_det;
    const int64_t off = r * n_det + j;
    uint32_t sd = 0, sf = 0;
    for (int f = 0; f < in.n_dark; ++f) sd += in.dark[f * in.frame_stride + off];
    for (int f = 0; f < in.n_flat; ++f) sf += in.flat[f * in.frame_stride + off];
    const float d = static_cast<float>(sd) / static_cast<float>(in.n_dark);
    const float fl = static_cast<float>(sf) / static_cast<float>(in.n_flat);
    dmean[p] = d;
    rden[p] = 1.0f / fmaxf(fl - d, 1.0f);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_normalize(RawInput in, const float* __restrict__ dmean, const float* __restrict__ den, int n_angles,
            int n_rows, int n_det, T* __restrict__ sino) {
    const int a = blockIdx.x;   // projection
    const int r = blockIdx.y;   // detector row
    const uint16_t* src = in.proj + a * in.proj_stride + static_cast<int64_t>(r) * n_det;
    const float* dm = dmean + static_cast<int64_t>(r) * n_det;
    const float* dn = den + static_cast<int64_t>(r) * n_det;
    T* dst = sino + (static_cast<int64_t>(r) * n_angles + a) * n_det;
    // vector path when the source row is 16-byte aligned and whole
    const bool vec = ((reinterpret_cast<uintptr_t>(src) & 15u) == 0) && ((n_det & 7) == 0);
    if (vec) {
        const int nv = n_det >> 3;
        for (int v = threadIdx.x; v < nv; v += blockDim.x) {
            const uint4 raw = reinterpret_cast<const uint4*>(src)[v];
            const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int j = v * 8 + k;
                const float P = static_cast<float>((w[k >> 1] >> ((k & 1) * 16)) & 0xffffu);
                store_from_float(dst, j, neglog_counts(P, dm[j], dn[j]));
            }
        }
    } else {
        for (int j = threadIdx.x; j < n_det; j += blockDim.x) {
            store_from_float(dst, j, neglog_counts(static_cast<float>(src[j]), dm[j], dn[j]));
        }
    }
}

}  // namespace

hipError_t normalize_scratch(float** dmean, float** den) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[dev] = static_cast<float*>(p);
    }
    *dmean = g_scratch_addr[dev];
    *den = g_scratch_addr[dev] + kNoAllocPixels;
    return hipSuccess;
}

hipError_t launch_darkflat(const RawInput& in, int n_rows, int n_det, float* dmean, float* den,
                           hipStream_t st) {
    const int64_t npix = static_cast<int64_t>(n_rows) * n_det;
    const int64_t blocks = (npix + 255) / 256;
    hipLaunchKernelGGL(k_darkflat, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, in, n_rows,
                       n_det, dmean, den);
    return hipGetLastError();
}

hipError_t launch_normalize(const RawInput& in, const float* dmean, const float* den, int n_angles,
                            int n_rows, int n_det, tp_dtype out_dtype, void* sino, hipStream_t st) {
    const dim3 grid(n_angles, n_rows);
    const dim3 block(256);
    switch (out_dtype) {
        case TP_F32:
            hipLaunchKernelGGL(k_normalize<float>, grid, block, 0, st, in, dmean, den, n_angles, n_rows,
                               n_det, static_cast<float*>(sino));
            break;
        case TP_F16:
            hipLaunchKernelGGL(k_normalize<__half>, grid, block, 0, st, in, dmean, den, n_angles, n_rows,
                               n_det, static_cast<__half*>(sino));
            break;
        case TP_BF16:
            hipLaunchKernelGGL(k_normalize<uint16_t>, grid, block, 0, st, in, dmean, den, n_angles,
                               n_rows, n_det, static_cast<uint16_t*>(sino));
            break;
    }
    return hipGetLastError();
}

}  // namespace tp
