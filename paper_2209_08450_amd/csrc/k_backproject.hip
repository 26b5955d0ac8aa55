// Pixel-driven backprojection with linear interpolation (paper, Sections 2.2
// and 3, "LineRec": direct discretisation of the backprojection line integral),
// and its exact transpose, the forward projector.
//
// Detector coordinate of voxel (ix, iy) at angle a, for tile (bx, by) =
// (ix / 32, iy / 32) and in-tile offset (dx, dy) = (ix % 32, iy % 32):
//   s = bi + fma(dx, cos_a, fma(dy, sin_a, bf)),
//   bi + bf = (bx*32 - N/2) cos_a + (by*32 - N/2) sin_a + center   (FP64 on the host,
//   split into integers xi + yi and FP32 fractions xf + yf).
// Keeping the FP32 part below 64 columns holds the coordinate error near
// 1e-6 column where a plain FP32 evaluation of |s| ~ 1000 loses ~1e-4.
// Both kernels evaluate exactly this expression (explicit fma, no
// reassociation), so they take identical floor and weight decisions.
//
// Backprojection work-group: one 32x32 voxel tile x K slices, 256 threads.
// Thread (wave w, lane l) owns voxels (l%8 + 8i, l/8 + 8w), i = 0..3, so each
// wave step covers an 8x8 block whose taps fall in a window of about 13
// detector bins -- distinct LDS banks, or broadcasts.  For a block of A angles
// the work-group stages, per slice and angle, the 48-bin window of filtered
// values the tile can touch as (Q[j], Q[j+1]) pairs in LDS; the inner loop is
// then one LDS read and two FMAs per voxel, slice and angle, with floor,
// fraction and address shared by the K slices.  The staged window starts at
// bi + floor(min over the tile corners of the FP32 offset); fma is monotone
// in each argument, so every voxel's floor lies in [0, 45) of the window.
#include "tp_internal.h"

namespace tp {
namespace {

template <typename T> struct Stage;  // LDS pair type per storage type
template <> struct Stage<float> {
    using P = float2;
    __device__ static P make(float a, float b) { return make_float2(a, b); }
    __device__ static float lo(P p) { return p.x; }
    __device__ static float hi(P p) { return p.y; }
};
template <> struct Stage<__half> {
    using P = __half2;
    __device__ static P make(float a, float b) { return __halves2half2(__float2half_rn(a), __float2half_rn(b)); }
    __device__ static float lo(P p) { return __low2float(p); }
    __device__ static float hi(P p) { return __high2float(p); }
};
template <> struct Stage<uint16_t> {  // bfloat16 storage: widened to FP32 pairs in LDS
    using P = float2;
    __device__ static P make(float a, float b) { return make_float2(a, b); }
    __device__ static float lo(P p) { return p.x; }
    __device__ static float hi(P p) { return p.y; }
};

template <typename T> __device__ __forceinline__ float ld(const T* p, int j) { return load_as_float(p, j); }

template <typename T, int K>
__global__ void __launch_bounds__(kBpThreads)
k_backproject(GeoTables g, const T* __restrict__ filt, int n_rows, int A, float scale,
              float* __restrict__ vol, int accumulate) {
    using S = Stage<T>;
    using P = typename S::P;
    extern __shared__ __align__(16) unsigned char smem[];
    P* sQ = reinterpret_cast<P*>(smem);                                // [K][A][kWin]
    float4* sGeo = reinterpret_cast<float4*>(sQ + K * A * kWin);        // [A] {bf, cos, sin, floor(min)}
    int* sWs = reinterpret_cast<int*>(sGeo + A);                        // [A] window start bin

    const int na = g.na, n = g.n, nb = g.nb;
    const int bx = blockIdx.x % nb, by = blockIdx.x / nb;
    const int z0 = blockIdx.y * K;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const float dy = static_cast<float>((lane >> 3) + 8 * wv);
    const float dx0 = static_cast<float>(lane & 7);
    const float dxs[4] = {dx0, dx0 + 8.0f, dx0 + 16.0f, dx0 + 24.0f};
    const int kstride = A * kWin;

    float acc[4][K];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[i][k] = 0.0f;

    for (int a0 = 0; a0 < na; a0 += A) {
        const int nA = min(A, na - a0);
        if (tid < nA) {
            const int a = a0 + tid;
            const float cs = g.cs[a], sn = g.sn[a];
            const int bi = g.xi[bx * na + a] + g.yi[by * na + a];
            const float bf = g.xf[bx * na + a] + g.yf[by * na + a];
            const float ty = __builtin_fmaf(sn >= 0.0f ? 0.0f : 31.0f, sn, bf);
            const float smin = __builtin_fmaf(cs >= 0.0f ? 0.0f : 31.0f, cs, ty);
            const float fmin = floorf(smin);
            sGeo[tid] = make_float4(bf, cs, sn, fmin);
            sWs[tid] = bi + static_cast<int>(fmin);
        }
        __syncthreads();
        // Stage K x nA windows: one wave per (slice, angle) row, lanes 0..48 load
        // Q[ws + lane]; the pair's upper element comes from the next lane.
        for (int row = wv; row < K * nA; row += kBpThreads / 64) {
            const int k = row / nA;
            const int a = row - k * nA;
            const int z = z0 + k;
            const int j = sWs[a] + lane;
            float q = 0.0f;
            if (z < n_rows && lane <= kWin && j >= 0 && j < n)
                q = ld(filt + (static_cast<int64_t>(z) * na + a0 + a) * n, j);
            const float q1 = __shfl_down(q, 1);
            if (lane < kWin) sQ[k * kstride + a * kWin + lane] = S::make(q, q1);
        }
        __syncthreads();
        for (int a = 0; a < nA; ++a) {
            const float4 ge = sGeo[a];
            const float t = __builtin_fmaf(dy, ge.z, ge.x);
            const P* rowp = sQ + a * kWin;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float s = __builtin_fmaf(dxs[i], ge.y, t);
                const float fl = floorf(s);
                const float w = s - fl;
                const float omw = 1.0f - w;
                // in [0, 44] by the monotonicity argument; the clamp (one
                // v_med3) only guards the staged window
                const int jl = min(max(static_cast<int>(fl - ge.w), 0), kWin - 2);
                const P* pp = rowp + jl;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const P pr = pp[k * kstride];
                    acc[i][k] = __builtin_fmaf(S::hi(pr), w, __builtin_fmaf(S::lo(pr), omw, acc[i][k]));
                }
            }
        }
        __syncthreads();
    }

    const int N = g.N;
    const int y = by * kGeoTile + (lane >> 3) + 8 * wv;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int x = bx * kGeoTile + (lane & 7) + 8 * i;
        if (x >= N || y >= N) continue;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int z = z0 + k;
            if (z >= n_rows) continue;
            const int64_t idx = (static_cast<int64_t>(z) * N + y) * N + x;
            const float v = scale * acc[i][k];
            vol[idx] = accumulate ? vol[idx] + v : v;
        }
    }
}

// Forward projection, gather form: wave = one angle, lanes = 64 consecutive
// detector bins, K slices.  Each bin sweeps the image along the axis the ray
// is closer to (rows when |cos| >= |sin|), takes the few voxels whose
// coordinate can fall in [j - 1, j + 1), recomputes their exact (j0, w) with
// the backprojector's expression and adds (1 - w) or w times the voxel.
template <int K>
__global__ void __launch_bounds__(256)
k_radon(GeoTables g, const float* __restrict__ vol, int n_rows, float* __restrict__ sino) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int jgroups = (g.n + 63) >> 6;
    const int a = (blockIdx.x / jgroups) * 4 + wv;
    const int j = (blockIdx.x % jgroups) * 64 + lane;
    const int z0 = blockIdx.y * K;
    if (a >= g.na || j >= g.n) return;  // no block-level synchronisation below
    const int na = g.na, N = g.N, half = N / 2;
    const float cs = g.cs[a], sn = g.sn[a];
    const bool rows_major = fabsf(cs) >= fabsf(sn);
    const float cmaj = rows_major ? cs : sn;   // coefficient of the swept (minor) coordinate
    const float cmin = rows_major ? sn : cs;   // coefficient of the major coordinate
    const float reach = 1.0f / fabsf(cmaj);
    float acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0f;
    int nz = min(K, n_rows - z0);

    for (int m = 0; m < N; ++m) {
        // approximate centre of the footprint on this line (FP32; a superset of
        // candidates is taken, the exact test below decides)
        const float um = static_cast<float>(m - half) * cmin + g.center_f;
        const float c = (static_cast<float>(j) - um) / cmaj + static_cast<float>(half);
        int lo = static_cast<int>(floorf(c - reach)) - 1;
        int hi = static_cast<int>(floorf(c + reach)) + 1;
        lo = max(lo, 0);
        hi = min(hi, N - 1);
        for (int v = lo; v <= hi; ++v) {
            const int ix = rows_major ? v : m;
            const int iy = rows_major ? m : v;
            const int bx = ix >> 5, by = iy >> 5;
            const float dx = static_cast<float>(ix & 31), dy = static_cast<float>(iy & 31);
            const int bi = g.xi[bx * na + a] + g.yi[by * na + a];
            const float bf = g.xf[bx * na + a] + g.yf[by * na + a];
            const float s = __builtin_fmaf(dx, cs, __builtin_fmaf(dy, sn, bf));
            const float fl = floorf(s);
            const int j0 = bi + static_cast<int>(fl);
            const float w = s - fl;
            float wt;
            if (j0 == j) wt = 1.0f - w;
            else if (j0 + 1 == j) wt = w;
            else continue;
            const int64_t off = static_cast<int64_t>(iy) * N + ix;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (k < nz) acc[k] = __builtin_fmaf(wt, vol[(static_cast<int64_t>(z0 + k) * N) * N + off], acc[k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (k < nz) sino[(static_cast<int64_t>(z0 + k) * na + a) * g.n + j] = acc[k];
    }
}

size_t bp_lds_bytes(tp_dtype dt, int K, int A) {
    const size_t pair = (dt == TP_F16) ? 4 : 8;
    return pair * K * A * kWin + static_cast<size_t>(A) * (sizeof(float4) + sizeof(int));
}

template <typename T, int K>
hipError_t launch_bp_t(const GeoTables& g, const void* filt, int n_rows, float scale, float* vol,
                       int accumulate, int A, size_t lds, hipStream_t st) {
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_backproject<T, K>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    const dim3 grid(static_cast<unsigned>(g.nb * g.nb), static_cast<unsigned>((n_rows + K - 1) / K));
    hipLaunchKernelGGL((k_backproject<T, K>), grid, dim3(kBpThreads), lds, st, g, static_cast<const T*>(filt),
                       n_rows, A, scale, vol, accumulate);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_bp_k(const GeoTables& g, const void* filt, int n_rows, float scale, float* vol,
                       int accumulate, int K, int A, size_t lds, hipStream_t st) {
    switch (K) {
        case 1: return launch_bp_t<T, 1>(g, filt, n_rows, scale, vol, accumulate, A, lds, st);
        case 2: return launch_bp_t<T, 2>(g, filt, n_rows, scale, vol, accumulate, A, lds, st);
        case 4: return launch_bp_t<T, 4>(g, filt, n_rows, scale, vol, accumulate, A, lds, st);
        case 8: return launch_bp_t<T, 8>(g, filt, n_rows, scale, vol, accumulate, A, lds, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

size_t backproject_lds_bytes(tp_dtype dt, int slices_per_block, int angles_per_block) {
    return bp_lds_bytes(dt, slices_per_block, angles_per_block);
}

hipError_t launch_backproject(const GeoTables& g, const void* filt, tp_dtype dt, int n_rows, float scale,
                              float* vol, int accumulate, int slices_per_block, int angles_per_block,
                              hipStream_t st) {
    const size_t lds = bp_lds_bytes(dt, slices_per_block, angles_per_block);
    switch (dt) {
        case TP_F32:
            return launch_bp_k<float>(g, filt, n_rows, scale, vol, accumulate, slices_per_block,
                                      angles_per_block, lds, st);
        case TP_F16:
            return launch_bp_k<__half>(g, filt, n_rows, scale, vol, accumulate, slices_per_block,
                                       angles_per_block, lds, st);
        case TP_BF16:
            return launch_bp_k<uint16_t>(g, filt, n_rows, scale, vol, accumulate, slices_per_block,
                                         angles_per_block, lds, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_radon(const GeoTables& g, const float* vol, int n_rows, float* sino, hipStream_t st) {
    constexpr int K = 4;
    const int jgroups = (g.n + 63) / 64;
    const dim3 grid(static_cast<unsigned>(jgroups * ((g.na + 3) / 4)), static_cast<unsigned>((n_rows + K - 1) / K));
    hipLaunchKernelGGL((k_radon<K>), grid, dim3(256), 0, st, g, vol, n_rows, sino);
    return hipGetLastError();
}

}  // namespace tp
