// Pixel-driven backprojection with linear interpolation (paper, Sections 2.2
// and 3, "LineRec": direct discretisation of the backprojection line integral).
// Its exact transpose, the forward projector, is in k_radon.hip.
//
// Detector coordinate of voxel (ix, iy) at angle a, for tile (bx, by) =
// (ix / 32, iy / 32) and in-tile offset (dx, dy) = (ix % 32, iy % 32):
//   s = bi + fma(dx, cos_a, fma(dy, sin_a, bf)),
//   bi + bf = (bx*32 - N/2) cos_a + (by*32 - N/2) sin_a + center   (FP64 on the host,
//   split into integers xi + yi and FP32 fractions xf + yf).
// Keeping the FP32 part below 64 columns holds the coordinate error near
// 1e-6 column where a plain FP32 evaluation of |s| ~ 1000 loses ~1e-4.
// The backprojector and the forward projector evaluate exactly this
// expression (shared helpers, explicit fma, no reassociation), so they take
// identical floor and weight decisions.
//
// Backprojection work-group: one 32x32 voxel tile x K slices, 256 threads.
// Thread (wave w, lane l) owns voxels (l%8 + 8i, l/8 + 8w), i = 0..3, so each
// wave step covers an 8x8 block whose taps fall in a window of about 13
// detector bins.  For a block of A angles, each wave stages whole angles: lane
// b loads bin ws + b of the K slices' filtered rows and writes them as one
// contiguous group, so LDS holds [angle][bin][slice] (bf16 widened to FP32;
// groups padded to an odd number of 16-byte bank groups).
// The window starts at ws = bi + floor(min over the tile corners of the
// FP32 offset); fma is monotone in each argument, so every voxel's floor
// lies in [0, 45) of the 48-bin window and both taps are staged.  The inner
// loop per voxel and angle: offset (1 FMA), fraction, floor, address, 1 - w,
// reads of the two bins' K-slice groups (16-byte LDS reads), then two FP32
// FMAs per slice.  Every slice sums its angles in order, so results do not
// depend on K or A.
//
// FP16 rows (the paper's 16-bit mode, Section 2.1) take a kernel of their own,
// k_backproject_h2: LDS holds for each (angle, bin j) the K slices' pairs
// (Q[j], Q[j+1]) as packed halves, staged with one 4-byte load per slice, and
// the weights (1 - w, w) are rounded to FP16 (nearest), so one v_dot2 per slice
// and voxel adds (1 - w) Q[j] + w Q[j+1] to the FP32 sum: half the VALU issue
// of two mixed-precision FMAs, the same LDS bytes.  The weights' rounding
// (at most 2^-12 of a bin's value) is the FP16 mode's only change to the
// arithmetic; every product is exact and every sum FP32.  Its output slices
// are FP32, or FP16 (each voxel's FP32 result rounded once) for 16-bit volumes.
#include <type_traits>

#include "tp_internal.h"

namespace tp {
namespace {

template <typename T> struct Lds { using U = T; };          // LDS element per storage type
template <> struct Lds<uint16_t> { using U = float; };     // bf16 widened

template <typename T> __device__ __forceinline__ float ld(const T* p, int j) { return load_as_float(p, j); }

// One staged element: raw copy, or bf16 widened to FP32.
template <typename T, typename U>
__device__ __forceinline__ U stage_load(const unsigned char* p) {
    if constexpr (std::is_same<T, U>::value) {
        return *reinterpret_cast<const T*>(p);
    } else {
        return ld(reinterpret_cast<const T*>(p), 0);
    }
}

__device__ __forceinline__ float lds_val(const float* v, int i) { return v[i]; }

// Copy BYTES between LDS and registers in chunks of CHUNK bytes (the
// alignment both addresses are known to have, at most 16).
template <int BYTES, int CHUNK>
__device__ __forceinline__ void copy_group(void* dst, const void* src) {
    static_assert(BYTES % CHUNK == 0, "size must be a multiple of the chunk");
    if constexpr (CHUNK >= 16) {
#pragma unroll
        for (int v = 0; v < BYTES / 16; ++v) reinterpret_cast<uint4*>(dst)[v] = reinterpret_cast<const uint4*>(src)[v];
    } else if constexpr (CHUNK == 8) {
#pragma unroll
        for (int v = 0; v < BYTES / 8; ++v) reinterpret_cast<uint2*>(dst)[v] = reinterpret_cast<const uint2*>(src)[v];
    } else if constexpr (CHUNK == 4) {
#pragma unroll
        for (int v = 0; v < BYTES / 4; ++v)
            reinterpret_cast<uint32_t*>(dst)[v] = reinterpret_cast<const uint32_t*>(src)[v];
    } else {
#pragma unroll
        for (int v = 0; v < BYTES / 2; ++v)
            reinterpret_cast<uint16_t*>(dst)[v] = reinterpret_cast<const uint16_t*>(src)[v];
    }
}

// Tile of work-group `wg` among nb x nb tiles.  Work-groups are dispatched
// round-robin over the 8 XCDs, so wg % 8 names the XCD; each XCD gets one
// eighth of the grid (nb/2 x nb/4 tiles) and walks it in Morton order, so the
// ~160 work-groups resident on an XCD at a time form a compact cluster whose
// detector windows overlap in that XCD's L2.  Bijective for power-of-two
// nb >= 8; other sizes use row-major order.
__device__ __forceinline__ void tile_of(int wg, int nb, int& bx, int& by) {
    if (nb >= 8 && (nb & (nb - 1)) == 0) {
        const int part = wg & 7, q = wg >> 3;
        const int hr = nb >> 2;                      // part is (2 hr) x hr tiles
        const int sq = hr * hr;
        const int half_x = q / sq;                   // left or right square of the part
        int r = q - half_x * sq, sx = 0, sy = 0;
        for (int bit = 0; (1 << (2 * bit)) < sq; ++bit) {
            sx |= ((r >> (2 * bit)) & 1) << bit;
            sy |= ((r >> (2 * bit + 1)) & 1) << bit;
        }
        bx = (part & 1) * (2 * hr) + half_x * hr + sx;
        by = (part >> 1) * hr + sy;
    } else {
        bx = wg % nb;
        by = wg / nb;
    }
}

// LDS pitch of one (angle, bin) group of BIN bytes.  With a pitch of four or
// more (an even number of) 16-byte bank groups, bins 4 apart share banks and
// a wave's 16-byte reads of its ~10 neighbouring bins conflict; one more
// group makes the pitch odd and spreads them.  (Two groups measured no
// better padded.)
constexpr int bin_pitch(int bin) { return (bin >= 64 && (bin / 16) % 2 == 0) ? bin + 16 : bin; }

// Lowest occupancy the register allocator must keep for the FP32-arithmetic
// kernel.  16 slices x 8 angles take 30.8 KB of LDS, room for 5 work-groups
// (5 waves per SIMD) per CU; the allocator alone gives that tile 98 registers
// (4 waves), and bounded to 5 waves it needs no spill.  Larger tiles are held
// to fewer work-groups by their LDS, smaller ones use few registers: they keep
// the default.
constexpr int bp_min_waves(int K, int A) { return (K == 16 && A == 8) ? 5 : 1; }

template <typename T, int K, int A>
__global__ void __launch_bounds__(kBpThreads) __attribute__((amdgpu_waves_per_eu(bp_min_waves(K, A))))
k_backproject(GeoTables g, const T* __restrict__ filt, int n_rows, float scale, float* __restrict__ vol,
              int accumulate) {
    using U = typename Lds<T>::U;
    constexpr int BIN = K * static_cast<int>(sizeof(U));  // bytes of one (angle, bin) group
    constexpr int P = bin_pitch(BIN);                       // LDS bytes between bins
    extern __shared__ __align__(16) unsigned char smem[];
    // smem: [A][kWin][K] values of U, then sGeo
    float4* sGeo = reinterpret_cast<float4*>(smem + A * kWin * P);          // [A] {bf, cos, sin, byte base}

    const int na = g.na, n = g.n, nb = g.nb;
    int bx, by;
    tile_of(blockIdx.x, nb, bx, by);
    const int z0 = blockIdx.y * K;
    const int kz = min(K, n_rows - z0);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: angle loads go scalar
    const float dy = static_cast<float>((lane >> 3) + 8 * wv);
    const float dx0 = static_cast<float>(lane & 7);
    const T* rows0 = filt + static_cast<int64_t>(z0) * na * n;
    const int64_t slice_bytes = static_cast<int64_t>(na) * n * static_cast<int64_t>(sizeof(T));

    float acc[4][K];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[i][k] = 0.0f;

    for (int a0 = 0; a0 < na; a0 += A) {
        const int nA = __builtin_amdgcn_readfirstlane(min(A, na - a0));  // keeps the angle loop scalar
        // stage: wave wv takes angles wv, wv+4, ...; lane b holds bin ws + b
        for (int a = wv; a < nA; a += kBpThreads / 64) {
            const int ag = a0 + a;
            const float cs = g.cs[ag], sn = g.sn[ag];
            const int bi = g.xi[bx * na + ag] + g.yi[by * na + ag];
            const float bf = g.xf[bx * na + ag] + g.yf[by * na + ag];
            const float smin = tile_offset(cs >= 0.0f ? 0.0f : 31.0f, sn >= 0.0f ? 0.0f : 31.0f, cs, sn, bf);
            const int fmin = coord_floor(smin);
            if (lane == 0) sGeo[a] = make_float4(bf, cs, sn, __int_as_float((a * kWin - fmin) * P));
            if (lane < kWin) {
                // Every slice uses the same 32-bit lane offset, of the bin
                // clamped onto the detector; slice k's row base is
                // wave-uniform: rowb + kk * slice_bytes with kk = min(k, kz - 1)
                // made opaque, so each base is a few scalar instructions at its
                // load instead of K hoisted 64-bit constants.  Slices past the
                // last row re-read it; their sums are never stored.  Lanes
                // whose bin is off the detector overwrite their group with
                // zeros afterwards (only edge waves take that branch).
                const int j = bi + fmin + lane;
                const uint32_t voff = static_cast<uint32_t>(min(max(j, 0), n - 1)) *
                                      static_cast<uint32_t>(sizeof(T));
                const unsigned char* rowb = reinterpret_cast<const unsigned char*>(rows0) +
                                            static_cast<int64_t>(ag) * n * static_cast<int64_t>(sizeof(T));
                U q[K];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    int kk = min(k, kz - 1);
                    asm volatile("" : "+s"(kk));
                    q[k] = stage_load<T, U>(rowb + kk * slice_bytes + voff);
                }
                unsigned char* dst = smem + (a * kWin + lane) * P;
                copy_group<BIN, (BIN < 16 ? BIN : 16)>(dst, q);
                if (j < 0 || j >= n) {
                    U zero[K];
#pragma unroll
                    for (int k = 0; k < K; ++k) zero[k] = static_cast<U>(0.0f);
                    copy_group<BIN, (BIN < 16 ? BIN : 16)>(dst, zero);
                }
            }
        }
        __syncthreads();
        for (int a = 0; a < nA; ++a) {
            const float4 ge = sGeo[a];
            const int base = __float_as_int(ge.w);
            U r[4][2 * K];  // bins (j, j+1) of K slices per voxel
            float w[4], omw[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float s = tile_offset(dx0 + 8.0f * i, dy, ge.y, ge.z, ge.x);
                w[i] = coord_frac(s);
                omw[i] = 1.0f - w[i];
                const unsigned char* tap = smem + base + coord_floor(s) * P;
                if constexpr (P == BIN) {
                    copy_group<2 * BIN, (BIN < 16 ? BIN : 16)>(r[i], tap);
                } else {
                    copy_group<BIN, 16>(r[i], tap);
                    copy_group<BIN, 16>(r[i] + K, tap + P);
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int k = 0; k < K; ++k)
                    acc[i][k] = __builtin_fmaf(lds_val(r[i], K + k), w[i],
                                               __builtin_fmaf(lds_val(r[i], k), omw[i], acc[i][k]));
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
            if (k >= kz) continue;
            const int64_t idx = (static_cast<int64_t>(z0 + k) * N + y) * N + x;
            const float v = scale * acc[i][k];
            vol[idx] = accumulate ? vol[idx] + v : v;
        }
    }
}


// FP16 rows: pairs (Q[j], Q[j+1]) per slice in LDS, FP16 weights, v_dot2.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

template <int K, int A, typename OutT>
__global__ void __launch_bounds__(kBpThreads)
k_backproject_h2(GeoTables g, const __half* __restrict__ filt, int n_rows, float scale, OutT* __restrict__ vol,
                 int accumulate) {
    constexpr int BIN = K * 4;            // bytes of one (angle, bin) group: K packed pairs
    constexpr int P = bin_pitch(BIN);     // LDS bytes between bins
    extern __shared__ __align__(16) unsigned char smem[];
    float4* sGeo = reinterpret_cast<float4*>(smem + A * kWin * P);  // [A] {bf, cos, sin, byte base}

    const int na = g.na, n = g.n, nb = g.nb;
    int bx, by;
    tile_of(blockIdx.x, nb, bx, by);
    const int z0 = blockIdx.y * K;
    const int kz = min(K, n_rows - z0);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const float dy = static_cast<float>((lane >> 3) + 8 * wv);
    const float dx0 = static_cast<float>(lane & 7);
    const __half* rows0 = filt + static_cast<int64_t>(z0) * na * n;
    const int64_t slice_bytes = static_cast<int64_t>(na) * n * 2;

    float acc[4][K];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[i][k] = 0.0f;

    for (int a0 = 0; a0 < na; a0 += A) {
        const int nA = __builtin_amdgcn_readfirstlane(min(A, na - a0));
        // stage: wave wv takes angles wv, wv+4, ...; lane b holds the pairs of bin ws + b
        for (int a = wv; a < nA; a += kBpThreads / 64) {
            const int ag = a0 + a;
            const float cs = g.cs[ag], sn = g.sn[ag];
            const int bi = g.xi[bx * na + ag] + g.yi[by * na + ag];
            const float bf = g.xf[bx * na + ag] + g.yf[by * na + ag];
            const float smin = tile_offset(cs >= 0.0f ? 0.0f : 31.0f, sn >= 0.0f ? 0.0f : 31.0f, cs, sn, bf);
            const int fmin = coord_floor(smin);
            if (lane == 0) sGeo[a] = make_float4(bf, cs, sn, __int_as_float((a * kWin - fmin) * P));
            if (lane < kWin) {
                const int ws = bi + fmin;  // wave-uniform
                const int j = ws + lane;
                const unsigned char* rowb = reinterpret_cast<const unsigned char*>(rows0) +
                                            static_cast<int64_t>(ag) * n * 2;
                uint32_t q[K];
                // Slice k's row base is rowb + kk * slice_bytes with kk = min(k, kz - 1)
                // made opaque (scalar, not K hoisted 64-bit constants); slices past the
                // last row re-read it and their sums are never stored.
                if (ws >= 0 && ws + kWin <= n - 1) {
                    // window inside the detector: bins j and j + 1 in one 4-byte load
                    // (2-byte aligned; the hardware serves unaligned global loads)
                    const uint32_t voff = static_cast<uint32_t>(j) * 2u;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        int kk = min(k, kz - 1);
                        asm volatile("" : "+s"(kk));
                        __builtin_memcpy(&q[k], rowb + kk * slice_bytes + voff, 4);
                    }
                } else {
                    // window at an edge: taps off the detector read zero
                    const uint32_t v0 = static_cast<uint32_t>(min(max(j, 0), n - 1)) * 2u;
                    const uint32_t v1 = static_cast<uint32_t>(min(max(j + 1, 0), n - 1)) * 2u;
                    const uint32_t m0 = (j >= 0 && j < n) ? 0xffffu : 0u;
                    const uint32_t m1 = (j + 1 >= 0 && j + 1 < n) ? 0xffffu : 0u;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        int kk = min(k, kz - 1);
                        asm volatile("" : "+s"(kk));
                        const unsigned char* rb = rowb + kk * slice_bytes;
                        const uint32_t lo = *reinterpret_cast<const uint16_t*>(rb + v0) & m0;
                        const uint32_t hi = *reinterpret_cast<const uint16_t*>(rb + v1) & m1;
                        q[k] = lo | (hi << 16);
                    }
                }
                copy_group<BIN, (BIN < 16 ? BIN : 16)>(smem + (a * kWin + lane) * P, q);
            }
        }
        __syncthreads();
        for (int a = 0; a < nA; ++a) {
            const float4 ge = sGeo[a];
            const int base = __float_as_int(ge.w);
            uint32_t r[4][K];  // pairs (Q[j0], Q[j0+1]) of K slices per voxel
            half2_t wt[4];     // (1 - w, w) rounded to FP16
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float s = tile_offset(dx0 + 8.0f * i, dy, ge.y, ge.z, ge.x);
                const float w = coord_frac(s);
                wt[i] = half2_t{static_cast<_Float16>(1.0f - w), static_cast<_Float16>(w)};
                // |floor(s)| < 2^23 and P < 2^8: the 24-bit multiply is exact
                const unsigned char* tap = smem + base + __mul24(coord_floor(s), P);
                copy_group<BIN, (BIN < 16 ? BIN : 16)>(r[i], tap);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int k = 0; k < K; ++k)
                    acc[i][k] = __builtin_amdgcn_fdot2(__builtin_bit_cast(half2_t, r[i][k]), wt[i], acc[i][k], false);
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
            if (k >= kz) continue;
            const int64_t idx = (static_cast<int64_t>(z0 + k) * N + y) * N + x;
            const float v = scale * acc[i][k];
            if constexpr (std::is_same<OutT, __half>::value) {
                // FP16 slices: the FP32 sum rounded once to nearest
                vol[idx] = __float2half(accumulate ? __half2float(vol[idx]) + v : v);
            } else {
                vol[idx] = accumulate ? vol[idx] + v : v;
            }
        }
    }
}

size_t bp_lds_bytes(tp_dtype dt, int K, int A) {
    (void)dt;  // 4 bytes per slice and bin: FP32, bf16 widened to FP32, or an FP16 pair
    return static_cast<size_t>(bin_pitch(4 * K)) * A * kWin + static_cast<size_t>(A) * sizeof(float4);
}

// A null `vol` only sets the instance's dynamic-LDS limit (tp_prepare), so
// that later launches, possibly graph-captured, make no attribute call.
// `half_out`: FP16 output slices (FP16 rows only).
template <typename T, int K, int A>
hipError_t launch_bp_t(const GeoTables& g, const void* filt, int n_rows, float scale, void* vol, bool half_out,
                       int accumulate, size_t lds, hipStream_t st) {
    if constexpr (!std::is_same<T, __half>::value) {
        if (half_out) return hipErrorInvalidValue;
    }
    if (lds > 65536) {
        const void* fns[2] = {nullptr, nullptr};
        if constexpr (std::is_same<T, __half>::value) {
            fns[0] = reinterpret_cast<const void*>(k_backproject_h2<K, A, float>);
            fns[1] = reinterpret_cast<const void*>(k_backproject_h2<K, A, __half>);
        } else {
            fns[0] = reinterpret_cast<const void*>(k_backproject<T, K, A>);
        }
        for (const void* fn : fns) {
            if (!fn) continue;
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
            if (e != hipSuccess) return e;
        }
    }
    if (vol == nullptr) return hipSuccess;
    const dim3 grid(static_cast<unsigned>(g.nb * g.nb), static_cast<unsigned>((n_rows + K - 1) / K));
    if constexpr (std::is_same<T, __half>::value) {
        if (half_out)
            hipLaunchKernelGGL((k_backproject_h2<K, A, __half>), grid, dim3(kBpThreads), lds, st, g,
                               static_cast<const __half*>(filt), n_rows, scale, static_cast<__half*>(vol), accumulate);
        else
            hipLaunchKernelGGL((k_backproject_h2<K, A, float>), grid, dim3(kBpThreads), lds, st, g,
                               static_cast<const __half*>(filt), n_rows, scale, static_cast<float*>(vol), accumulate);
    } else {
        hipLaunchKernelGGL((k_backproject<T, K, A>), grid, dim3(kBpThreads), lds, st, g, static_cast<const T*>(filt),
                           n_rows, scale, static_cast<float*>(vol), accumulate);
    }
    return hipGetLastError();
}

template <typename T, int K>
hipError_t launch_bp_a(const GeoTables& g, const void* filt, int n_rows, float scale, void* vol, bool half_out,
                       int accumulate, int A, size_t lds, hipStream_t st) {
    switch (A) {
        case 8: return launch_bp_t<T, K, 8>(g, filt, n_rows, scale, vol, half_out, accumulate, lds, st);
        case 16: return launch_bp_t<T, K, 16>(g, filt, n_rows, scale, vol, half_out, accumulate, lds, st);
        case 32: return launch_bp_t<T, K, 32>(g, filt, n_rows, scale, vol, half_out, accumulate, lds, st);
        case 64: return launch_bp_t<T, K, 64>(g, filt, n_rows, scale, vol, half_out, accumulate, lds, st);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_bp_k(const GeoTables& g, const void* filt, int n_rows, float scale, void* vol, bool half_out,
                       int accumulate, int K, int A, size_t lds, hipStream_t st) {
    switch (K) {
        case 1: return launch_bp_a<T, 1>(g, filt, n_rows, scale, vol, half_out, accumulate, A, lds, st);
        case 2: return launch_bp_a<T, 2>(g, filt, n_rows, scale, vol, half_out, accumulate, A, lds, st);
        case 4: return launch_bp_a<T, 4>(g, filt, n_rows, scale, vol, half_out, accumulate, A, lds, st);
        case 8: return launch_bp_a<T, 8>(g, filt, n_rows, scale, vol, half_out, accumulate, A, lds, st);
        case 16: return launch_bp_a<T, 16>(g, filt, n_rows, scale, vol, half_out, accumulate, A, lds, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

size_t backproject_lds_bytes(tp_dtype dt, int slices_per_block, int angles_per_block) {
    return bp_lds_bytes(dt, slices_per_block, angles_per_block);
}

hipError_t prepare_backproject(tp_dtype dt, int slices_per_block, int angles_per_block) {
    GeoTables g{};
    return launch_backproject(g, nullptr, dt, 0, 0.0f, nullptr, TP_F32, 0, slices_per_block, angles_per_block,
                              nullptr);
}

hipError_t launch_backproject(const GeoTables& g, const void* filt, tp_dtype dt, int n_rows, float scale,
                              void* vol, tp_dtype vol_dt, int accumulate, int slices_per_block,
                              int angles_per_block, hipStream_t st) {
    const size_t lds = bp_lds_bytes(dt, slices_per_block, angles_per_block);
    const bool half_out = vol_dt == TP_F16;
    if (vol_dt != TP_F32 && !half_out) return hipErrorInvalidValue;
    switch (dt) {
        case TP_F32:
            return launch_bp_k<float>(g, filt, n_rows, scale, vol, half_out, accumulate, slices_per_block,
                                      angles_per_block, lds, st);
        case TP_F16:
            return launch_bp_k<__half>(g, filt, n_rows, scale, vol, half_out, accumulate, slices_per_block,
                                       angles_per_block, lds, st);
        case TP_BF16:
            return launch_bp_k<uint16_t>(g, filt, n_rows, scale, vol, half_out, accumulate, slices_per_block,
                                         angles_per_block, lds, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace tp
