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
// detector bins.  For a block of A angles, each wave stages whole angles: lane
// b loads bin ws + b of the K slices' filtered rows and writes them as one
// contiguous group, so LDS holds [angle][bin][slice] (bf16 widened to FP32;
// groups padded to an odd number of 16-byte bank groups).
// The window starts at ws = bi + floor(min over the tile corners of the
// FP32 offset); fma is monotone in each argument, so every voxel's floor
// lies in [0, 45) of the 48-bin window and both taps are staged.  The inner
// loop per voxel and angle: offset (1 FMA), fraction, floor, address, 1 - w,
// reads of the two bins' K-slice groups (16-byte LDS reads), then two
// FMAs per slice (v_fma_mix_f32 reads FP16 operands directly).  Every slice
// sums its angles in order, so results do not depend on K or A.
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
__device__ __forceinline__ float lds_val(const __half* v, int i) { return __half2float(v[i]); }

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

template <typename T, int K, int A>
__global__ void __launch_bounds__(kBpThreads)
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

// Forward projection, gather form.  Work-group: 4 waves = 4 neighbouring
// angles that sweep the same axis (the plan lists angles grouped by sweep
// axis and sorted), lanes = 64 consecutive detector bins, K slices.  Each bin
// sweeps the image along the axis the ray is closer to (rows when |cos| >=
// |sin|).  On each line the voxels whose coordinate can fall in [j-1, j+1)
// lie within 1/|c| <= sqrt(2) of the line's crossing point; a fixed window of
// kCand candidates starting just below it covers them with margin (the
// crossing point is an FP32 estimate good to ~1e-3 voxel), so every lane runs
// the same unrolled loop.  Each candidate's exact (j0, w) comes from the
// backprojector's expression with the angle's tile tables staged in LDS;
// weights are (1-w) for j0 == j, w for j0+1 == j, else 0.
// Lines are processed in blocks of radon_lines: the work-group stages the
// strip its 4 angles x 64 bins can touch on those lines (all K slices,
// [line][slice / 4][position] of float4, so a wave's read of one 4-slice
// chunk at its ~1.2-voxel-spaced positions touches near-consecutive 16-byte
// words) into LDS with coalesced loads, so each voxel is
// fetched once per work-group instead of once per bin and angle.  A strip
// wider than kRadonStrip (sparse angle sets) is read from global memory
// instead, with the same arithmetic and order.  No atomics: every output is
// summed by one lane, lines ascending, candidates ascending.
constexpr int kCand = 3;
// lines staged per block: 4, or 2 for 32 slices (keeps the strip at 32 KB,
// four work-groups per CU)
template <int K> constexpr int radon_lines() { return K >= 32 ? 2 : 4; }
constexpr int kRadonStrip = 128;
constexpr int W = 4;  // angles (waves) per work-group

// One line of the sweep for bin j: first candidate and the line's tile entries.
struct RadonLine {
    int lo, li;
    float lf, dm;
};

__device__ __forceinline__ RadonLine radon_line(int m, int j, int half, float cmin, float inv, float start,
                                                float center_f, const int2* tl) {
    RadonLine ln;
    const float um = static_cast<float>(m - half) * cmin + center_f;
    // first candidate: ceil of the window's left end (the window is
    // 2/|c| + 0.02 <= 2.85 voxels long, so 3 candidates cover it)
    ln.lo = -coord_floor(-__builtin_fmaf(static_cast<float>(j) - um, inv, start));
    const int2 e = tl[m >> 5];
    ln.li = e.x;
    ln.lf = __int_as_float(e.y);
    ln.dm = static_cast<float>(m & 31);
    return ln;
}

// Weight of candidate t of a line in bin j, from the backprojector's exact
// expression (bi = xi + yi, bf = xf + yf, then tile_offset): (1 - w) when
// floor lands on j, w when on j - 1, else 0.  vc: the clamped voxel index.
template <bool ROWS>
__device__ __forceinline__ float radon_weight(const RadonLine& ln, int t, int j, int N, float cs, float sn,
                                              const int2* tc, int& vc) {
    const int v = ln.lo + t;
    vc = min(max(v, 0), N - 1);
    const int bv = vc >> 5;
    const float dv = static_cast<float>(vc & 31);
    const int2 e = tc[bv];
    const int bi = e.x + ln.li;
    const float bf = __int_as_float(e.y) + ln.lf;
    const float s = ROWS ? tile_offset(dv, ln.dm, cs, sn, bf) : tile_offset(ln.dm, dv, cs, sn, bf);
    const int j0 = bi + coord_floor(s);
    const float w = coord_frac(s);
    const float wt = (j0 == j) ? 1.0f - w : ((j0 + 1 == j) ? w : 0.0f);
    return (v >= 0 && v < N) ? wt : 0.0f;
}

template <int K, bool ROWS>
__global__ void __launch_bounds__(64 * W)
k_radon(GeoTables g, const float* __restrict__ vol, int n_rows, float* __restrict__ sino) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_lo[W][4];
    const int nb = g.nb, na = g.na, N = g.N, half = N / 2;
    float4* strip = reinterpret_cast<float4*>(smem);                      // [lines][K / 4][kRadonStrip]
    constexpr int LINES = radon_lines<K>();
    int2* tabs = reinterpret_cast<int2*>(strip + LINES * (K / 4) * kRadonStrip);  // [W waves][2][nb]
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int jgroups = (g.n + 63) >> 6;
    const int jb = (blockIdx.x % jgroups) * 64;
    const int grp = blockIdx.x / jgroups;
    // this launch covers the angles that sweep rows (ROWS) or columns
    const int e0 = ROWS ? grp * W : g.n_rows_major + grp * W;
    const int e_end = ROWS ? min(g.n_rows_major, e0 + W) : min(g.n_order, e0 + W);
    if (g.order[e0] < 0) return;  // a group of padding only (whole work-group, before any barrier)
    const int e = e0 + wv;
    // padding entries (-1) and entries past the class are inactive waves
    const bool active = e < e_end && g.order[e] >= 0;
    const int a = active ? g.order[e] : g.order[e0];
    const int j = jb + lane;
    const int z0 = blockIdx.y * K;
    const int nz = min(K, n_rows - z0);
    // tables of this wave's angle: the candidate's tile (along the line) and
    // the line's tile, integer and fraction parts
    int2* tc = tabs + wv * 2 * nb;  // (integer, fraction bits) per tile
    int2* tl = tc + nb;
    for (int b = lane; b < nb; b += 64) {
        const int xi = g.xi[b * na + a], yi = g.yi[b * na + a];
        const int xf = __float_as_int(g.xf[b * na + a]), yf = __float_as_int(g.yf[b * na + a]);
        tc[b] = ROWS ? make_int2(xi, xf) : make_int2(yi, yf);
        tl[b] = ROWS ? make_int2(yi, yf) : make_int2(xi, xf);
    }
    const float cs = g.cs[a], sn = g.sn[a];
    const float cmaj = ROWS ? cs : sn;   // coefficient of the swept coordinate
    const float cmin = ROWS ? sn : cs;   // coefficient of the line coordinate
    const float inv = 1.0f / cmaj;
    // left end of the window of voxels whose coordinate can fall in [j-1, j+1)
    const float start = static_cast<float>(half) - 1.0f / fabsf(cmaj) - 0.01f;
    const int64_t slab = static_cast<int64_t>(N) * N;
    // a line is a row of the volume (ROWS) or of its transpose: contiguous
    const float* vz = vol + static_cast<int64_t>(z0) * slab;
    float acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0f;

    for (int m0 = 0; m0 < N; m0 += LINES) {
        const int mr = min(LINES, N - m0);
        // candidate starts at the block's corners (first/last bin, first/last line)
        if (lane < 4) {
            const int jj = min((lane & 1) ? jb + 63 : jb, g.n - 1);
            const int mm = (lane & 2) ? m0 + mr - 1 : m0;
            const float um = static_cast<float>(mm - half) * cmin + g.center_f;
            s_lo[wv][lane] = -coord_floor(-__builtin_fmaf(static_cast<float>(jj) - um, inv, start));
        }
        __syncthreads();
        int xmin = 1 << 30, xmax = -(1 << 30);
        for (int w = 0; w < W; ++w) {
            if (e0 + w >= e_end || g.order[e0 + w] < 0) continue;
            for (int c = 0; c < 4; ++c) {
                xmin = min(xmin, s_lo[w][c]);
                xmax = max(xmax, s_lo[w][c] + kCand - 1);
            }
        }
        xmin = max(xmin - 1, 0);  // one voxel of margin for the FP32 corner estimates
        xmax = min(xmax + 1, N - 1);
        const int width = xmax - xmin + 1;
        const bool staged = width > 0 && width <= kRadonStrip;
        if (staged) {
            // jobs of 64 positions of one line, spread over the waves
            constexpr int kChunks = kRadonStrip / 64;
            for (int job = wv; job < mr * kChunks; job += W) {
                const int r = job / kChunks;
                const int x = lane + 64 * (job - r * kChunks);
                if (x < width) {
                    const float* row = vz + static_cast<int64_t>(m0 + r) * N + xmin;
                    float v[K];
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        // slices past the last row re-read it (their sums are never
                        // stored); the opaque index keeps the offsets scalar, not hoisted
                        int kk = min(k, nz - 1);
                        asm volatile("" : "+s"(kk));
                        v[k] = row[x + kk * slab];
                    }
                    float4* dst = strip + r * (K / 4) * kRadonStrip + x;
#pragma unroll
                    for (int q = 0; q < K / 4; ++q) dst[q * kRadonStrip] = reinterpret_cast<const float4*>(v)[q];
                }
            }
        }
        __syncthreads();
        if (active && j < g.n) {
            // the staged and the global variant are separate loops, so the
            // uniform choice is not re-tested (and the sums not copied) per candidate
            if (staged) {
                for (int r = 0; r < mr; ++r) {
                    RadonLine ln = radon_line(m0 + r, j, half, cmin, inv, start, g.center_f, tl);
#pragma unroll
                    for (int t = 0; t < kCand; ++t) {
                        int vc;
                        const float wt = radon_weight<ROWS>(ln, t, j, N, cs, sn, tc, vc);
                        const int xo = min(max(vc - xmin, 0), kRadonStrip - 1);
                        const float4* src = strip + r * (K / 4) * kRadonStrip + xo;
                        float val[K];
#pragma unroll
                        for (int q = 0; q < K / 4; ++q) reinterpret_cast<float4*>(val)[q] = src[q * kRadonStrip];
                        // zero weights add exact zeros: no branch
#pragma unroll
                        for (int k = 0; k < K; ++k) acc[k] = __builtin_fmaf(wt, val[k], acc[k]);
                    }
                }
            } else {
                for (int r = 0; r < mr; ++r) {
                    const int m = m0 + r;
                    RadonLine ln = radon_line(m, j, half, cmin, inv, start, g.center_f, tl);
#pragma unroll
                    for (int t = 0; t < kCand; ++t) {
                        int vc;
                        const float wt = radon_weight<ROWS>(ln, t, j, N, cs, sn, tc, vc);
                        if (wt != 0.0f) {
                            const float* p = vz + static_cast<int64_t>(m) * N + vc;
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                int kk = min(k, nz - 1);
                                asm volatile("" : "+s"(kk));
                                acc[k] = __builtin_fmaf(wt, p[kk * slab], acc[k]);
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (active && j < g.n) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (k < nz) sino[(static_cast<int64_t>(z0 + k) * na + a) * g.n + j] = acc[k];
    }
}

size_t bp_lds_bytes(tp_dtype dt, int K, int A) {
    const int elem = (dt == TP_F16) ? 2 : 4;  // bf16 is widened to FP32 in LDS
    return static_cast<size_t>(bin_pitch(elem * K)) * A * kWin + static_cast<size_t>(A) * sizeof(float4);
}

template <typename T, int K, int A>
hipError_t launch_bp_t(const GeoTables& g, const void* filt, int n_rows, float scale, float* vol,
                       int accumulate, size_t lds, hipStream_t st) {
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_backproject<T, K, A>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    const dim3 grid(static_cast<unsigned>(g.nb * g.nb), static_cast<unsigned>((n_rows + K - 1) / K));
    hipLaunchKernelGGL((k_backproject<T, K, A>), grid, dim3(kBpThreads), lds, st, g, static_cast<const T*>(filt),
                       n_rows, scale, vol, accumulate);
    return hipGetLastError();
}

template <typename T, int K>
hipError_t launch_bp_a(const GeoTables& g, const void* filt, int n_rows, float scale, float* vol,
                       int accumulate, int A, size_t lds, hipStream_t st) {
    switch (A) {
        case 8: return launch_bp_t<T, K, 8>(g, filt, n_rows, scale, vol, accumulate, lds, st);
        case 16: return launch_bp_t<T, K, 16>(g, filt, n_rows, scale, vol, accumulate, lds, st);
        case 32: return launch_bp_t<T, K, 32>(g, filt, n_rows, scale, vol, accumulate, lds, st);
        case 64: return launch_bp_t<T, K, 64>(g, filt, n_rows, scale, vol, accumulate, lds, st);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_bp_k(const GeoTables& g, const void* filt, int n_rows, float scale, float* vol,
                       int accumulate, int K, int A, size_t lds, hipStream_t st) {
    switch (K) {
        case 1: return launch_bp_a<T, 1>(g, filt, n_rows, scale, vol, accumulate, A, lds, st);
        case 2: return launch_bp_a<T, 2>(g, filt, n_rows, scale, vol, accumulate, A, lds, st);
        case 4: return launch_bp_a<T, 4>(g, filt, n_rows, scale, vol, accumulate, A, lds, st);
        case 8: return launch_bp_a<T, 8>(g, filt, n_rows, scale, vol, accumulate, A, lds, st);
        case 16: return launch_bp_a<T, 16>(g, filt, n_rows, scale, vol, accumulate, A, lds, st);
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

namespace {

// out[z][x][y] = in[z][y][x] for N x N slices: 64 x 64 tiles through LDS
// (65-float rows, so the transposed reads do not share banks), coalesced
// reads and writes.
__global__ void __launch_bounds__(256) k_transpose(const float* __restrict__ in, float* __restrict__ out, int N) {
    __shared__ float t[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int x0 = blockIdx.x * 64, y0 = blockIdx.y * 64;
    const int64_t slab = static_cast<int64_t>(N) * N;
    const float* src = in + blockIdx.z * slab;
    float* dst = out + blockIdx.z * slab;
    for (int r = ty; r < 64; r += 4) {
        const int y = y0 + r, x = x0 + tx;
        if (y < N && x < N) t[r][tx] = src[static_cast<int64_t>(y) * N + x];
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int x = x0 + r, y = y0 + tx;
        if (y < N && x < N) dst[static_cast<int64_t>(x) * N + y] = t[tx][r];
    }
}

template <int K, bool ROWS>
hipError_t launch_radon_k(const GeoTables& g, const float* vol, int n_rows, float* sino, hipStream_t st) {
    const int jgroups = (g.n + 63) / 64;
    const int groups = ROWS ? (g.n_rows_major + W - 1) / W : (g.n_order - g.n_rows_major + W - 1) / W;
    if (groups == 0) return hipSuccess;
    const size_t lds = sizeof(float) * radon_lines<K>() * K * kRadonStrip +
                       sizeof(int2) * 2 * W * static_cast<size_t>(g.nb);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_radon<K, ROWS>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    const dim3 grid(static_cast<unsigned>(jgroups * groups), static_cast<unsigned>((n_rows + K - 1) / K));
    hipLaunchKernelGGL((k_radon<K, ROWS>), grid, dim3(64 * W), lds, st, g, vol, n_rows, sino);
    return hipGetLastError();
}

template <int K>
hipError_t launch_radon_both(const GeoTables& g, const float* vol, const float* volT, int n_rows, float* sino,
                             hipStream_t st) {
    hipError_t e = launch_radon_k<K, true>(g, vol, n_rows, sino, st);
    if (e != hipSuccess) return e;
    return launch_radon_k<K, false>(g, volT, n_rows, sino, st);
}

}  // namespace

size_t radon_workspace_bytes(const GeoTables& g, int n_rows) {
    return g.n_rows_major < g.n_order ? sizeof(float) * static_cast<size_t>(n_rows) * g.N * g.N : 0;
}

// Angles that sweep columns (|sin| > |cos|) read a transposed copy of the
// volume, so their lines are contiguous too.  32 slices per work-group
// amortise each candidate's coordinate; smaller chunks use 16 or 8.
hipError_t launch_radon(const GeoTables& g, const float* vol, int n_rows, float* sino, float* workspace,
                        hipStream_t st) {
    const float* volT = vol;
    if (g.n_rows_major < g.n_order) {
        const dim3 tg(static_cast<unsigned>((g.N + 63) / 64), static_cast<unsigned>((g.N + 63) / 64),
                      static_cast<unsigned>(n_rows));
        hipLaunchKernelGGL(k_transpose, tg, dim3(256), 0, st, vol, workspace, g.N);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        volT = workspace;
    }
    if (n_rows > 16) return launch_radon_both<32>(g, vol, volT, n_rows, sino, st);
    return n_rows > 8 ? launch_radon_both<16>(g, vol, volT, n_rows, sino, st)
                      : launch_radon_both<8>(g, vol, volT, n_rows, sino, st);
}

}  // namespace tp
