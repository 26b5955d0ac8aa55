// Laminographic backprojection (paper, Section 2.2: the direct line-integral
// backprojector is kept because it also serves laminographic geometry, where
// the rotation axis is tilted with respect to the beam).
//
// Geometry: axis tilted by phi from the beam (phi = pi/2 is tomography); the
// voxel (x, y, z) is seen at detector column and row
//   u = x cos(theta) + y sin(theta) + center_u
//   v = (-x sin(theta) + y cos(theta)) cos(phi) + z sin(phi) + center_v
// and the volume is scale * sum over angles of the bilinear interpolation of
// the filtered projection at (v, u), zero off the detector.
//
// Work-group: a 32 x 32 tile of (x, y) voxels and kLamK consecutive slices;
// thread (tx, ty) owns voxels (tx, ty + 8 i), i < 4, of every slice.  Angles
// are processed kLamA at a time: for each, the window of the projection that
// the tile's voxels can reach (kLamCols columns: the column range of a
// 32-voxel tile is < 31 sqrt(2) + 2; and at most 31 sqrt(2) |cos phi| +
// (kLamK - 1) sin phi + 6 rows, sized per launch from the tilt) is staged in
// LDS as FP32 pairs (sample, next column's sample minus it), so a bilinear
// tap is one 16-byte read and two FMAs across the columns.  The column
// coordinate u is the backprojector's split expression (the plan's tile
// tables, integer + FP32 fraction); the row coordinate v uses tables of the
// same split form per tile edge and per slice, so both keep FP32 precision at
// any detector size, and each slice's coordinates are the same however the
// volume is split into calls.  Every LDS index is clamped into the staged
// window, which the window bounds (from the tile's corners, with one sample
// of margin) make a no-op.
#include "tp_internal.h"

namespace tp {
namespace {

constexpr int kLamK = 8;      // slices per work-group
constexpr int kLamA = 4;      // angles staged per block
constexpr int kLamCols = 48;  // staged columns
constexpr int kLamRows = 64;  // staged rows (at most; a launch sizes its windows from the tilt)
constexpr int kLamRowBatch = 3;  // window rows whose loads a lane issues before it waits
static_assert(kLamA * 64 == 256, "one wave of the 256-thread work-group stages each angle's window");

constexpr int kXcds = 8;  // XCDs of the chip (work-group ids go to them round robin)

// Bijection of [0, total): work-group id b runs on XCD b % kXcds as that
// XCD's (b / kXcds)-th work-group; XCD x receives items
// [x q + min(x, r), ...) of the q = total / kXcds (+1 for x < r) it runs.
__device__ __forceinline__ int lamino_work_item(int b, int total) {
    const int q = total / kXcds, r = total - q * kXcds;
    const int x = b % kXcds, s = b / kXcds;
    return x * q + min(x, r) + s;
}

template <typename TI>
__global__ void __launch_bounds__(256)
k_lamino(GeoTables g, LaminoTables t, const TI* __restrict__ filt, int z0, int nz, float scale,
         float* __restrict__ vol, int wrows, int nzb) {
    // [kLamA][wrows][kLamCols] float2: windows of wrows rows (sized from the tilt by the launcher)
    extern __shared__ float win_mem[];
    __shared__ int s_ci[kLamA], s_ri[kLamA], s_nr[kLamA];   // window origin (column, row), rows staged
    __shared__ int s_ui[kLamA], s_vi[kLamA];                // integer parts of the tile origin's u, v (x, y terms)
    __shared__ float s_uf[kLamA], s_vf[kLamA];              // FP32 fractions of the same
    const int nb = g.nb, na = g.na, N = g.N, n = g.n;
    // Work item of this work-group: the hardware hands work-group ids to the
    // XCDs round robin, and the remap gives each XCD a contiguous range of
    // work items, ordered slice block first, so the slice blocks of one tile
    // run together on one XCD and share their overlapping windows in its L2.
    const int w = lamino_work_item(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
    const int tile = w / nzb;
    const int bx = tile % nb, by = tile / nb;
    const int zl0 = (w - tile * nzb) * kLamK;   // first slice of this block, relative to z0
    const int zs = z0 + zl0;                    // ... and absolute in the volume
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const float dx = static_cast<float>(tx);
    // each slice's own row term (integer + fraction) from the per-slice table,
    // so a slice's coordinates do not depend on how the volume is split
    float fz[kLamK];
    int iz[kLamK];
#pragma unroll
    for (int k = 0; k < kLamK; ++k) {
        const int z = min(zs + k, t.Nz - 1);  // slices past the range are computed, never stored
        fz[k] = t.vzf[z];
        iz[k] = t.vzi[z];
    }
    float acc[4][kLamK];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < kLamK; ++k) acc[i][k] = 0.0f;

    for (int a0 = 0; a0 < na; a0 += kLamA) {
        const int cnt = min(kLamA, na - a0);
        __syncthreads();  // the previous block's windows are no longer read
        if (threadIdx.x < cnt) {
            const int a = a0 + threadIdx.x;
            const float cs = g.cs[a], sn = g.sn[a];
            const int ui = g.xi[bx * na + a] + g.yi[by * na + a];
            const float uf = g.xf[bx * na + a] + g.yf[by * na + a];
            const int vi = t.vxi[bx * na + a] + t.vyi[by * na + a];
            const float vf = t.vxf[bx * na + a] + t.vyf[by * na + a];
            const float dvx = t.dvdx[a], dvy = t.dvdy[a];
            // extremes of the in-tile offsets over the tile's corners, per slice
            const float umin = fminf(0.0f, 31.0f * cs) + fminf(0.0f, 31.0f * sn);
            const float vmin = fminf(0.0f, 31.0f * dvx) + fminf(0.0f, 31.0f * dvy);
            const float vmax = fmaxf(0.0f, 31.0f * dvx) + fmaxf(0.0f, 31.0f * dvy);
            const int ci = ui + coord_floor(uf + umin) - 1;
            int lo = 1 << 30, hi = -(1 << 30);
#pragma unroll
            for (int k = 0; k < kLamK; ++k) {
                lo = min(lo, iz[k] + coord_floor(vf + fz[k] + vmin));
                hi = max(hi, iz[k] + coord_floor(vf + fz[k] + vmax));
            }
            const int ri = vi + lo - 1;
            const int rhi = vi + hi + 2;
            s_ci[threadIdx.x] = ci;
            s_ri[threadIdx.x] = ri;
            s_nr[threadIdx.x] = min(rhi - ri + 1, wrows);
            s_ui[threadIdx.x] = ui;
            s_uf[threadIdx.x] = uf;
            s_vi[threadIdx.x] = vi;
            s_vf[threadIdx.x] = vf;
        }
        __syncthreads();
        // stage the windows: wave j stages angle j's rows r < nr as pairs
        // (sample at column c, sample at c + 1 minus it), c < kLamCols, zeros
        // off the detector.  Lane (lr, lc) = (lane / 16, lane % 16) stages
        // columns lc + 16 m (m < 3) of rows lr + 4 b.  Every load reads an
        // in-bounds sample (an element off the detector reads the image's
        // first one and is replaced by zero afterwards); the empty asm uses
        // make each load unconditional, so a batch of kLamRowBatch rows of
        // loads is issued before its first wait.
        {
            // the wave's angle, made scalar so the image base lives in scalar registers
            const int j = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
            const int lane = threadIdx.x & 63;
            if (j < cnt) {
                const int nr = s_nr[j], r0 = s_ri[j], c0 = s_ci[j];
                const TI* img = filt + static_cast<int64_t>(a0 + j) * t.rows * n;
                const int lr = lane >> 4, lc = lane & 15;
                int col[3][2];
                bool cin[3][2];
#pragma unroll
                for (int m = 0; m < 3; ++m)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int c = c0 + lc + 16 * m + h;
                        cin[m][h] = c >= 0 && c < n;
                        col[m][h] = cin[m][h] ? c : 0;
                    }
                float2* w = reinterpret_cast<float2*>(win_mem) + j * wrows * kLamCols + lc;
                for (int r = lr; r < nr; r += 4 * kLamRowBatch) {
                    float x[kLamRowBatch][3][2];
                    bool rin[kLamRowBatch];
#pragma unroll
                    for (int b = 0; b < kLamRowBatch; ++b) {
                        const int rr = r + 4 * b, row = r0 + rr;
                        rin[b] = rr < nr && row >= 0 && row < t.rows;
                        // rows * n < 2^31 (checked by the host): 32-bit offsets from the image's base
                        const unsigned base = rin[b] ? static_cast<unsigned>(row * n) : 0u;
#pragma unroll
                        for (int m = 0; m < 3; ++m)
#pragma unroll
                            for (int h = 0; h < 2; ++h)
                                x[b][m][h] = load_as_float(img + (base + static_cast<unsigned>(col[m][h])), 0);
                    }
#pragma unroll
                    for (int b = 0; b < kLamRowBatch; ++b)
#pragma unroll
                        for (int m = 0; m < 3; ++m)
#pragma unroll
                            for (int h = 0; h < 2; ++h) asm volatile("" : "+v"(x[b][m][h]));
#pragma unroll
                    for (int b = 0; b < kLamRowBatch; ++b) {
                        const int rr = r + 4 * b;
                        if (rr < nr) {
#pragma unroll
                            for (int m = 0; m < 3; ++m) {
                                const float v0 = (rin[b] && cin[m][0]) ? x[b][m][0] : 0.0f;
                                const float v1 = (rin[b] && cin[m][1]) ? x[b][m][1] : 0.0f;
                                w[rr * kLamCols + 16 * m] = make_float2(v0, v1 - v0);
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const int a = a0 + j;
            const float cs = g.cs[a], sn = g.sn[a], dvx = t.dvdx[a], dvy = t.dvdy[a];
            const int ubase = s_ui[j] - s_ci[j], vbase = s_vi[j] - s_ri[j];
            // the largest row index a bilinear read may start at; the unsigned
            // clamp also sends a negative index there (reads stay in the window)
            const unsigned rmax = static_cast<unsigned>(s_nr[j] - 2);
            const float uf = s_uf[j], vf = s_vf[j];
            float cz[kLamK];  // the slice's row fraction plus the tile origin's (uniform)
            int rb[kLamK];    // the slice's integer row offset into the window (uniform)
#pragma unroll
            for (int k = 0; k < kLamK; ++k) {
                cz[k] = vf + fz[k];
                rb[k] = vbase + iz[k];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float dy = static_cast<float>(ty + 8 * i);
                const float u = tile_offset(dx, dy, cs, sn, uf);
                const int c = min(max(coord_floor(u) + ubase, 0), kLamCols - 2);
                const float wu = coord_frac(u);
                const float va = __builtin_fmaf(dx, dvx, dy * dvy);  // the voxel's in-tile row offset
                // byte offset of (angle j, row 0, column c) in the windows
                const unsigned cb = static_cast<unsigned>((j * wrows * kLamCols + c) * sizeof(float2));
#pragma unroll
                for (int k = 0; k < kLamK; ++k) {
                    const float v = va + cz[k];
                    const unsigned r = min(static_cast<unsigned>(coord_floor(v) + rb[k]), rmax);
                    const float wv = coord_frac(v);
                    const float2* p = reinterpret_cast<const float2*>(
                        reinterpret_cast<const char*>(win_mem) + (__umul24(r, kLamCols * sizeof(float2)) + cb));
                    const float2 e0 = p[0], e1 = p[kLamCols];
                    const float top = __builtin_fmaf(wu, e0.y, e0.x);
                    const float bot = __builtin_fmaf(wu, e1.y, e1.x);
                    acc[i][k] += __builtin_fmaf(wv, bot - top, top);
                }
            }
        }
    }
    const int x = bx * 32 + tx;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = by * 32 + ty + 8 * i;
#pragma unroll
        for (int k = 0; k < kLamK; ++k) {
            const int zl = zl0 + k;
            if (x < N && y < N && zl < nz) vol[(static_cast<int64_t>(zl) * N + y) * N + x] = scale * acc[i][k];
        }
    }
}

template <typename TI>
hipError_t launch_lamino_t(const GeoTables& g, const LaminoTables& t, const void* filt, int z0, int nz, float scale,
                           float* vol, hipStream_t st) {
    const int nzb = (nz + kLamK - 1) / kLamK;
    const dim3 grid(static_cast<unsigned>(static_cast<int64_t>(g.nb) * g.nb * nzb));  // < 2^31 (checked by the host)
    // rows a tile's window can span: 31 sqrt(2) |cos phi| + (kLamK - 1) sin phi, plus the second tap,
    // the one-row margins on both sides and FP32 slack
    const float span = 31.0f * 1.41421356f * fabsf(t.dvdcos) + (kLamK - 1) * t.dvdz;
    const int wrows = min(kLamRows, static_cast<int>(span) + 6);
    const size_t lds = sizeof(float2) * kLamA * wrows * kLamCols;
    if (lds > 65536) {  // small tilts: windows above the default dynamic LDS limit (at most 96 KiB)
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_lamino<TI>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_lamino<TI>), grid, dim3(256), lds, st, g, t, static_cast<const TI*>(filt), z0, nz, scale,
                       vol, wrows, nzb);
    return hipGetLastError();
}

}  // namespace

int lamino_max_rows() { return kLamRows; }
int lamino_slices_per_block() { return kLamK; }

hipError_t launch_lamino(const GeoTables& g, const LaminoTables& t, const void* filt, tp_dtype dt, int z0, int nz,
                         float scale, float* vol, hipStream_t st) {
    switch (dt) {
        case TP_F32: return launch_lamino_t<float>(g, t, filt, z0, nz, scale, vol, st);
        case TP_F16: return launch_lamino_t<__half>(g, t, filt, z0, nz, scale, vol, st);
        case TP_BF16: return launch_lamino_t<uint16_t>(g, t, filt, z0, nz, scale, vol, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace tp
