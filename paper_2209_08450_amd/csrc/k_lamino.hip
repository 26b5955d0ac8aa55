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
// tap is one 16-byte read and two FMAs across the columns.  The blocks of
// angles are software-pipelined: while a block is accumulated, the table
// entries of the block after next and the window samples of the next block
// (up to 4 kLamPre rows) are in flight into registers, and are written to
// LDS after the block's last read.  The column coordinate u is the
// backprojector's split expression (the plan's tile tables, integer + FP32
// fraction); the row coordinate v uses tables of the same split form per
// tile edge and per slice, so both keep FP32 precision at any detector size,
// and each slice's coordinates are the same however the volume is split into
// calls.  Every LDS index is clamped into the staged window, which the window
// bounds (from the tile's corners, with one sample of margin) make a no-op.
#include <type_traits>

#include "tp_internal.h"

namespace tp {
namespace {

constexpr int kLamK = 8;      // slices per work-group
constexpr int kLamA = 4;      // angles staged per block
constexpr int kLamCols = 48;  // staged columns (also the row pitch of a window, in pairs)
constexpr int kLamRows = 64;  // staged rows (at most; a launch sizes its windows from the tilt)
constexpr int kLamPre = 8;  // window rows per lane loaded one block ahead (4 kLamPre = 32 rows)
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

// A stored sample as loaded (its bits, zero-extended to 32), and its value:
// the conversion is deferred so loads issued a block ahead are not waited for.
__device__ __forceinline__ uint32_t lam_raw(const float* p) { return __float_as_uint(*p); }
__device__ __forceinline__ uint32_t lam_raw(const __half* p) { return __half_as_ushort(*p); }
__device__ __forceinline__ uint32_t lam_raw(const uint16_t* p) { return *p; }
template <typename TI> __device__ __forceinline__ float lam_value(uint32_t r);
template <> __device__ __forceinline__ float lam_value<float>(uint32_t r) { return __uint_as_float(r); }
template <> __device__ __forceinline__ float lam_value<__half>(uint32_t r) {
    return __half2float(__ushort_as_half(static_cast<unsigned short>(r)));
}
template <> __device__ __forceinline__ float lam_value<uint16_t>(uint32_t r) { return __uint_as_float(r << 16); }

// One angle's per-tile table entries, as loaded (summed when used, so the
// loads of the next block can be in flight during this block's compute).
struct LamEntry {
    float cs, sn, dvx, dvy, xf, yf, vxf, vyf;
    int xi, yi, vxi, vyi;
};

__device__ __forceinline__ LamEntry lam_entry(const GeoTables& g, const LaminoTables& t, int bx, int by, int a) {
    LamEntry e;
    const int na = g.na;
    e.cs = g.cs[a];
    e.sn = g.sn[a];
    e.dvx = t.dvdx[a];
    e.dvy = t.dvdy[a];
    e.xi = g.xi[bx * na + a];
    e.yi = g.yi[by * na + a];
    e.xf = g.xf[bx * na + a];
    e.yf = g.yf[by * na + a];
    e.vxi = t.vxi[bx * na + a];
    e.vyi = t.vyi[by * na + a];
    e.vxf = t.vxf[bx * na + a];
    e.vyf = t.vyf[by * na + a];
    return e;
}

// Three work-groups per CU is what the windows' LDS allows at mid tilts, so
// the kernel may use the registers of three waves per SIMD (168 VGPRs): the
// next block's window is held in registers while the current one is used.
template <typename TI>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_lamino(GeoTables g, LaminoTables t, const TI* __restrict__ filt, int z0, int nz, float scale,
         float* __restrict__ vol, int wrows, int nzb) {
    // [kLamA][wrows][kLamCols] elements: windows of wrows rows (sized from the
    // tilt by the launcher).  An element is the pair (sample at column c,
    // sample at c + 1): for FP16 projections the two raw FP16 values (4 bytes,
    // interpolated by mixed-precision FMAs), otherwise the FP32 sample and the
    // difference to the next (8 bytes).
    constexpr bool kH = std::is_same<TI, __half>::value;
    using WinT = typename std::conditional<kH, uint32_t, float2>::type;
    extern __shared__ float win_mem[];
    // per-angle window parameters, double-buffered by block parity: the next
    // block's are written while the current block's are read
    __shared__ int s_ci[2][kLamA], s_ri[2][kLamA], s_nr[2][kLamA];  // window origin (column, row), rows staged
    __shared__ int s_ui[2][kLamA];                                  // integer part of the tile origin's u
    __shared__ float s_uf[2][kLamA];                                // its FP32 fraction
    __shared__ float s_cs[2][kLamA], s_sn[2][kLamA], s_dvx[2][kLamA], s_dvy[2][kLamA];
    // each slice's row coordinate in the window at the tile origin: fractions
    // of the slice and the tile origin, plus the slice's integer offset into
    // the window (a sum rounded in FP32, the same for a slice in any call
    // since its block is fixed)
    __shared__ float s_cz[2][kLamA][kLamK];
    const int nb = g.nb, na = g.na, N = g.N, n = g.n;
    // Work item of this work-group: the hardware hands work-group ids to the
    // XCDs round robin, and the remap gives each XCD a contiguous range of
    // work items, ordered slice block first, so the slice blocks of one tile
    // run together on one XCD and share their overlapping windows in its L2.
    const int w = lamino_work_item(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
    const int tile = w / nzb;
    const int bx = tile % nb, by = tile / nb;
    // slice blocks are aligned to multiples of kLamK in the whole volume, so a
    // slice's block, window and arithmetic do not depend on the call's range
    const int zs = (z0 / kLamK + (w - tile * nzb)) * kLamK;  // first slice of this block (absolute)
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const float dx = static_cast<float>(tx);
    // each slice's own row term (integer + fraction) from the per-slice table,
    // so a slice's coordinates do not depend on how the volume is split
    float fz[kLamK];
    int iz[kLamK];
#pragma unroll
    for (int k = 0; k < kLamK; ++k) {
        const int z = min(zs + k, t.Nz - 1);  // slices outside the call's range are computed, never stored
        fz[k] = t.vzf[z];
        iz[k] = t.vzi[z];
    }
    float acc[4][kLamK];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < kLamK; ++k) acc[i][k] = 0.0f;

    // the staging wave's angle (scalar) and its lane's place in the 4 x 16 lane grid
    const int sj = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63, lr = lane >> 4, lc = lane & 15;
    // source lane of the next column: (lc + 1) mod 16 in the same row group
    const int nbr_lane = (lr << 4) | ((lc + 1) & 15);

    // Setup threads (the first kLamA of wave 0) hold the table entries of the
    // next block, loaded one block ahead.
    LamEntry ent{};
    if (threadIdx.x < kLamA && static_cast<int>(threadIdx.x) < na) ent = lam_entry(g, t, bx, by, threadIdx.x);

    // Window bounds of block b0 (angles b0 .. b0 + cnt - 1) from the held
    // entries into parameter buffer `buf`, then the entries of the block after.
    auto setup = [&](int b0, int buf) {
        const int cnt = min(kLamA, na - b0);
        if (static_cast<int>(threadIdx.x) < cnt) {
            const int ui = ent.xi + ent.yi, vi = ent.vxi + ent.vyi;
            const float uf = ent.xf + ent.yf, vf = ent.vxf + ent.vyf;
            // extremes of the in-tile offsets over the tile's corners, per slice
            const float umin = fminf(0.0f, 31.0f * ent.cs) + fminf(0.0f, 31.0f * ent.sn);
            const float vmin = fminf(0.0f, 31.0f * ent.dvx) + fminf(0.0f, 31.0f * ent.dvy);
            const float vmax = fmaxf(0.0f, 31.0f * ent.dvx) + fmaxf(0.0f, 31.0f * ent.dvy);
            int lo = 1 << 30, hi = -(1 << 30);
#pragma unroll
            for (int k = 0; k < kLamK; ++k) {
                lo = min(lo, iz[k] + coord_floor(vf + fz[k] + vmin));
                hi = max(hi, iz[k] + coord_floor(vf + fz[k] + vmax));
            }
            const int ri = vi + lo - 1;
            const int rhi = vi + hi + 2;
            const int q = threadIdx.x;
#pragma unroll
            for (int k = 0; k < kLamK; ++k) s_cz[buf][q][k] = (vf + fz[k]) + static_cast<float>(vi - ri + iz[k]);
            s_ci[buf][q] = ui + coord_floor(uf + umin) - 1;
            s_ri[buf][q] = ri;
            s_nr[buf][q] = min(rhi - ri + 1, wrows);
            s_ui[buf][q] = ui;
            s_uf[buf][q] = uf;
            s_cs[buf][q] = ent.cs;
            s_sn[buf][q] = ent.sn;
            s_dvx[buf][q] = ent.dvx;
            s_dvy[buf][q] = ent.dvy;
            const int an = b0 + kLamA + q;
            if (an < na) ent = lam_entry(g, t, bx, by, an);
        }
    };

    // Window staging of wave sj's angle of the block whose parameters are in
    // `buf`: lane (lr, lc) covers columns lc + 16 m (m < 3) of rows lr + 4 p.
    // The first kLamPre rows per lane are loaded into registers by issue()
    // (no wait) and written by store(); rows past 4 kLamPre (small tilts
    // only) are loaded and written by store() itself.  Every load reads an
    // in-bounds sample; an element off the detector is replaced by zero.
    uint32_t X[kLamPre][3];
    auto col_of = [&](int c0, int m, bool* in) {
        const int c = c0 + lc + 16 * m;
        *in = c >= 0 && c < n;
        return *in ? c : 0;
    };
    auto issue = [&](int b0, int buf) {
        if (sj < min(kLamA, na - b0)) {
            const int nr = s_nr[buf][sj], r0 = s_ri[buf][sj], c0 = s_ci[buf][sj];
            const TI* img = filt + static_cast<int64_t>(b0 + sj) * t.rows * n;
            int col[3];
            bool cin[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) col[m] = col_of(c0, m, &cin[m]);
#pragma unroll
            for (int p = 0; p < kLamPre; ++p) {
                const int rr = lr + 4 * p, row = r0 + rr;
                const bool rin = rr < nr && row >= 0 && row < t.rows;
                // rows * n < 2^31 (checked by the host): 32-bit offsets from the image's base
                const unsigned base = rin ? static_cast<unsigned>(row * n) : 0u;
#pragma unroll
                for (int m = 0; m < 3; ++m) X[p][m] = lam_raw(img + (base + static_cast<unsigned>(col[m])));
            }
        }
    };
    // one row of the window: masked values v[m] at columns lc + 16 m; the
    // next column's value comes from the neighbouring lane (lane 15 of a row
    // group takes lane 0's next chunk; column kLamCols, never read, gets 0)
    auto put_row_h = [&](uint32_t* wrow, const uint32_t v[3], bool store) {
        const uint32_t s0 = __shfl(static_cast<int>(v[0]), nbr_lane), s1 = __shfl(static_cast<int>(v[1]), nbr_lane),
                       s2 = __shfl(static_cast<int>(v[2]), nbr_lane);
        const bool wrap = lc == 15;
        const uint32_t n0 = wrap ? s1 : s0, n1 = wrap ? s2 : s1, n2 = wrap ? v[2] : s2;
        if (store) {
            wrow[0] = v[0] | (n0 << 16);
            wrow[16] = v[1] | (n1 << 16);
            wrow[32] = v[2] | (n2 << 16);
        }
    };
    auto put_row = [&](float2* wrow, const float v[3], bool store) {
        const float s0 = __shfl(v[0], nbr_lane), s1 = __shfl(v[1], nbr_lane), s2 = __shfl(v[2], nbr_lane);
        const bool wrap = lc == 15;
        const float n0 = wrap ? s1 : s0, n1 = wrap ? s2 : s1, n2 = wrap ? v[2] : s2;
        if (store) {
            wrow[0] = make_float2(v[0], n0 - v[0]);
            wrow[16] = make_float2(v[1], n1 - v[1]);
            wrow[32] = make_float2(v[2], n2 - v[2]);
        }
    };
    auto store = [&](int b0, int buf) {
        if (sj < min(kLamA, na - b0)) {
            const int nr = s_nr[buf][sj], r0 = s_ri[buf][sj], c0 = s_ci[buf][sj];
            bool cin[3];
            int col[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) col[m] = col_of(c0, m, &cin[m]);
            WinT* wj = reinterpret_cast<WinT*>(win_mem) + sj * wrows * kLamCols + lc;
#pragma unroll
            for (int p = 0; p < kLamPre; ++p) {
                const int rr = lr + 4 * p, row = r0 + rr;
                const bool rin = rr < nr && row >= 0 && row < t.rows;
                if constexpr (kH) {
                    uint32_t v[3];  // raw FP16 bits, zero (+0.0) off the detector
#pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        asm volatile("" : "+v"(X[p][m]));
                        v[m] = (rin && cin[m]) ? X[p][m] : 0u;
                    }
                    put_row_h(wj + rr * kLamCols, v, rr < nr);
                } else {
                    float v[3];
#pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        asm volatile("" : "+v"(X[p][m]));
                        v[m] = (rin && cin[m]) ? lam_value<TI>(X[p][m]) : 0.0f;
                    }
                    put_row(wj + rr * kLamCols, v, rr < nr);
                }
            }
            if (nr > 4 * kLamPre) {  // wave-uniform
                const TI* img = filt + static_cast<int64_t>(b0 + sj) * t.rows * n;
                for (int rr = lr + 4 * kLamPre; rr - lr < nr; rr += 4) {
                    const int row = r0 + rr;
                    const bool rin = rr < nr && row >= 0 && row < t.rows;
                    const unsigned base = rin ? static_cast<unsigned>(row * n) : 0u;
                    if constexpr (kH) {
                        uint32_t v[3];
#pragma unroll
                        for (int m = 0; m < 3; ++m) {
                            const uint32_t x = lam_raw(img + (base + static_cast<unsigned>(col[m])));
                            v[m] = (rin && cin[m]) ? x : 0u;
                        }
                        put_row_h(wj + rr * kLamCols, v, rr < nr);
                    } else {
                        float v[3];
#pragma unroll
                        for (int m = 0; m < 3; ++m) {
                            const float x = load_as_float(img + (base + static_cast<unsigned>(col[m])), 0);
                            v[m] = (rin && cin[m]) ? x : 0.0f;
                        }
                        put_row(wj + rr * kLamCols, v, rr < nr);
                    }
                }
            }
        }
    };

    // prologue: block 0's parameters and window
    setup(0, 0);
    __syncthreads();
    issue(0, 0);
    store(0, 0);
    __syncthreads();
    for (int a0 = 0; a0 < na; a0 += kLamA) {
        const int cur = (a0 / kLamA) & 1, nxt = cur ^ 1;
        const int cnt = min(kLamA, na - a0);
        const bool more = a0 + kLamA < na;  // uniform
        if (more) {
            setup(a0 + kLamA, nxt);
            __syncthreads();  // the next block's parameters are visible
            issue(a0 + kLamA, nxt);
        }
        for (int j = 0; j < cnt; ++j) {
            const float cs = s_cs[cur][j], sn = s_sn[cur][j], dvx = s_dvx[cur][j], dvy = s_dvy[cur][j];
            const int ubase = s_ui[cur][j] - s_ci[cur][j];
            // the largest row index a bilinear read may start at; the unsigned
            // clamp also sends a negative index there (reads stay in the window)
            const unsigned rmax = static_cast<unsigned>(s_nr[cur][j] - 2);
            const float uf = s_uf[cur][j];
            float cz[kLamK];
#pragma unroll
            for (int k = 0; k < kLamK; ++k) cz[k] = s_cz[cur][j][k];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float dy = static_cast<float>(ty + 8 * i);
                const float u = tile_offset(dx, dy, cs, sn, uf);
                const int c = min(max(coord_floor(u) + ubase, 0), kLamCols - 2);
                const float wu = coord_frac(u);
                const float va = __builtin_fmaf(dx, dvx, dy * dvy);  // the voxel's in-tile row offset
                // byte offset of (angle j, row 0, column c) in the windows
                const unsigned cb = static_cast<unsigned>((j * wrows * kLamCols + c) * sizeof(WinT));
                // all slices' reads first, then the arithmetic, so the LDS
                // reads of a voxel column are in flight together
                WinT e0[kLamK], e1[kLamK];
                float wv[kLamK];
#pragma unroll
                for (int k = 0; k < kLamK; ++k) {
                    const float v = va + cz[k];  // row in the window
                    const unsigned r = min(static_cast<unsigned>(coord_floor(v)), rmax);
                    wv[k] = coord_frac(v);
                    const WinT* p = reinterpret_cast<const WinT*>(
                        reinterpret_cast<const char*>(win_mem) + (__umul24(r, kLamCols * sizeof(WinT)) + cb));
                    e0[k] = p[0];
                    e1[k] = p[kLamCols];
                }
#pragma unroll
                for (int k = 0; k < kLamK; ++k) {
                    float top, bot;
                    if constexpr (kH) {
                        // (1 - wu) q0 + wu q1 from the raw FP16 pair, in FP32
                        __half2 h0, h1;
                        __builtin_memcpy(&h0, &e0[k], sizeof(h0));
                        __builtin_memcpy(&h1, &e1[k], sizeof(h1));
                        top = __builtin_fmaf(wu, __high2float(h0), __builtin_fmaf(-wu, __low2float(h0), __low2float(h0)));
                        bot = __builtin_fmaf(wu, __high2float(h1), __builtin_fmaf(-wu, __low2float(h1), __low2float(h1)));
                    } else {
                        top = __builtin_fmaf(wu, e0[k].y, e0[k].x);
                        bot = __builtin_fmaf(wu, e1[k].y, e1[k].x);
                    }
                    acc[i][k] += __builtin_fmaf(wv[k], bot - top, top);
                }
            }
        }
        if (more) {
            __syncthreads();  // this block's windows are no longer read
            store(a0 + kLamA, nxt);
            __syncthreads();  // the next block's windows are visible
        }
    }
    const int x = bx * 32 + tx;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = by * 32 + ty + 8 * i;
#pragma unroll
        for (int k = 0; k < kLamK; ++k) {
            const int zl = zs + k - z0;  // index in the call's output
            if (x < N && y < N && zl >= 0 && zl < nz)
                vol[(static_cast<int64_t>(zl) * N + y) * N + x] = scale * acc[i][k];
        }
    }
}

template <typename TI>
hipError_t launch_lamino_t(const GeoTables& g, const LaminoTables& t, const void* filt, int z0, int nz, float scale,
                           float* vol, hipStream_t st) {
    const int nzb = (z0 + nz - 1) / kLamK - z0 / kLamK + 1;  // blocks aligned to multiples of kLamK
    const dim3 grid(static_cast<unsigned>(static_cast<int64_t>(g.nb) * g.nb * nzb));  // < 2^31 (checked by the host)
    // rows a tile's window can span: 31 sqrt(2) |cos phi| + (kLamK - 1) sin phi, plus the second tap,
    // the one-row margins on both sides and FP32 slack
    const float span = 31.0f * 1.41421356f * fabsf(t.dvdcos) + (kLamK - 1) * t.dvdz;
    const int wrows = min(kLamRows, static_cast<int>(span) + 6);
    const size_t elem = std::is_same<TI, __half>::value ? sizeof(uint32_t) : sizeof(float2);  // window element
    const size_t lds = elem * kLamA * wrows * kLamCols;
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
