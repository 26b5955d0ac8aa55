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
// the tile's voxels can reach (at most kLamRows rows x kLamCols columns:
// the column range of a 32-voxel tile is < 31 sqrt(2) + 2, the row range
// < 31 sqrt(2) |cos phi| + (kLamK - 1) sin phi + 2) is staged in LDS as FP32.
// The column coordinate u is the backprojector's split expression (the plan's
// tile tables, integer + FP32 fraction); the row coordinate v uses tables of
// the same split form per tile edge and per slice, so both keep FP32
// precision at any detector size, and each slice's coordinates are the same
// however the volume is split into calls.  Every LDS index is clamped into the staged
// window, which the window bounds (from the tile's corners, with one sample
// of margin) make a no-op.
#include "tp_internal.h"

namespace tp {
namespace {

constexpr int kLamK = 4;      // slices per work-group
constexpr int kLamA = 4;      // angles staged per block
constexpr int kLamCols = 48;  // staged columns
constexpr int kLamRows = 64;  // staged rows (at most)

template <typename TI>
__global__ void __launch_bounds__(256)
k_lamino(GeoTables g, LaminoTables t, const TI* __restrict__ filt, int z0, int nz, float scale,
         float* __restrict__ vol) {
    __shared__ float win[kLamA][kLamRows][kLamCols];
    __shared__ int s_ci[kLamA], s_ri[kLamA], s_nr[kLamA];   // window origin (column, row), rows staged
    __shared__ int s_ui[kLamA], s_vi[kLamA];                // integer parts of the tile origin's u, v (x, y terms)
    __shared__ float s_uf[kLamA], s_vf[kLamA];              // FP32 fractions of the same
    const int nb = g.nb, na = g.na, N = g.N, n = g.n;
    const int bx = blockIdx.x % nb, by = blockIdx.x / nb;
    const int zl0 = blockIdx.y * kLamK;         // first slice of this block, relative to z0
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
            s_nr[threadIdx.x] = min(rhi - ri + 1, kLamRows);
            s_ui[threadIdx.x] = ui;
            s_uf[threadIdx.x] = uf;
            s_vi[threadIdx.x] = vi;
            s_vf[threadIdx.x] = vf;
        }
        __syncthreads();
        // stage the windows: rows r < nr, all kLamCols columns (zeros off the detector)
        for (int j = 0; j < cnt; ++j) {
            const int a = a0 + j;
            const int nr = s_nr[j], r0 = s_ri[j], c0 = s_ci[j];
            const TI* img = filt + static_cast<int64_t>(a) * t.rows * n;
            for (int e = threadIdx.x; e < nr * kLamCols; e += blockDim.x) {
                const int r = e / kLamCols, c = e - r * kLamCols;
                const int row = r0 + r, col = c0 + c;
                float v = 0.0f;
                if (row >= 0 && row < t.rows && col >= 0 && col < n)
                    v = load_as_float(img, static_cast<int64_t>(row) * n + col);
                win[j][r][c] = v;
            }
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const int a = a0 + j;
            const float cs = g.cs[a], sn = g.sn[a], dvx = t.dvdx[a], dvy = t.dvdy[a];
            const int ubase = s_ui[j] - s_ci[j], vbase = s_vi[j] - s_ri[j], nr = s_nr[j];
            const float uf = s_uf[j], vf = s_vf[j];
            float cz[kLamK];  // the slice's row fraction plus the tile origin's (uniform)
#pragma unroll
            for (int k = 0; k < kLamK; ++k) cz[k] = vf + fz[k];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float dy = static_cast<float>(ty + 8 * i);
                const float u = tile_offset(dx, dy, cs, sn, uf);
                const int c = min(max(coord_floor(u) + ubase, 0), kLamCols - 2);
                const float wu = coord_frac(u);
                const float va = __builtin_fmaf(dx, dvx, dy * dvy);  // the voxel's in-tile row offset
#pragma unroll
                for (int k = 0; k < kLamK; ++k) {
                    const float v = va + cz[k];
                    const int r = min(max(coord_floor(v) + vbase + iz[k], 0), nr - 2);
                    const float wv = coord_frac(v);
                    const float q00 = win[j][r][c], q01 = win[j][r][c + 1];
                    const float q10 = win[j][r + 1][c], q11 = win[j][r + 1][c + 1];
                    const float top = __builtin_fmaf(wu, q01 - q00, q00);
                    const float bot = __builtin_fmaf(wu, q11 - q10, q10);
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
    const dim3 grid(static_cast<unsigned>(g.nb * g.nb), static_cast<unsigned>((nz + kLamK - 1) / kLamK));
    hipLaunchKernelGGL((k_lamino<TI>), grid, dim3(256), 0, st, g, t, static_cast<const TI*>(filt), z0, nz, scale, vol);
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
