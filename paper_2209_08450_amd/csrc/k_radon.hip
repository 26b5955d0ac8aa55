// Forward projector: the exact transpose of the linear-interpolation
// backprojector in k_backproject.hip (the iterative use of such a pair is
// named in the paper's Sections 1 and 5).  Each voxel's detector coordinate
// at an angle is the backprojector's split expression
//   s = bi + fma(dx, cos_a, fma(dy, sin_a, bf))
// through the shared helpers tile_offset / coord_floor / coord_frac, so the
// two operators' matrices are bitwise transposes.
#include "tp_internal.h"

namespace tp {
namespace {

// Forward projection, gather form.  Work-group: W waves = W neighbouring
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
// The work-group sweeps the lines one at a time through a double-buffered
// strip in LDS: the voxels its W angles x 64 bins can touch on a line (all K
// slices, [slice / 4][position] of float4, so a wave's read of one 4-slice
// chunk at its ~1.2-voxel-spaced positions touches near-consecutive 16-byte
// words), so each voxel is fetched once per work-group instead of once per
// bin and angle.  The strip of line m + 2 is loaded into registers while line
// m is summed and written to the free buffer one line later: one barrier per
// line.  A work-group with a strip wider than kRadonStrip on some line
// (sparse angle sets) is summed instead by k_radon_wide, which reads every
// candidate from global memory with the same arithmetic and order.  No
// atomics: every output is summed by one lane, lines ascending, candidates
// ascending.
// Cost on gfx950: besides the 3 FMAs per update, the candidate arithmetic is
// mostly half-rate VALU (conversions, fract, compare/select), so 32 slices
// share it; the strip loads use one scalar base per slice, fixed for the
// kernel, and a 32-bit vector offset (no per-load address arithmetic).  The
// LDS reads of the candidates bound the kernel: the third candidate weighs
// only where the window holds three voxels (a quarter of the lanes at
// typical angles), so it is read under that lane mask and the other lanes
// make no LDS request.
constexpr int kCand = 3;
constexpr int kRadonStrip = 128;

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
    // clamp to [0, N - 1] in one instruction (the compiler emits max + min)
    asm("v_med3_i32 %0, %1, 0, %2" : "=v"(vc) : "v"(v), "s"(N - 1));
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

// A work-group's share of the sweep: W angle slots of the plan's order (one
// per wave), 64 bins from jb, K slices from z0; the wave's angle tables in LDS.
struct RadonGroup {
    int jb, jlast, e0, e_end, a, j, z0, nz;
    unsigned live;  // which of the W slots hold an angle
    bool active;    // this wave's slot holds one
    float cs, sn, cmin, inv, start;
    const int2* tc;  // (integer, fraction bits) per tile along the line
    const int2* tl;  // the same for the line's tile
};

// Fills r, this wave's angle tables (tabs: [W][2][nb] int2 in LDS) and its
// slot's strip parameters; false for a group of padding only (the whole
// work-group returns, before any barrier).
template <bool ROWS, int W>
__device__ __forceinline__ bool radon_group(const GeoTables& g, int K, int n_rows, int2* tabs,
                                            float (*s_par)[3], RadonGroup& r) {
    const int nb = g.nb, na = g.na, half = g.N / 2;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int jgroups = (g.n + 63) >> 6;
    r.jb = (blockIdx.x % jgroups) * 64;
    r.jlast = min(r.jb + 63, g.n - 1);
    const int grp = blockIdx.x / jgroups;
    // this launch covers the angles that sweep rows (ROWS) or columns
    r.e0 = ROWS ? grp * W : g.n_rows_major + grp * W;
    r.e_end = ROWS ? min(g.n_rows_major, r.e0 + W) : min(g.n_order, r.e0 + W);
    if (g.order[r.e0] < 0) return false;
    const int e = r.e0 + wv;
    // padding entries (-1) and entries past the class are inactive waves
    r.active = e < r.e_end && g.order[e] >= 0;
    unsigned live = 0;
    for (int w = 0; w < W; ++w)
        if (r.e0 + w < r.e_end && g.order[r.e0 + w] >= 0) live |= 1u << w;
    r.live = __builtin_amdgcn_readfirstlane(live);
    r.a = r.active ? g.order[e] : g.order[r.e0];
    r.j = r.jb + lane;
    r.z0 = blockIdx.y * K;
    r.nz = min(K, n_rows - r.z0);
    int2* tc = tabs + wv * 2 * nb;
    int2* tl = tc + nb;
    for (int b = lane; b < nb; b += 64) {
        const int xi = g.xi[b * na + r.a], yi = g.yi[b * na + r.a];
        const int xf = __float_as_int(g.xf[b * na + r.a]), yf = __float_as_int(g.yf[b * na + r.a]);
        tc[b] = ROWS ? make_int2(xi, xf) : make_int2(yi, yf);
        tl[b] = ROWS ? make_int2(yi, yf) : make_int2(xi, xf);
    }
    r.tc = tc;
    r.tl = tl;
    r.cs = g.cs[r.a];
    r.sn = g.sn[r.a];
    const float cmaj = ROWS ? r.cs : r.sn;  // coefficient of the swept coordinate
    r.cmin = ROWS ? r.sn : r.cs;            // coefficient of the line coordinate
    r.inv = 1.0f / cmaj;
    // left end of the window of voxels whose coordinate can fall in [j-1, j+1)
    r.start = static_cast<float>(half) - 1.0f / fabsf(cmaj) - 0.01f;
    if (lane == 0) {
        s_par[wv][0] = r.cmin;
        s_par[wv][1] = r.inv;
        s_par[wv][2] = r.start;
    }
    return true;
}

// Strip of line m: the candidate windows of every live slot's first and last
// bin (candidate starts are monotone in the bin), one voxel of margin for the
// FP32 estimates, clipped to the image.  Returns its width (<= 0: no bin of
// the group reaches the image on this line).
template <int W>
__device__ __forceinline__ int radon_strip(const GeoTables& g, const RadonGroup& r, const float (*s_par)[3], int m,
                                           int& xmin) {
    const int N = g.N, half = N / 2;
    int lo = 1 << 30, hi = -(1 << 30);
    for (int w = 0; w < W; ++w) {
        if (!((r.live >> w) & 1u)) continue;
        const float cm = s_par[w][0], iv = s_par[w][1], st = s_par[w][2];
        const float um = static_cast<float>(m - half) * cm + g.center_f;
        const int l0 = -coord_floor(-__builtin_fmaf(static_cast<float>(r.jb) - um, iv, st));
        const int l1 = -coord_floor(-__builtin_fmaf(static_cast<float>(r.jlast) - um, iv, st));
        lo = min(lo, min(l0, l1));
        hi = max(hi, max(l0, l1) + kCand - 1);
    }
    xmin = max(lo - 1, 0);
    return min(hi + 1, N - 1) - xmin + 1;
}

// Whether some line's strip is wider than kRadonStrip (sparse angle sets):
// such a work-group is summed by k_radon_wide instead.  A barrier (the slot
// parameters written by radon_group are read here).
template <int W>
__device__ __forceinline__ bool radon_group_wide(const GeoTables& g, const RadonGroup& r, const float (*s_par)[3]) {
    __syncthreads();
    int wide = 0;
    for (int m = static_cast<int>(threadIdx.x); m < g.N; m += 64 * W) {
        int xmin;
        wide |= radon_strip<W>(g, r, s_par, m, xmin) > kRadonStrip;
    }
    return __syncthreads_or(wide) != 0;
}

// Occupancy the fast kernel's registers allow: 6 waves per SIMD for 16 and
// 32 slices (80 VGPRs; three work-groups of eight waves per CU), 8 for 8.
template <int K> constexpr int radon_waves() { return K >= 16 ? 6 : 8; }

template <int K, bool ROWS, int W>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(radon_waves<K>(), radon_waves<K>())))
k_radon(GeoTables g, const float* __restrict__ vol, int n_rows, float* __restrict__ sino) {
    constexpr int S = kRadonStrip;
    constexpr int KQ = K / 4;         // float4 chunks of slices per position
    constexpr int NT = 64 * W;        // threads
    constexpr int TPP = NT / S;       // staging threads per strip position
    constexpr int KH = K / TPP;       // slices staged per thread
    static_assert(KH % 4 == 0, "a thread stages whole float4 chunks");
    extern __shared__ __align__(16) unsigned char smem[];
    // per angle slot: coefficient of the line coordinate, 1 / swept coefficient, window start
    __shared__ float s_par[W][3];
    // strip bounds of NT lines, two chunks in flight: xmin | width << 16 (0: nothing to sum)
    __shared__ unsigned s_bnd[2][NT];
    const int N = g.N, half = N / 2;
    float4* strip = reinterpret_cast<float4*>(smem);                // [2 buffers][KQ][S]
    int2* tabs = reinterpret_cast<int2*>(strip + 2 * KQ * S);       // [W waves][2][nb]
    RadonGroup r;
    if (!radon_group<ROWS, W>(g, K, n_rows, tabs, s_par, r)) return;
    if (radon_group_wide<W>(g, r, s_par)) return;
    const int j = r.j, nz = r.nz;
    // the angle's coefficients in vector registers: an FMA with a scalar
    // operand issues at half rate
    asm volatile("" : "+v"(r.cs), "+v"(r.sn), "+v"(r.cmin), "+v"(r.inv), "+v"(r.start));
    const int64_t slab = static_cast<int64_t>(N) * N;
    // a line is a row of the volume (ROWS) or of its transpose: contiguous
    const float* vz = vol + static_cast<int64_t>(r.z0) * slab;

    auto line_bounds = [&](int chunk) {
        const int m = chunk * NT + static_cast<int>(threadIdx.x);
        if (m < N) {
            int xmin;
            const int width = radon_strip<W>(g, r, s_par, m, xmin);
            s_bnd[chunk & 1][threadIdx.x] =
                width > 0 ? static_cast<unsigned>(xmin) | (static_cast<unsigned>(width) << 16) : 0u;
        }
    };

    // Staging: thread -> (position px of the strip, share pg of the slices).
    // The next-but-one line is loaded into registers while the current line
    // is summed, and written to the free strip buffer one line later.
    const int px = static_cast<int>(threadIdx.x) & (S - 1);
    const int pg = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / S);
    float pre[KH];
    // the thread's slices: one scalar base each, computed once (slices past
    // the last row re-read it; their sums are never stored)
    const char* sbase[KH];
#pragma unroll
    for (int i = 0; i < KH; ++i)
        sbase[i] = reinterpret_cast<const char*>(vz + static_cast<int64_t>(min(pg * KH + i, nz - 1)) * slab);
    auto load_line = [&](int m, unsigned bd) {
        if (px < static_cast<int>(bd >> 16)) {
            // byte offset in the slice (below 2^32: N <= 32768)
            const uint32_t off = (static_cast<uint32_t>(m) * static_cast<uint32_t>(N) + (bd & 0xffffu) +
                                  static_cast<uint32_t>(px)) * 4u;
#pragma unroll
            for (int i = 0; i < KH; ++i) pre[i] = *reinterpret_cast<const float*>(sbase[i] + off);
        }
    };
    auto write_line = [&](int buf, unsigned bd) {
        if (px < static_cast<int>(bd >> 16)) {
            float4* dst = strip + (buf * KQ + pg * (KH / 4)) * S + px;
#pragma unroll
            for (int q = 0; q < KH / 4; ++q) dst[q * S] = reinterpret_cast<const float4*>(pre)[q];
        }
    };

    float acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0f;

    line_bounds(0);
    if (N > NT) line_bounds(1);
    __syncthreads();
    unsigned bm = s_bnd[0][0];
    unsigned bm1 = N > 1 ? s_bnd[0][1] : 0u;
    load_line(0, bm);
    write_line(0, bm);
    if (N > 1) load_line(1, bm1);
    __syncthreads();

    for (int m = 0; m < N; ++m) {
        const int buf = m & 1;
        // line m + 1 goes to the buffer line m - 1 used (every wave is past it)
        if (m + 1 < N) write_line(buf ^ 1, bm1);
        unsigned bm2 = 0u;
        if (m + 2 < N) {
            bm2 = s_bnd[((m + 2) / NT) & 1][(m + 2) % NT];
            load_line(m + 2, bm2);
        }
        // bounds of chunk c + 1 at the chunk's first line: its buffer held
        // chunk c - 1, whose last entry was read two lines ago
        if (m % NT == 0 && m > 0 && (m / NT + 1) * NT < N) line_bounds(m / NT + 1);
        // a line no bin of the group reaches adds nothing
        if (r.active && j < g.n && (bm >> 16)) {
            const RadonLine ln = radon_line(m, j, half, r.cmin, r.inv, r.start, g.center_f, r.tl);
            float wt[kCand];
            int vcs[kCand];
#pragma unroll
            for (int t = 0; t < kCand; ++t) wt[t] = radon_weight<ROWS>(ln, t, j, N, r.cs, r.sn, r.tc, vcs[t]);
            const int xmin = static_cast<int>(bm & 0xffffu);
            const float4* sb = strip + buf * KQ * S;
            int xo[kCand];
#pragma unroll
            for (int t = 0; t < kCand; ++t) xo[t] = min(max(vcs[t] - xmin, 0), S - 1);
            // chunk by chunk (few reads in flight); each slice still adds its
            // candidates in order: the first two here, the third below
#pragma unroll
            for (int q = 0; q < KQ; ++q) {
                float4 v[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) v[t] = sb[q * S + xo[t]];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    acc[4 * q + 0] = __builtin_fmaf(wt[t], v[t].x, acc[4 * q + 0]);
                    acc[4 * q + 1] = __builtin_fmaf(wt[t], v[t].y, acc[4 * q + 1]);
                    acc[4 * q + 2] = __builtin_fmaf(wt[t], v[t].z, acc[4 * q + 2]);
                    acc[4 * q + 3] = __builtin_fmaf(wt[t], v[t].w, acc[4 * q + 3]);
                }
            }
            // the third candidate weighs only where the window holds three
            // voxels: the other lanes read nothing
            if (wt[2] != 0.0f) {
#pragma unroll
                for (int q = 0; q < KQ; ++q) {
                    const float4 v = sb[q * S + xo[2]];
                    acc[4 * q + 0] = __builtin_fmaf(wt[2], v.x, acc[4 * q + 0]);
                    acc[4 * q + 1] = __builtin_fmaf(wt[2], v.y, acc[4 * q + 1]);
                    acc[4 * q + 2] = __builtin_fmaf(wt[2], v.z, acc[4 * q + 2]);
                    acc[4 * q + 3] = __builtin_fmaf(wt[2], v.w, acc[4 * q + 3]);
                }
            }
        }
        __syncthreads();
        bm = bm1;
        bm1 = bm2;
    }
    if (r.active && j < g.n) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (k < nz) sino[(static_cast<int64_t>(r.z0 + k) * g.na + r.a) * g.n + j] = acc[k];
    }
}

// The work-groups k_radon leaves (a strip wider than kRadonStrip on some
// line): each candidate is read from global memory, with the same arithmetic
// and order (zero weights skipped: they would add exact zeros).
template <int K, bool ROWS, int W>
__global__ void __launch_bounds__(64 * W) k_radon_wide(GeoTables g, const float* __restrict__ vol, int n_rows,
                                                      float* __restrict__ sino) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float s_par[W][3];
    int2* tabs = reinterpret_cast<int2*>(smem);  // [W waves][2][nb]
    RadonGroup r;
    if (!radon_group<ROWS, W>(g, K, n_rows, tabs, s_par, r)) return;
    if (!radon_group_wide<W>(g, r, s_par)) return;
    const int N = g.N, half = N / 2, j = r.j, nz = r.nz;
    const int64_t slab = static_cast<int64_t>(N) * N;
    const float* vz = vol + static_cast<int64_t>(r.z0) * slab;
    if (!r.active || j >= g.n) return;  // no barrier below
    float acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0f;
    for (int m = 0; m < N; ++m) {
        const RadonLine ln = radon_line(m, j, half, r.cmin, r.inv, r.start, g.center_f, r.tl);
#pragma unroll
        for (int t = 0; t < kCand; ++t) {
            int vc;
            const float wt = radon_weight<ROWS>(ln, t, j, N, r.cs, r.sn, r.tc, vc);
            if (wt != 0.0f) {
                // byte offset of the voxel in its slice, a scalar base per slice
                const uint32_t off = (static_cast<uint32_t>(m) * static_cast<uint32_t>(N) +
                                      static_cast<uint32_t>(vc)) * 4u;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    int kk = min(k, nz - 1);
                    asm volatile("" : "+s"(kk));
                    const char* sp = reinterpret_cast<const char*>(vz + static_cast<int64_t>(kk) * slab);
                    acc[k] = __builtin_fmaf(wt, *reinterpret_cast<const float*>(sp + off), acc[k]);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (k < nz) sino[(static_cast<int64_t>(r.z0 + k) * g.na + r.a) * g.n + j] = acc[k];
}

}  // namespace

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

template <int K, bool ROWS, int W>
hipError_t launch_radon_k(const GeoTables& g, const float* vol, int n_rows, float* sino, hipStream_t st) {
    const int jgroups = (g.n + 63) / 64;
    const int groups = ROWS ? (g.n_rows_major + W - 1) / W : (g.n_order - g.n_rows_major + W - 1) / W;
    if (groups == 0) return hipSuccess;
    const size_t tabs = sizeof(int2) * 2 * W * static_cast<size_t>(g.nb);
    const size_t lds = sizeof(float) * 2 * K * kRadonStrip + tabs;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_radon<K, ROWS, W>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    if (tabs > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_radon_wide<K, ROWS, W>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(tabs));
        if (e != hipSuccess) return e;
    }
    const dim3 grid(static_cast<unsigned>(jgroups * groups), static_cast<unsigned>((n_rows + K - 1) / K));
    hipLaunchKernelGGL((k_radon<K, ROWS, W>), grid, dim3(64 * W), lds, st, g, vol, n_rows, sino);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_radon_wide<K, ROWS, W>), grid, dim3(64 * W), tabs, st, g, vol, n_rows, sino);
    return hipGetLastError();
}

template <int K>
hipError_t launch_radon_both(const GeoTables& g, const float* vol, const float* volT, int n_rows, float* sino,
                             hipStream_t st) {
    // Eight angles per strip unless their tile tables (16 x nb int2) would
    // take the work-group past the 160 KB of LDS (slices above ~30976 voxels
    // wide); both kernels of an axis must group the angles alike.
    if constexpr (K >= 16) {
        const size_t lds8 = sizeof(float) * 2 * K * kRadonStrip + sizeof(int2) * 2 * 8 * static_cast<size_t>(g.nb) +
                            sizeof(float) * 3 * 8 + sizeof(unsigned) * 2 * 64 * 8;
        if (lds8 <= 160 * 1024) {
            hipError_t e = launch_radon_k<K, true, 8>(g, vol, n_rows, sino, st);
            if (e != hipSuccess) return e;
            return launch_radon_k<K, false, 8>(g, volT, n_rows, sino, st);
        }
    }
    hipError_t e = launch_radon_k<K, true, 4>(g, vol, n_rows, sino, st);
    if (e != hipSuccess) return e;
    return launch_radon_k<K, false, 4>(g, volT, n_rows, sino, st);
}

}  // namespace

size_t radon_workspace_bytes(const GeoTables& g, int n_rows) {
    return g.n_rows_major < g.n_order ? sizeof(float) * static_cast<size_t>(n_rows) * g.N * g.N : 0;
}

// Angles that sweep columns (|sin| > |cos|) read a transposed copy of the
// volume, so their lines are contiguous too.  32 slices per work-group
// amortise each candidate's coordinate; smaller chunks use 16 or 8.  Eight
// angles share a strip (half the staging per update of four) when a thread
// then still stages whole float4 chunks (16 or more slices) and their tables
// fit the LDS.
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
