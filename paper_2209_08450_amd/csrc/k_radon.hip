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
// line.  A strip wider than kRadonStrip (sparse angle sets) is read from
// global memory instead, with the same arithmetic and order.  No atomics:
// every output is summed by one lane, lines ascending, candidates ascending.
// Cost on gfx950: besides the 3 FMAs per update, the candidate arithmetic is
// mostly half-rate VALU (conversions, fract, compare/select), so 32 slices
// share it; the strip loads use one scalar base per slice, fixed for the
// kernel, and a 32-bit vector offset (no per-load address arithmetic).
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

template <int K, bool ROWS, int W>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(4, 4)))
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
    // strip bounds of NT lines, two chunks in flight: xmin | width << 16 (0: not staged)
    __shared__ unsigned s_bnd[2][NT];
    const int nb = g.nb, na = g.na, N = g.N, half = N / 2;
    float4* strip = reinterpret_cast<float4*>(smem);                // [2 buffers][KQ][S]
    int2* tabs = reinterpret_cast<int2*>(strip + 2 * KQ * S);       // [W waves][2][nb]
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
    // which of the work-group's W angle slots hold an angle
    unsigned live = 0;
    for (int w = 0; w < W; ++w)
        if (e0 + w < e_end && g.order[e0 + w] >= 0) live |= 1u << w;
    live = __builtin_amdgcn_readfirstlane(live);
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
    if (lane == 0) {
        s_par[wv][0] = cmin;
        s_par[wv][1] = inv;
        s_par[wv][2] = start;
    }
    const int64_t slab = static_cast<int64_t>(N) * N;
    // a line is a row of the volume (ROWS) or of its transpose: contiguous
    const float* vz = vol + static_cast<int64_t>(z0) * slab;
    const int jlast = min(jb + 63, g.n - 1);

    // Strip bounds of the lines of a chunk (one line per thread): the
    // candidate windows of every live slot's first and last bin (candidate
    // starts are monotone in the bin), one voxel of margin for the FP32
    // estimates.  A line whose strip is wider than S is read from global memory.
    auto line_bounds = [&](int chunk) {
        const int m = chunk * NT + static_cast<int>(threadIdx.x);
        if (m < N) {
            int lo = 1 << 30, hi = -(1 << 30);
            for (int w = 0; w < W; ++w) {
                if (!((live >> w) & 1u)) continue;
                const float cm = s_par[w][0], iv = s_par[w][1], st = s_par[w][2];
                const float um = static_cast<float>(m - half) * cm + g.center_f;
                const int l0 = -coord_floor(-__builtin_fmaf(static_cast<float>(jb) - um, iv, st));
                const int l1 = -coord_floor(-__builtin_fmaf(static_cast<float>(jlast) - um, iv, st));
                lo = min(lo, min(l0, l1));
                hi = max(hi, max(l0, l1) + kCand - 1);
            }
            const int xmin = max(lo - 1, 0), xmax = min(hi + 1, N - 1);
            const int width = xmax - xmin + 1;
            s_bnd[chunk & 1][threadIdx.x] =
                (width > 0 && width <= S) ? static_cast<unsigned>(xmin) | (static_cast<unsigned>(width) << 16) : 0u;
        }
    };

    // Staging: thread -> (position px of the strip, half pg of the slices).
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

    __syncthreads();  // s_par, tables
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
        if (active && j < g.n) {
            const RadonLine ln = radon_line(m, j, half, cmin, inv, start, g.center_f, tl);
            float wt[kCand];
            int vcs[kCand];
#pragma unroll
            for (int t = 0; t < kCand; ++t) wt[t] = radon_weight<ROWS>(ln, t, j, N, cs, sn, tc, vcs[t]);
            if (bm >> 16) {
                const int xmin = static_cast<int>(bm & 0xffffu);
                const float4* sb = strip + buf * KQ * S;
#pragma unroll
                for (int t = 0; t < kCand; ++t) {
                    const int xo = min(max(vcs[t] - xmin, 0), S - 1);
                    const float4* src = sb + xo;
                    float val[K];
#pragma unroll
                    for (int q = 0; q < KQ; ++q) reinterpret_cast<float4*>(val)[q] = src[q * S];
                    // zero weights add exact zeros: no branch
#pragma unroll
                    for (int k = 0; k < K; ++k) acc[k] = __builtin_fmaf(wt[t], val[k], acc[k]);
                }
            } else {
#pragma unroll
                for (int t = 0; t < kCand; ++t) {
                    if (wt[t] != 0.0f) {
                        const float* p = vz + static_cast<int64_t>(m) * N + vcs[t];
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            int kk = min(k, nz - 1);
                            asm volatile("" : "+s"(kk));
                            acc[k] = __builtin_fmaf(wt[t], p[kk * slab], acc[k]);
                        }
                    }
                }
            }
        }
        __syncthreads();
        bm = bm1;
        bm1 = bm2;
    }
    if (active && j < g.n) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (k < nz) sino[(static_cast<int64_t>(z0 + k) * na + a) * g.n + j] = acc[k];
    }
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
    const size_t lds = sizeof(float) * 2 * K * kRadonStrip + sizeof(int2) * 2 * W * static_cast<size_t>(g.nb);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_radon<K, ROWS, W>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    const dim3 grid(static_cast<unsigned>(jgroups * groups), static_cast<unsigned>((n_rows + K - 1) / K));
    hipLaunchKernelGGL((k_radon<K, ROWS, W>), grid, dim3(64 * W), lds, st, g, vol, n_rows, sino);
    return hipGetLastError();
}

template <int K>
hipError_t launch_radon_both(const GeoTables& g, const float* vol, const float* volT, int n_rows, float* sino,
                             hipStream_t st) {
    constexpr int W8 = K >= 16 ? 8 : 4;
    hipError_t e = launch_radon_k<K, true, W8>(g, vol, n_rows, sino, st);
    if (e != hipSuccess) return e;
    return launch_radon_k<K, false, W8>(g, volT, n_rows, sino, st);
}

}  // namespace

size_t radon_workspace_bytes(const GeoTables& g, int n_rows) {
    return g.n_rows_major < g.n_order ? sizeof(float) * static_cast<size_t>(n_rows) * g.N * g.N : 0;
}

// Angles that sweep columns (|sin| > |cos|) read a transposed copy of the
// volume, so their lines are contiguous too.  32 slices per work-group
// amortise each candidate's coordinate; smaller chunks use 16 or 8.  Eight
// angles share a strip (half the staging per update of four) when a thread
// then still stages whole float4 chunks (16 or more slices).
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
