// Fourier-domain filtered backprojection (paper, Section 2.2: backprojection
// evaluated with exponential interpolation kernels in the frequency domain;
// Section 3 uses it as the reference method).
//
// By the Fourier slice theorem the spectrum of the projection at angle theta
// is the line of the 2-D image spectrum through the origin in direction
// theta.  Filtered backprojection with band-limited interpolation along each
// ray is therefore a non-uniform inverse DFT from these polar samples to the
// voxel grid:
//   f(x) = sum_{a,k} c_{a,k} exp(2 pi i (k / L) theta_a . x),
//   c_{a,k} = (pi / na) / L * w_k * H[k] * U_a[k] * exp(2 pi i k pos0 / L),
// where U_a is the DFT of the padded row, H the filter response, w_k = 1/2 at
// the two Nyquist terms and pos0 the padded-row position of the axis.  It is
// evaluated as an unequally spaced FFT: every polar sample is spread with a
// Gaussian phi(u) = exp(-|u|^2 / (4 tau)) onto a Cartesian grid of M points
// per side (oversampling >= 2), the grid is inverse-transformed, and each
// voxel is divided by the Gaussian's Fourier transform.
//
// Two slices travel as the real and imaginary parts of one complex row, so
// every transform and the spreading are complex and the two reconstructions
// come back as the real and imaginary parts of the image.
//
// Stages (one launch each):
//   k_fr_spectra  normalise two rows, pad, FFT, multiply by the E table and
//                 store the L + 1 signed-frequency samples of the angle;
//   k_fr_grid     for every grid point, sum the Gaussian-weighted samples of
//                 every angle whose ray passes within the truncation radius
//                 (a gather: no atomics, a fixed summation order; FP64
//                 accumulation over batches of 16 angles);
//   k_fr_rows     inverse FFT along the grid's fast axis, keeping the N
//                 output rows, stored in 16-wide column groups;
//   k_fr_cols     inverse FFT along the other axis, deconvolution, split of
//                 the two slices, store.
#include "fft_device.h"

namespace tp {
namespace {

constexpr float kPiF = 3.14159265358979323846f;
constexpr int kFrTile = 16;             // grid points per tile side (4 waves of 8x8)
constexpr int kFrBatch = 16;            // angles staged per batch
constexpr float kFrHalfDiag = 10.6066017f;   // 7.5 sqrt(2): tile centre to its farthest point
constexpr float kFrWaveHalfDiag = 4.9497475f;  // 3.5 sqrt(2): the same for a wave's 8x8 block

__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, 0.0f - a.y); }

// Store one voxel: FP32, or the FP32 value rounded once to FP16.  The value is
// fenced into a register first: otherwise the compiler contracts the product
// that forms it with the conversion (one mixed-precision multiply rounding the
// exact product to FP16), which differs from the FP32 slice rounded at ties.
__device__ __forceinline__ void fr_store(float* p, int64_t i, float v) { p[i] = v; }
__device__ __forceinline__ void fr_store(__half* p, int64_t i, float v) {
    asm volatile("" : "+v"(v));
    p[i] = __float2half_rn(v);
}

int fr_block(int L) {
    int b = L / 16;
    if (b < 64) b = 64;
    if (b > 1024) b = 1024;
    return b;
}

template <typename K>
hipError_t fr_lds(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

// ---------------------------------------------------------------------------
// Spectra: one work-group per (pair of slices, angle).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024)
k_fr_spectra(RawInput in, int rows, const float* __restrict__ dmean, const float* __restrict__ rden,
             const float2* __restrict__ tw, FourierTables t, float2* __restrict__ spec) {
    extern __shared__ float2 buf[];
    const int tid = threadIdx.x, B = blockDim.x;
    const int L = t.L, n = t.n, off = (L - n) / 2, h = L / 2;
    const int p = blockIdx.x / t.na;
    const int a = blockIdx.x - p * t.na;
    const int z0 = 2 * p;
    const bool has1 = z0 + 1 < rows;
    const uint16_t* p0 = in.proj + a * in.proj_stride + static_cast<int64_t>(z0) * n;
    const uint16_t* p1 = has1 ? p0 + n : p0;
    const float* d0 = dmean + static_cast<int64_t>(z0) * n;
    const float* e0 = rden + static_cast<int64_t>(z0) * n;
    const float* d1 = has1 ? d0 + n : d0;
    const float* e1 = has1 ? e0 + n : e0;
    // clamping the column onto the detector gives the edge-replicated padding
    for (int m = tid; m < L; m += B) {
        const int c = min(max(m - off, 0), n - 1);
        const float v0 = neglog_counts(static_cast<float>(p0[c]), d0[c], e0[c]);
        const float v1 = has1 ? neglog_counts(static_cast<float>(p1[c]), d1[c], e1[c]) : 0.0f;
        buf[m] = make_float2(v0, v1);
    }
    __syncthreads();
    fft_forward_lds(buf, L, t.log2L, tw);
    const int sl = t.slot[a];
    const bool rev = (sl & 1) != 0;
    float2* row = spec + (static_cast<int64_t>(p) * t.na + (sl >> 1)) * t.SL;
    for (int m = tid; m < L; m += B) {
        const float2 X = buf[m];
        const int k = m < h ? m : m - L;  // m = L/2 is the -L/2 term
        row[(rev ? -k : k) + h] = cmul(X, t.E[k + h]);
        if (m == h) row[(rev ? -h : h) + h] = cmul(X, t.E[L]);  // and its +L/2 copy
    }
}

// ---------------------------------------------------------------------------
// Gather onto the Cartesian frequency grid.
//
// Work-group: one 16x16 tile of one pair's grid, 4 waves of 8x8 points.  The
// grid is periodic (M points per side), so tiles near its edge also gather
// through their images shifted by +-M.  For each tile image only the angles
// whose ray passes within (radius + half-diagonal) of its centre can
// contribute; they form one interval of the sorted reduced angles (two when
// it wraps past pi), found by binary search.  Each batch of 16 angles stages,
// per angle, the window of samples the tile can reach; each lane then sums its
// taps along the ray with the Gaussian weights from a two-ratio recurrence:
//   w(k+1) = w(k) r(k),  r(k+1) = r(k) exp2(-2 kappa s^2).
// The tile centre's along-ray position and perpendicular offset are formed in
// FP64 (integer + FP32 fraction), lanes add only their in-tile offsets, so the
// coordinates keep FP32 precision at any grid size.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lower_bound_f(const float* v, int n, float x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (v[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ int upper_bound_f(const float* v, int n, float x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (v[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <int NT>
__global__ void __launch_bounds__(256)
k_fr_grid(FourierTables t, const float2* __restrict__ spec, float2* __restrict__ grid) {
    extern __shared__ float4 stage[];  // [kFrBatch][sw]: (sample k, sample -k)
    __shared__ int s_kc[kFrBatch];
    __shared__ float4 s_geo[kFrBatch];  // (fraction of the centre's position, perpendicular offset, cos, sin)
    const int M = t.M, hM = M / 2, tps = M / kFrTile;
    const int p = blockIdx.x / t.ntiles;
    const int tile = t.tile_order[blockIdx.x - p * t.ntiles];
    const int ty = tile / tps, tx = tile - ty * tps;
    // tile rows ty >= tps/2 (uy >= 0) also produce the mirror points -u;
    // tile row 0 only supplies the grid row uy = -M/2, which no mirror reaches
    const bool nyq = ty == 0;
    const int ux0 = tx * kFrTile - hM, uy0 = ty * kFrTile - hM;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int ox = (w >> 1) * 8 + (l >> 3), oy = (w & 1) * 8 + (l & 7);
    // lane and wave-centre offsets from the tile centre
    const float dx = static_cast<float>(ox) - 7.5f, dy = static_cast<float>(oy) - 7.5f;
    const float wdx = static_cast<float>((w >> 1) * 8) - 4.0f, wdy = static_cast<float>((w & 1) * 8) - 4.0f;
    const float2* sp = spec + static_cast<int64_t>(p) * t.na * t.SL;
    const int h = t.L / 2;
    const float reach = t.msp + kFrHalfDiag + 1.0f;
    // each batch of angles is summed in FP32, the batches in FP64: central
    // grid points collect thousands of angles
    double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0;
    for (int img = 0; img < 9; ++img) {
        const float Cx = static_cast<float>(ux0 + (img % 3 - 1) * M) + 7.5f;
        const float Cy = static_cast<float>(uy0 + (img / 3 - 1) * M) + 7.5f;
        const float rho = sqrtf(Cx * Cx + Cy * Cy);
        if (rho > static_cast<float>(hM) + reach) continue;  // samples lie within radius M/2
        int lo0 = 0, hi0 = t.na, lo1 = 0, hi1 = 0;
        if (rho > reach) {
            const float d = asinf(reach / rho) + 1e-4f;
            if (d < 1.5f) {
                float al = atan2f(Cy, Cx);
                if (al < 0.0f) al += kPiF;
                if (al >= kPiF) al -= kPiF;
                const float lo = al - d, hi = al + d;
                if (lo < 0.0f) {
                    lo0 = lower_bound_f(t.beta, t.na, lo + kPiF);
                    hi1 = upper_bound_f(t.beta, t.na, hi);
                } else if (hi >= kPiF) {
                    lo0 = lower_bound_f(t.beta, t.na, lo);
                    hi1 = upper_bound_f(t.beta, t.na, hi - kPiF);
                } else {
                    lo0 = lower_bound_f(t.beta, t.na, lo);
                    hi0 = upper_bound_f(t.beta, t.na, hi);
                }
            }
        }
        const double Cxd = static_cast<double>(Cx), Cyd = static_cast<double>(Cy);
        for (int rr = 0; rr < 2; ++rr) {
            const int alo = rr ? lo1 : lo0, ahi = rr ? hi1 : hi0;
            for (int a0 = alo; a0 < ahi; a0 += kFrBatch) {
                const int cnt = min(kFrBatch, ahi - a0);
                __syncthreads();  // the previous batch's reads are done
                if (threadIdx.x < cnt) {
                    const int ap = a0 + threadIdx.x;
                    const double cbd = t.cbd[ap], sbd = t.sbd[ap];
                    const double tc = (Cxd * cbd + Cyd * sbd) * static_cast<double>(t.inv_s);
                    const double kc = floor(tc);
                    s_kc[threadIdx.x] = static_cast<int>(kc);
                    s_geo[threadIdx.x] = make_float4(static_cast<float>(tc - kc),
                                                     static_cast<float>(Cyd * cbd - Cxd * sbd), t.cb[ap], t.sb[ap]);
                }
                __syncthreads();
                // wave w stages angles w, w + 4, ...; lane l the window's sample l (sw <= 64)
                for (int j = w; j < cnt; j += 4) {
                    if (l < t.sw) {
                        const int k = s_kc[j] - t.back + l;  // signed frequency index
                        const float2* row = sp + static_cast<int64_t>(a0 + j) * t.SL + h;
                        const bool in = k >= -h && k <= h;
                        const float2 v = in ? row[k] : make_float2(0.0f, 0.0f);
                        const float2 u = in ? row[-k] : make_float2(0.0f, 0.0f);
                        stage[j * t.sw + l] = make_float4(v.x, v.y, u.x, u.y);
                    }
                }
                __syncthreads();
                // FP32 partial sums over the batch (at most 16 angles x NT taps)
                float pa = 0.0f, pb = 0.0f, pc = 0.0f, pd = 0.0f;
                for (int j = 0; j < cnt; ++j) {
                    const float4 geo = s_geo[j];
                    const float cb = geo.z, sb = geo.w, cp = geo.y;
                    // no lane of this wave within the radius of the ray
                    if (fabsf(cp + wdy * cb - wdx * sb) > t.msp + kFrWaveHalfDiag + 0.01f) continue;
                    const float tr = geo.x + (dx * cb + dy * sb) * t.inv_s;  // along-ray, samples, from kc
                    const float dp = cp + dy * cb - dx * sb;                  // perpendicular, grid points
                    if (fabsf(dp) > t.msp) continue;  // outside the band: no LDS reads for this lane
                    const int k0 = coord_floor(tr) - NT / 2 + 1;
                    const float q = (tr - static_cast<float>(k0)) * t.s;    // distance to tap k0, grid points
                    // for grid spacings s <= 8 and half widths 3..8 the exponents stay within
                    // (-80, 70): the hardware exp2 needs no range handling
                    float wgt = __builtin_amdgcn_exp2f(-t.kappa * (dp * dp + q * q));
                    float r = __builtin_amdgcn_exp2f(t.kappa * (2.0f * t.s * q - t.s * t.s));
                    const int idx = min(max(k0 + t.back, 0), t.sw - NT);
                    const float4* sv = stage + j * t.sw + idx;
#pragma unroll
                    for (int tap = 0; tap < NT; ++tap) {
                        const float4 v = sv[tap];
                        pa = __builtin_fmaf(wgt, v.x, pa);
                        pb = __builtin_fmaf(wgt, v.y, pb);
                        pc = __builtin_fmaf(wgt, v.z, pc);
                        pd = __builtin_fmaf(wgt, v.w, pd);
                        if (tap + 1 < NT) {
                            wgt *= r;
                            r *= t.ratio2;
                        }
                    }
                }
                ax += static_cast<double>(pa);
                ay += static_cast<double>(pb);
                bx += static_cast<double>(pc);
                by += static_cast<double>(pd);
            }
        }
    }
    const int ux = ux0 + ox, uy = uy0 + oy;
    if (nyq) {
        if (uy == -hM) grid[(static_cast<int64_t>(p) * M + (ux & (M - 1))) * M + (uy & (M - 1))] =
            make_float2(static_cast<float>(ax), static_cast<float>(ay));
        return;
    }
    grid[(static_cast<int64_t>(p) * M + (ux & (M - 1))) * M + (uy & (M - 1))] =
        make_float2(static_cast<float>(ax), static_cast<float>(ay));
    if (uy > 0)  // the row uy = 0 is its own mirror
        grid[(static_cast<int64_t>(p) * M + ((-ux) & (M - 1))) * M + ((-uy) & (M - 1))] =
            make_float2(static_cast<float>(bx), static_cast<float>(by));
}

// ---------------------------------------------------------------------------
// Inverse FFT along the grid's fast axis (frequency uy -> image y) for one
// (pair, ux) row; the inverse transform is conj(FFT(conj(.))).  Outputs
// y = iy - N/2 for iy in [0, N) go to cols[p][iy / 16][ux][iy % 16], so the
// column pass reads 16 neighbouring image rows from one 128-byte line.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024)
k_fr_rows(const float2* __restrict__ grid, const float2* __restrict__ tw, FourierTables t,
          float2* __restrict__ cols) {
    extern __shared__ float2 buf[];
    const int tid = threadIdx.x, B = blockDim.x;
    const int M = t.M, N = t.N, hN = N / 2;
    const int64_t rid = blockIdx.x;
    const int p = static_cast<int>(rid / M);
    const int ux = static_cast<int>(rid - static_cast<int64_t>(p) * M);
    const float2* g = grid + rid * M;
    for (int m = tid; m < M; m += B) buf[m] = cconj(g[m]);
    __syncthreads();
    fft_forward_lds(buf, M, t.log2M, tw);
    const int ng = (N + 15) / 16;
    float2* cp = cols + static_cast<int64_t>(p) * ng * M * 16;
    for (int m = tid; m < M; m += B) {
        const int y = m < M / 2 ? m : m - M;
        const int iy = y + hN;
        if (iy >= 0 && iy < N) cp[(static_cast<int64_t>(iy >> 4) * M + ux) * 16 + (iy & 15)] = cconj(buf[m]);
    }
}

// ---------------------------------------------------------------------------
// Inverse FFT along ux for one (pair, image row iy), deconvolution by the
// Gaussian's transform, and the split into the pair's two slices.  The 16
// work-groups of one column group run back to back on one XCD (work-groups
// are dealt to the 8 XCDs in turn), so their shared 128-byte lines are read
// from that XCD's L2.
// ---------------------------------------------------------------------------
template <typename OutT>
__global__ void __launch_bounds__(1024)
k_fr_cols(const float2* __restrict__ cols, const float2* __restrict__ tw, FourierTables t, int pairs, int rows,
          OutT* __restrict__ vol) {
    extern __shared__ float2 buf[];
    const int tid = threadIdx.x, B = blockDim.x;
    const int M = t.M, N = t.N, hN = N / 2;
    const int ng = (N + 15) / 16;
    const int b = blockIdx.x;
    const int xcd = b & 7, r = b >> 3;
    const int gidx = (r >> 4) * 8 + xcd;
    const int p = gidx / ng, gi = gidx - p * ng;
    const int iy = gi * 16 + (r & 15);
    if (p >= pairs || iy >= N) return;  // whole work-group
    const float2* src = cols + (static_cast<int64_t>(p) * ng + gi) * M * 16 + (iy & 15);
    for (int m = tid; m < M; m += B) buf[m] = cconj(src[static_cast<int64_t>(m) * 16]);
    __syncthreads();
    fft_forward_lds(buf, M, t.log2M, tw);
    const float fy = t.D[iy];
    const int z0 = 2 * p;
    const bool has1 = z0 + 1 < rows;
    OutT* o0 = vol + (static_cast<int64_t>(z0) * N + iy) * N;
    OutT* o1 = o0 + static_cast<int64_t>(N) * N;
    for (int m = tid; m < M; m += B) {
        const int x = m < M / 2 ? m : m - M;
        const int ix = x + hN;
        if (ix >= 0 && ix < N) {
            const float2 v = buf[m];  // conj of the inverse transform: (re, -im)
            const float f = t.D[ix] * fy;
            fr_store(o0, ix, v.x * f);  // FP16 slices: the FP32 value rounded once
            if (has1) fr_store(o1, ix, (0.0f - v.y) * f);
        }
    }
}

// ---------------------------------------------------------------------------
// Register-resident variants of the three transform kernels for lengths
// 1024..8192: thread t holds elements t + B s (B = length / 16) and the
// radix-16 passes exchange only their outputs through LDS; after the last
// pass slot s holds output index t + B s in natural order.
// ---------------------------------------------------------------------------
// Angles per work-group of the register spectra kernel: each angle's raw
// counts are prefetched while the previous angle is transformed.
constexpr int kFrAnglesPerGroup = 8;

template <int L>
__global__ void __launch_bounds__(L / kRegPts)
k_fr_spectra_reg(RawInput in, int rows, const float* __restrict__ dmean, const float* __restrict__ rden,
                 const float2* __restrict__ tw, FourierTables t, float2* __restrict__ spec) {
    extern __shared__ float2 lds[];
    constexpr int B = L / kRegPts, h = L / 2;
    const int n = t.n, off = (L - n) / 2;
    const int groups = (t.na + kFrAnglesPerGroup - 1) / kFrAnglesPerGroup;
    const int p = blockIdx.x / groups;
    const int a0 = (blockIdx.x - p * groups) * kFrAnglesPerGroup;
    const int a1 = min(t.na, a0 + kFrAnglesPerGroup);
    const int z0 = 2 * p;
    const bool has1 = z0 + 1 < rows;
    const int64_t r0 = static_cast<int64_t>(z0) * n;
    const int64_t r1 = has1 ? r0 + n : r0;
    // slot s holds padded position t + B s; the column clamped onto the
    // detector gives the edge-replicated padding
    auto load_raw = [&](int a, int tid, uint32_t (&raw)[kRegPts]) {
        const uint16_t* q0 = in.proj + a * in.proj_stride + r0;
        const uint16_t* q1 = in.proj + a * in.proj_stride + r1;
#pragma unroll
        for (int s = 0; s < kRegPts; ++s) {
            const int c = min(max(tid + B * s - off, 0), n - 1);
            raw[s] = static_cast<uint32_t>(q0[c]) | (static_cast<uint32_t>(q1[c]) << 16);
        }
    };
    uint32_t cur[kRegPts], nxt[kRegPts];
    load_raw(a0, threadIdx.x, cur);
#pragma unroll 1
    for (int a = a0; a < a1; ++a) {
        // an opaque thread index per angle keeps per-thread offsets from being
        // hoisted into registers held across the loop
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        if (a + 1 < a1) load_raw(a + 1, tid, nxt);
        float2 x[kRegPts];
#pragma unroll
        for (int s = 0; s < kRegPts; ++s) {
            const int c = min(max(tid + B * s - off, 0), n - 1);
            x[s] = make_float2(neglog_counts(static_cast<float>(cur[s] & 0xffffu), dmean[r0 + c], rden[r0 + c]),
                               has1 ? neglog_counts(static_cast<float>(cur[s] >> 16), dmean[r1 + c], rden[r1 + c])
                                    : 0.0f);
        }
        reg_fft<L>(x, lds, tw, tid);
        const int sl = t.slot[a];
        const bool rev = (sl & 1) != 0;
        float2* row = spec + (static_cast<int64_t>(p) * t.na + (sl >> 1)) * t.SL;
#pragma unroll
        for (int s = 0; s < kRegPts; ++s) {
            const int m = tid + B * s;
            const int k = m < h ? m : m - L;
            row[(rev ? -k : k) + h] = cmul(x[s], t.E[k + h]);
            if (m == h) row[(rev ? -h : h) + h] = cmul(x[s], t.E[L]);
        }
#pragma unroll
        for (int s = 0; s < kRegPts; ++s) cur[s] = nxt[s];
    }
}

template <int M>
__global__ void __launch_bounds__(M / kRegPts)
k_fr_rows_reg(const float2* __restrict__ grid, const float2* __restrict__ tw, FourierTables t,
              float2* __restrict__ cols) {
    extern __shared__ float2 lds[];
    constexpr int B = M / kRegPts;
    const int tid = threadIdx.x;
    const int N = t.N, hN = N / 2;
    const int64_t rid = blockIdx.x;
    const int p = static_cast<int>(rid / M);
    const int ux = static_cast<int>(rid - static_cast<int64_t>(p) * M);
    const float2* g = grid + rid * M;
    float2 x[kRegPts];
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) x[s] = cconj(g[tid + B * s]);
    reg_fft<M>(x, lds, tw, tid);
    const int ng = (N + 15) / 16;
    float2* cp = cols + static_cast<int64_t>(p) * ng * M * 16;
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) {
        const int m = tid + B * s;
        const int y = m < M / 2 ? m : m - M;
        const int iy = y + hN;
        if (iy >= 0 && iy < N) cp[(static_cast<int64_t>(iy >> 4) * M + ux) * 16 + (iy & 15)] = cconj(x[s]);
    }
}

template <int M, typename OutT>
__global__ void __launch_bounds__(M / kRegPts)
k_fr_cols_reg(const float2* __restrict__ cols, const float2* __restrict__ tw, FourierTables t, int pairs, int rows,
              OutT* __restrict__ vol) {
    // two neighbouring image rows (iy, iy + 1) per work-group: 16-byte loads
    extern __shared__ float2 lds[];
    constexpr int B = M / kRegPts;
    const int tid = threadIdx.x;
    const int N = t.N, hN = N / 2;
    const int ng = (N + 15) / 16;
    const int b = blockIdx.x;
    const int xcd = b & 7, r = b >> 3;
    const int gidx = (r >> 3) * 8 + xcd;
    const int p = gidx / ng, gi = gidx - p * ng;
    const int iy = gi * 16 + 2 * (r & 7);
    if (p >= pairs || iy >= N) return;  // whole work-group
    const float4* src = reinterpret_cast<const float4*>(cols + (static_cast<int64_t>(p) * ng + gi) * M * 16 + (iy & 15));
    float2 x[kRegPts], y[kRegPts];
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) {
        const float4 v = src[static_cast<int64_t>(tid + B * s) * 8];
        x[s] = make_float2(v.x, 0.0f - v.y);
        y[s] = make_float2(v.z, 0.0f - v.w);
    }
    const int z0 = 2 * p;
    const bool has1 = z0 + 1 < rows;
    OutT* o0 = vol + (static_cast<int64_t>(z0) * N + iy) * N;
    OutT* o1 = o0 + static_cast<int64_t>(N) * N;
    // each row is transformed and stored before the next one is transformed
    auto finish = [&](float2 (&v)[kRegPts], int row) {
        reg_fft<M>(v, lds, tw, tid);
        const float fy = t.D[iy + row];
#pragma unroll
        for (int s = 0; s < kRegPts; ++s) {
            const int m = tid + B * s;
            const int x0 = m < M / 2 ? m : m - M;
            const int ix = x0 + hN;
            if (ix >= 0 && ix < N) {
                const float f = t.D[ix] * fy;
                fr_store(o0, row * N + ix, v[s].x * f);
                if (has1) fr_store(o1, row * N + ix, (0.0f - v[s].y) * f);
            }
        }
    };
    finish(x, 0);
    if (iy + 1 < N) finish(y, 1);
}

size_t reg_lds(int L) { return static_cast<size_t>(L + L / 16) * sizeof(float2); }

template <int NT>
hipError_t launch_grid_nt(const FourierTables& t, const float2* spec, int pairs, float2* grid, hipStream_t st) {
    const size_t lds = static_cast<size_t>(kFrBatch) * t.sw * sizeof(float4);
    hipError_t e = fr_lds(k_fr_grid<NT>, lds);
    if (e != hipSuccess) return e;
    const dim3 g(static_cast<unsigned>(static_cast<int64_t>(pairs) * t.ntiles));
    hipLaunchKernelGGL((k_fr_grid<NT>), g, dim3(256), lds, st, t, spec, grid);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fourier_spectra(const RawInput& in, int rows, const float* dmean, const float* rden,
                                  const float2* tw_L, const FourierTables& t, float2* spec, hipStream_t st) {
    const int pairs = (rows + 1) / 2;
#define TP_FR_REG(LL)                                                                                      \
    case LL: {                                                                                            \
        const int64_t ag = (t.na + kFrAnglesPerGroup - 1) / kFrAnglesPerGroup;                             \
        const dim3 g(static_cast<unsigned>(static_cast<int64_t>(pairs) * ag));                            \
        const hipError_t e = fr_lds(k_fr_spectra_reg<LL>, reg_lds(LL));                                   \
        if (e != hipSuccess) return e;                                                                    \
        hipLaunchKernelGGL((k_fr_spectra_reg<LL>), g, dim3(LL / kRegPts), reg_lds(LL), st, in, rows, dmean, rden, \
                           tw_L, t, spec);                                                               \
        return hipGetLastError();                                                                         \
    }
    switch (t.L) {
        TP_FR_REG(1024)
        TP_FR_REG(2048)
        TP_FR_REG(4096)
        TP_FR_REG(8192)
        default: break;
    }
#undef TP_FR_REG
    const size_t lds = static_cast<size_t>(t.L) * sizeof(float2);
    hipError_t e = fr_lds(k_fr_spectra, lds);
    if (e != hipSuccess) return e;
    const dim3 grid(static_cast<unsigned>(static_cast<int64_t>(pairs) * t.na));
    hipLaunchKernelGGL(k_fr_spectra, grid, dim3(fr_block(t.L)), lds, st, in, rows, dmean, rden, tw_L, t, spec);
    return hipGetLastError();
}

size_t fourier_grid_tiles(int M) {
    const size_t tps = static_cast<size_t>(M) / kFrTile;
    return tps * (tps / 2) + tps;  // rows with uy >= 0, plus the row holding uy = -M/2
}

hipError_t launch_fourier_grid(const FourierTables& t, const float2* spec, int pairs, float2* grid, hipStream_t st) {
    switch (t.nt) {
        case 2: return launch_grid_nt<2>(t, spec, pairs, grid, st);
        case 4: return launch_grid_nt<4>(t, spec, pairs, grid, st);
        case 6: return launch_grid_nt<6>(t, spec, pairs, grid, st);
        case 8: return launch_grid_nt<8>(t, spec, pairs, grid, st);
        case 10: return launch_grid_nt<10>(t, spec, pairs, grid, st);
        case 12: return launch_grid_nt<12>(t, spec, pairs, grid, st);
        case 14: return launch_grid_nt<14>(t, spec, pairs, grid, st);
        case 16: return launch_grid_nt<16>(t, spec, pairs, grid, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fourier_rows(const FourierTables& t, const float2* tw_M, const float2* grid, int pairs,
                               float2* cols, hipStream_t st) {
#define TP_FR_REG(MM)                                                                                      \
    case MM: {                                                                                            \
        const dim3 g(static_cast<unsigned>(static_cast<int64_t>(pairs) * MM));                            \
        const hipError_t e = fr_lds(k_fr_rows_reg<MM>, reg_lds(MM));                                      \
        if (e != hipSuccess) return e;                                                                    \
        hipLaunchKernelGGL((k_fr_rows_reg<MM>), g, dim3(MM / kRegPts), reg_lds(MM), st, grid, tw_M, t, cols); \
        return hipGetLastError();                                                                         \
    }
    switch (t.M) {
        TP_FR_REG(1024)
        TP_FR_REG(2048)
        TP_FR_REG(4096)
        TP_FR_REG(8192)
        default: break;
    }
#undef TP_FR_REG
    const size_t lds = static_cast<size_t>(t.M) * sizeof(float2);
    hipError_t e = fr_lds(k_fr_rows, lds);
    if (e != hipSuccess) return e;
    const dim3 g(static_cast<unsigned>(static_cast<int64_t>(pairs) * t.M));
    hipLaunchKernelGGL(k_fr_rows, g, dim3(fr_block(t.M)), lds, st, grid, tw_M, t, cols);
    return hipGetLastError();
}

namespace {
template <typename OutT>
hipError_t launch_fourier_cols_t(const FourierTables& t, const float2* tw_M, const float2* cols, int pairs, int rows,
                                 OutT* vol, hipStream_t st) {
    const int64_t groups = static_cast<int64_t>(pairs) * ((t.N + 15) / 16);
    const dim3 g(static_cast<unsigned>(((groups + 7) / 8) * 8 * 16));
    const dim3 g2(static_cast<unsigned>(((groups + 7) / 8) * 8 * 8));  // two rows per work-group
#define TP_FR_REG(MM)                                                                                      \
    case MM: {                                                                                            \
        const hipError_t e = fr_lds(k_fr_cols_reg<MM, OutT>, reg_lds(MM));                                \
        if (e != hipSuccess) return e;                                                                    \
        hipLaunchKernelGGL((k_fr_cols_reg<MM, OutT>), g2, dim3(MM / kRegPts), reg_lds(MM), st, cols, tw_M, t, pairs, \
                           rows, vol);                                                                    \
        return hipGetLastError();                                                                         \
    }
    switch (t.M) {
        TP_FR_REG(1024)
        TP_FR_REG(2048)
        TP_FR_REG(4096)
        TP_FR_REG(8192)
        default: break;
    }
#undef TP_FR_REG
    const size_t lds = static_cast<size_t>(t.M) * sizeof(float2);
    hipError_t e = fr_lds(k_fr_cols<OutT>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fr_cols<OutT>, g, dim3(fr_block(t.M)), lds, st, cols, tw_M, t, pairs, rows, vol);
    return hipGetLastError();
}
}  // namespace

// vol: FP32 slices, or FP16 (`half_out`: each voxel's FP32 value rounded once).
hipError_t launch_fourier_cols(const FourierTables& t, const float2* tw_M, const float2* cols, int pairs, int rows,
                               void* vol, bool half_out, hipStream_t st) {
    if (half_out) return launch_fourier_cols_t(t, tw_M, cols, pairs, rows, static_cast<__half*>(vol), st);
    return launch_fourier_cols_t(t, tw_M, cols, pairs, rows, static_cast<float*>(vol), st);
}

}  // namespace tp
