// Log-polar-based backprojection (paper, Sections 2.2 and 3: the backprojection
// over a range of equally spaced angles is a convolution in log-polar
// coordinates, computed with FFTs, with spline interpolations to and from the
// log-polar grid in the image domain).
//
// For a span of angles phi_k (rotated so that they are centred on zero) and
// the image moved by a0 along the first axis, a voxel at x'' = e^rho (cos psi,
// sin psi) sees the ray offset e^rho cos(psi - phi_k), so the span's
// backprojection is
//   F(psi, rho) = dtheta sum_k G_k(rho + log cos(psi - phi_k)),
//   G_k(sigma) = Y_a(e^sigma - a0 cos phi_k + pos0),
// a convolution over (angle, log-radius).  Along sigma it is a shift, exact
// in the DFT domain; along psi a linear convolution of the spectra G^_k(eta)
// placed at every M-th fine-angle index with exp(2 pi i eta log cos(d dpsi) /
// (delta Ns)), done with FFTs of length NA.
//
// Two slices travel as the real and imaginary parts of one complex sequence
// throughout (every operator maps real data to real data).
//
// Stages (one launch each, per batch of slice pairs):
//   k_lp_rows       normalise two rows, pad, FFT, multiply by the filter and
//                   the quintic B-spline prefilter at half-sample spacing,
//                   two inverse FFTs (even and odd half-samples): B-spline
//                   coefficients of each row's trigonometric interpolant;
//   k_lp_logradial  per (span, angle slot): G_k(sigma_j) from six coefficient
//                   taps at FP64 positions, tapered, FFT over sigma;
//   k_lp_conv       per (span, eta): the kernel column exp(...) over d, FFT,
//                   prefilter and scale folded in (built once per launch);
//                   per pair: FFT of the angle column, tiled M times,
//                   multiply, inverse FFT, keep the rows of the image sector;
//   k_lp_sigma      per (span, two rows): inverse FFT over eta, keep the rho
//                   window: B-spline coefficients of F on the log-polar grid;
//   k_lp_interp     per voxel: coordinates of every span in FP64 once, then
//                   the 6 x 6 quintic taps of every span for every pair.
#include <algorithm>

#include "fft_device.h"

namespace tp {
namespace {

__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, 0.0f - a.y); }

// Centred quintic B-spline at the six taps floor(u) - 2 .. floor(u) + 3 for
// fraction f = u - floor(u) in [0, 1): w[i] = beta5(f + 2 - i).
__device__ __forceinline__ void quintic_weights(float f, float (&w)[6]) {
    const float g = 1.0f - f;
    // |x| < 1 piece: 11/20 - x^2/2 + x^4/4 - x^5/12
    auto inner = [](float x) {
        const float x2 = x * x;
        return 0.55f + x2 * (-0.5f + x2 * (0.25f - x * (1.0f / 12.0f)));
    };
    // 1 <= |x| < 2 piece: 17/40 + 5x/8 - 7x^2/4 + 5x^3/4 - 3x^4/8 + x^5/24
    auto middle = [](float x) {
        return 0.425f + x * (0.625f + x * (-1.75f + x * (1.25f + x * (-0.375f + x * (1.0f / 24.0f)))));
    };
    const float g2 = g * g, f2 = f * f;
    w[0] = g2 * g2 * g * (1.0f / 120.0f);
    w[1] = middle(f + 1.0f);
    w[2] = inner(f);
    w[3] = inner(g);
    w[4] = middle(g + 1.0f);
    w[5] = f2 * f2 * f * (1.0f / 120.0f);
}

template <typename K>
hipError_t lds_limit(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(bytes));
}

size_t reg_lds_bytes(int L) { return static_cast<size_t>(L + L / 16) * sizeof(float2); }

int rows_block(int L) { return L / 16 < 64 ? 64 : (L / 16 > 1024 ? 1024 : L / 16); }

// ---------------------------------------------------------------------------
// Row splines: one work-group per (angle, pair of slices).
// ---------------------------------------------------------------------------
constexpr int kRowSlots = 16;  // L / blockDim elements per thread (blockDim >= L / 16)

__global__ void __launch_bounds__(512)
k_lp_rows(RawInput in, int rows, const float* __restrict__ dmean, const float* __restrict__ rden, LprecTables t,
          float2* __restrict__ out) {
    extern __shared__ float2 buf[];
    const int a = blockIdx.x, p = blockIdx.y;
    const int L = t.L, n = t.n, off = (L - n) / 2, B = blockDim.x, tid = threadIdx.x;
    const int z0 = 2 * p;
    const bool has1 = z0 + 1 < rows;
    const int64_t r0 = static_cast<int64_t>(z0) * n;
    const int64_t r1 = has1 ? r0 + n : r0;
    const uint16_t* q0 = in.proj + a * in.proj_stride + r0;
    const uint16_t* q1 = in.proj + a * in.proj_stride + r1;
    for (int m = tid; m < L; m += B) {
        const int c = min(max(m - off, 0), n - 1);
        buf[m] = make_float2(neglog_counts(static_cast<float>(q0[c]), dmean[r0 + c], rden[r0 + c]),
                             has1 ? neglog_counts(static_cast<float>(q1[c]), dmean[r1 + c], rden[r1 + c]) : 0.0f);
    }
    __syncthreads();
    fft_forward_lds(buf, L, t.log2L, t.twL);
    float2 X[kRowSlots];
#pragma unroll
    for (int s = 0; s < kRowSlots; ++s) {
        const int k = tid + B * s;
        X[s] = k < L ? buf[k] : make_float2(0.0f, 0.0f);
    }
    float2* dst = out + (static_cast<int64_t>(p) * t.na + a) * (2 * L);
#pragma unroll 1
    for (int b = 0; b < 2; ++b) {
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kRowSlots; ++s) {
            const int k = tid + B * s;
            if (k < L) {
                const float2 v = b == 0 ? make_float2(X[s].x * t.T0[k], X[s].y * t.T0[k]) : cmul(X[s], t.T1[k]);
                buf[k] = cconj(v);
            }
        }
        __syncthreads();
        fft_forward_lds(buf, L, t.log2L, t.twL);
        for (int i = tid; i < L; i += B) dst[2 * i + b] = cconj(buf[i]);
    }
}

// ---------------------------------------------------------------------------
// Log-radial samples and their spectra: one work-group per (angle slot of a
// span, pair).  Output layout [pair][span][eta / 16][slot][16].
// ---------------------------------------------------------------------------
template <int NS>
__global__ void __launch_bounds__(NS / kRegPts)
k_lp_logradial(const float2* __restrict__ rows, LprecTables t, float2* __restrict__ ghat) {
    extern __shared__ float2 lds[];
    constexpr int B = NS / kRegPts;
    const int tid = threadIdx.x;
    const int slot = blockIdx.x, p = blockIdx.y;
    const int span = slot / t.n_span, k = slot - span * t.n_span;
    const int a = span * t.n_span + k;
    float2* dst = ghat + (static_cast<int64_t>(p) * t.spans + span) * (NS / 16) * t.n_span * 16 + k * 16;
    if (a >= t.na) {  // empty slot of the last span
#pragma unroll
        for (int s = 0; s < kRegPts; ++s) {
            const int eta = tid + B * s;
            dst[static_cast<int64_t>(eta >> 4) * t.n_span * 16 + (eta & 15)] = make_float2(0.0f, 0.0f);
        }
        return;
    }
    const int L2 = 2 * t.L;
    const float2* src = rows + (static_cast<int64_t>(p) * t.na + a) * L2;
    for (int i = tid; i < L2; i += B) lds[i] = src[i];
    __syncthreads();
    const double Ak = t.A[k];
    float2 x[kRegPts];
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) {
        const int j = tid + B * s;
        const double u = 2.0 * (t.E[j] - Ak);
        const double fl = floor(u);
        const int i0 = static_cast<int>(fl);
        float w[6];
        quintic_weights(static_cast<float>(u - fl), w);
        float2 acc = make_float2(0.0f, 0.0f);
#pragma unroll
        for (int o = 0; o < 6; ++o) {
            const float2 c = lds[(i0 + o - 2) & (L2 - 1)];
            acc.x = __builtin_fmaf(w[o], c.x, acc.x);
            acc.y = __builtin_fmaf(w[o], c.y, acc.y);
        }
        const float tw = t.taper[j];
        x[s] = make_float2(acc.x * tw, acc.y * tw);
    }
    __syncthreads();  // the coefficient row is dead; the FFT reuses the LDS
    reg_fft<NS>(x, lds, t.twNs, tid);
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) {
        const int eta = tid + B * s;
        dst[static_cast<int64_t>(eta >> 4) * t.n_span * 16 + (eta & 15)] = x[s];
    }
}

// ---------------------------------------------------------------------------
// Convolution over the angle: one work-group per (span, eta), looping over the
// pairs.  Work-groups are dealt to the 8 XCDs so that the 16 eta of one
// 128-byte line of the input run back to back on one XCD.  Output layout
// [pair][span][m / 16][eta][16].
// ---------------------------------------------------------------------------
template <int NA>
__global__ void __launch_bounds__(NA / kRegPts)
k_lp_conv(const float2* __restrict__ ghat, LprecTables t, int pairs, float2* __restrict__ fhat) {
    extern __shared__ float2 lds[];
    constexpr int B = NA / kRegPts;
    const int tid = threadIdx.x;
    const int NS = t.Ns;
    const int id = blockIdx.x;
    const int xcd = id & 7, r = id >> 3;
    const int c = ((r >> 4) * 8 + xcd) * 16 + (r & 15);
    const int span = c / NS, eta = c - span * NS;
    const int eta_s = eta < NS / 2 ? eta : eta - NS;
    const bool nyq = eta == NS / 2;
    // kernel column over d = d_lo + d', transformed once
    float2 Kh[kRegPts];
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) {
        const int d = tid + B * s;
        float2 v = make_float2(0.0f, 0.0f);
        if (d < t.D) {
            double ph = static_cast<double>(eta_s) * t.cd[d];
            ph -= floor(ph);
            float sn, cs;
            sincospif(2.0f * static_cast<float>(ph), &sn, &cs);
            v = nyq ? make_float2(cs, 0.0f) : make_float2(cs, sn);
        }
        Kh[s] = v;
    }
    reg_fft<NA>(Kh, lds, t.twNA, tid);
    const float cscale = t.colscale[eta];
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) {
        const float f = t.preA[tid + B * s] * cscale;
        Kh[s] = make_float2(Kh[s].x * f, Kh[s].y * f);
    }
    const int first = t.M * (t.n_span - 1);
    const int NAc = t.NAc;
#pragma unroll 1
    for (int p = 0; p < pairs; ++p) {
        const float2* src = ghat + ((static_cast<int64_t>(p) * t.spans + span) * (NS / 16) + (eta >> 4)) *
                                       t.n_span * 16 + (eta & 15);
        __syncthreads();
        for (int k = tid; k < NAc; k += B)
            lds[k] = k < t.n_span ? src[static_cast<int64_t>(k) * 16] : make_float2(0.0f, 0.0f);
        __syncthreads();
        fft_forward_lds(lds, NAc, t.log2NAc, t.twNAc);
        float2 x[kRegPts];
#pragma unroll
        for (int s = 0; s < kRegPts; ++s) x[s] = cconj(cmul(lds[(tid + B * s) & (NAc - 1)], Kh[s]));
        __syncthreads();
        reg_fft<NA>(x, lds, t.twNA, tid);
        float2* dst = fhat + (static_cast<int64_t>(p) * t.spans + span) * t.nmb * NS * 16;
#pragma unroll
        for (int s = 0; s < kRegPts; ++s) {
            const int m = tid + B * s - first;
            if (m >= 0 && m < t.rows)
                dst[(static_cast<int64_t>(m >> 4) * NS + eta) * 16 + (m & 15)] = cconj(x[s]);
        }
    }
}

// The same convolution for NA = 8192 and 16384.  Beside a kernel column held
// in registers the register transform of these lengths spills, so the column
// (transformed, prefilter and scale folded in) is built once per plan into a
// table kt[eta][nu] (k_lp_ktable) and read per pair; the 3 spans share it.
template <int NA>
__global__ void __launch_bounds__(NA / kRegPts)
k_lp_ktable(LprecTables t, float2* __restrict__ kt) {
    extern __shared__ float2 lds[];
    constexpr int B = NA / kRegPts;
    const int tid = threadIdx.x;
    const int NS = t.Ns;
    const int eta = blockIdx.x;
    const int eta_s = eta < NS / 2 ? eta : eta - NS;
    const bool nyq = eta == NS / 2;
    float2 x[kRegPts];
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) {
        const int d = tid + B * s;
        float2 v = make_float2(0.0f, 0.0f);
        if (d < t.D) {
            double ph = static_cast<double>(eta_s) * t.cd[d];
            ph -= floor(ph);
            float sn, cs;
            sincospif(2.0f * static_cast<float>(ph), &sn, &cs);
            v = nyq ? make_float2(cs, 0.0f) : make_float2(cs, sn);
        }
        x[s] = v;
    }
    reg_fft<NA>(x, lds, t.twNA, tid);
    const float cscale = t.colscale[eta];
    float2* dst = kt + static_cast<int64_t>(eta) * NA;
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) {
        const float f = t.preA[tid + B * s] * cscale;
        dst[tid + B * s] = make_float2(x[s].x * f, x[s].y * f);
    }
}

// One (span, eta, pair) per work-group (a 16-wave work-group fills a CU, so
// nothing is gained by looping over pairs inside it).  On each XCD the 16 eta
// of one 128-byte line of the input run for every (span, pair) in turn:
// the line is fetched once, and the 16 kernel columns (2 MB) are read from
// that XCD's L2 after their first use.
template <int NA>
__global__ void __launch_bounds__(NA / kRegPts)
k_lp_conv_tab(const float2* __restrict__ ghat, LprecTables t, int pairs, float2* __restrict__ fhat) {
    extern __shared__ float2 lds[];
    constexpr int B = NA / kRegPts;
    const int tid = threadIdx.x;
    const int NS = t.Ns;
    const int id = blockIdx.x;
    const int xcd = id & 7, r = id >> 3;
    const int per = t.spans * pairs * 16;  // work-groups per 16-eta group on one XCD
    const int G = r / per, rem = r - G * per;
    const int sp = rem >> 4;
    const int span = sp / pairs, p = sp - span * pairs;
    const int eta = (G * 8 + xcd) * 16 + (rem & 15);
    const float2* kcol = t.kt + static_cast<int64_t>(eta) * NA;
    const int first = t.M * (t.n_span - 1);
    const int NAc = t.NAc;
    const float2* src = ghat + ((static_cast<int64_t>(p) * t.spans + span) * (NS / 16) + (eta >> 4)) *
                                   t.n_span * 16 + (eta & 15);
    for (int k = tid; k < NAc; k += B)
        lds[k] = k < t.n_span ? src[static_cast<int64_t>(k) * 16] : make_float2(0.0f, 0.0f);
    __syncthreads();
    fft_forward_lds(lds, NAc, t.log2NAc, t.twNAc);
    float2 x[kRegPts];
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) x[s] = cconj(cmul(lds[(tid + B * s) & (NAc - 1)], kcol[tid + B * s]));
    __syncthreads();
    reg_fft<NA>(x, lds, t.twNA, tid);
    float2* dst = fhat + (static_cast<int64_t>(p) * t.spans + span) * t.nmb * NS * 16;
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) {
        const int m = tid + B * s - first;
        if (m >= 0 && m < t.rows) dst[(static_cast<int64_t>(m >> 4) * NS + eta) * 16 + (m & 15)] = cconj(x[s]);
    }
}

// ---------------------------------------------------------------------------
// Inverse transform over sigma: one work-group per (pair, span, two rows);
// the 8 work-groups of one 16-row line group run back to back on one XCD.
// Output F [pair][span][row][nj] (the rho window).
// ---------------------------------------------------------------------------
template <int NS>
__global__ void __launch_bounds__(NS / kRegPts)
k_lp_sigma(const float2* __restrict__ fhat, LprecTables t, int pairs, float2* __restrict__ F) {
    extern __shared__ float2 lds[];
    constexpr int B = NS / kRegPts;
    const int tid = threadIdx.x;
    const int id = blockIdx.x;
    const int xcd = id & 7, r = id >> 3;
    const int r2 = r & 7;
    const int64_t gidx = static_cast<int64_t>(r >> 3) * 8 + xcd;
    const int64_t G = static_cast<int64_t>(pairs) * t.spans * t.nmb;
    if (gidx >= G) return;  // whole work-group
    const int mb = static_cast<int>(gidx % t.nmb);
    const int64_t ps = gidx / t.nmb;  // pair * spans + span
    const int m = mb * 16 + 2 * r2;
    if (m >= t.rows) return;
    const float4* src = reinterpret_cast<const float4*>(fhat + (ps * t.nmb + mb) * NS * 16 + (m & 15));
    float2 x[kRegPts], y[kRegPts];
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) {
        const float4 v = src[static_cast<int64_t>(tid + B * s) * 8];
        x[s] = make_float2(v.x, 0.0f - v.y);
        y[s] = make_float2(v.z, 0.0f - v.w);
    }
    auto finish = [&](float2 (&v)[kRegPts], int row) {
        reg_fft<NS>(v, lds, t.twNs, tid);
        float2* dst = F + (ps * t.rows + row) * t.nj;
#pragma unroll
        for (int s = 0; s < kRegPts; ++s) {
            const int j = tid + B * s - t.j_lo;
            if (j >= 0 && j < t.nj) dst[j] = cconj(v[s]);
        }
    };
    finish(x, m);
    if (m + 1 < t.rows) finish(y, m + 1);
}

// ---------------------------------------------------------------------------
// Evaluation at the voxels: one thread per voxel of a 16 x 16 tile, every
// pair of the launch.
// ---------------------------------------------------------------------------
constexpr int kMaxSpans = 4;  // the host refuses more spans

__global__ void __launch_bounds__(256)
k_lp_interp(const float2* __restrict__ F, LprecTables t, int pairs, int rows, float* __restrict__ vol) {
    const int N = t.N;
    const int tiles = (N + 15) / 16;
    const int by = blockIdx.x / tiles, bx = blockIdx.x - by * tiles;
    const int ix = bx * 16 + (threadIdx.x & 15), iy = by * 16 + (threadIdx.x >> 4);
    if (ix >= N || iy >= N) return;
    const double x = static_cast<double>(ix - N / 2), y = static_cast<double>(iy - N / 2);
    int base[kMaxSpans];
    float wm[kMaxSpans][6], wj[kMaxSpans][6];
#pragma unroll
    for (int sp = 0; sp < kMaxSpans; ++sp) {
        if (sp >= t.spans) break;
        const double xp = t.cb[sp] * x + t.sb[sp] * y + t.a0;
        const double yp = t.cb[sp] * y - t.sb[sp] * x;
        const double rho = 0.5 * log(xp * xp + yp * yp);
        const double psi = atan2(yp, xp);
        const double tj = (rho - t.sigma0) / t.delta - t.j_lo;
        const double tm = (psi - t.phi0) / t.dpsi - t.m_lo;
        const double fj = floor(tj), fm = floor(tm);
        quintic_weights(static_cast<float>(tj - fj), wj[sp]);
        quintic_weights(static_cast<float>(tm - fm), wm[sp]);
        base[sp] = (static_cast<int>(fm) - 2) * t.nj + static_cast<int>(fj) - 2;
    }
    const int64_t plane = static_cast<int64_t>(t.rows) * t.nj;
    const int64_t NN = static_cast<int64_t>(N) * N;
#pragma unroll 1
    for (int p = 0; p < pairs; ++p) {
        float ax = 0.0f, ay = 0.0f;
#pragma unroll
        for (int sp = 0; sp < kMaxSpans; ++sp) {
            if (sp >= t.spans) break;
            const float2* f = F + (static_cast<int64_t>(p) * t.spans + sp) * plane + base[sp];
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                float rx = 0.0f, ry = 0.0f;
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    const float2 v = f[i * t.nj + q];
                    rx = __builtin_fmaf(wj[sp][q], v.x, rx);
                    ry = __builtin_fmaf(wj[sp][q], v.y, ry);
                }
                ax = __builtin_fmaf(wm[sp][i], rx, ax);
                ay = __builtin_fmaf(wm[sp][i], ry, ay);
            }
        }
        const int z0 = 2 * p;
        const int64_t o = static_cast<int64_t>(iy) * N + ix;
        vol[z0 * NN + o] = ax;
        if (z0 + 1 < rows) vol[(z0 + 1) * NN + o] = ay;
    }
}

template <int NS>
hipError_t launch_logradial_t(const LprecTables& t, const float2* rows, int pairs, float2* ghat, hipStream_t st) {
    const size_t lds = std::max(reg_lds_bytes(NS), static_cast<size_t>(2 * t.L) * sizeof(float2));
    hipLaunchKernelGGL(k_lp_logradial<NS>, dim3(t.spans * t.n_span, pairs), dim3(NS / kRegPts), lds, st, rows, t,
                       ghat);
    return hipGetLastError();
}

size_t conv_lds_bytes(int NA, int NAc) {
    return std::max(reg_lds_bytes(NA), static_cast<size_t>(NAc) * sizeof(float2));
}

template <int NA>
hipError_t launch_conv_t(const LprecTables& t, const float2* ghat, int pairs, float2* fhat, hipStream_t st) {
    const size_t lds = conv_lds_bytes(NA, t.NAc);
    if constexpr (NA >= 8192) {
        // one work-group per (span, eta, pair); the eta-group order needs Ns / 16 divisible by 8
        if (static_cast<int64_t>(t.spans) * t.Ns * pairs > 0x7fffffff || (t.Ns / 16) % 8 != 0)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_lp_conv_tab<NA>, dim3(t.spans * t.Ns * pairs), dim3(NA / kRegPts), lds, st, ghat, t,
                           pairs, fhat);
    } else {
        hipLaunchKernelGGL(k_lp_conv<NA>, dim3(t.spans * t.Ns), dim3(NA / kRegPts), lds, st, ghat, t, pairs, fhat);
    }
    return hipGetLastError();
}

template <int NA>
hipError_t launch_ktable_t(const LprecTables& t, float2* kt, hipStream_t st) {
    if constexpr (NA >= 8192) {
        hipLaunchKernelGGL(k_lp_ktable<NA>, dim3(t.Ns), dim3(NA / kRegPts), reg_lds_bytes(NA), st, t, kt);
        return hipGetLastError();
    } else {
        return hipSuccess;
    }
}

template <int NS>
hipError_t launch_sigma_t(const LprecTables& t, const float2* fhat, int pairs, float2* F, hipStream_t st) {
    const int64_t G = static_cast<int64_t>(pairs) * t.spans * t.nmb;
    const int64_t blocks = ((G + 7) / 8) * 64;
    hipLaunchKernelGGL(k_lp_sigma<NS>, dim3(static_cast<unsigned>(blocks)), dim3(NS / kRegPts), reg_lds_bytes(NS),
                       st, fhat, t, pairs, F);
    return hipGetLastError();
}

#define TP_LP_DISPATCH(len, fn, ...)                      \
    switch (len) {                                        \
        case 1024: return fn<1024>(__VA_ARGS__);          \
        case 2048: return fn<2048>(__VA_ARGS__);          \
        case 4096: return fn<4096>(__VA_ARGS__);          \
        case 8192: return fn<8192>(__VA_ARGS__);          \
        case 16384: return fn<16384>(__VA_ARGS__);        \
        default: return hipErrorInvalidValue;             \
    }

template <int NS>
hipError_t prep_ns(const LprecTables& t) {
    hipError_t e = lds_limit(k_lp_logradial<NS>, std::max(reg_lds_bytes(NS), static_cast<size_t>(2 * t.L) * 8));
    if (e != hipSuccess) return e;
    return lds_limit(k_lp_sigma<NS>, reg_lds_bytes(NS));
}

template <int NA>
hipError_t prep_na(const LprecTables& t) {
    if constexpr (NA >= 8192) {
        hipError_t e = lds_limit(k_lp_ktable<NA>, reg_lds_bytes(NA));
        if (e != hipSuccess) return e;
        return lds_limit(k_lp_conv_tab<NA>, conv_lds_bytes(NA, t.NAc));
    } else {
        return lds_limit(k_lp_conv<NA>, conv_lds_bytes(NA, t.NAc));
    }
}

}  // namespace

hipError_t prepare_lprec(const LprecTables& t) {
    hipError_t e = lds_limit(k_lp_rows, static_cast<size_t>(t.L) * sizeof(float2));
    if (e != hipSuccess) return e;
    e = [&]() -> hipError_t { TP_LP_DISPATCH(t.Ns, prep_ns, t) }();
    if (e != hipSuccess) return e;
    TP_LP_DISPATCH(t.NA, prep_na, t)
}

hipError_t launch_lprec_rows(const RawInput& in, int rows, const float* dmean, const float* rden,
                             const LprecTables& t, float2* out, hipStream_t st) {
    const int pairs = (rows + 1) / 2;
    hipLaunchKernelGGL(k_lp_rows, dim3(t.na, pairs), dim3(rows_block(t.L)), static_cast<size_t>(t.L) * sizeof(float2),
                       st, in, rows, dmean, rden, t, out);
    return hipGetLastError();
}

hipError_t launch_lprec_logradial(const LprecTables& t, const float2* rows, int pairs, float2* ghat,
                                  hipStream_t st) {
    TP_LP_DISPATCH(t.Ns, launch_logradial_t, t, rows, pairs, ghat, st)
}

hipError_t launch_lprec_conv(const LprecTables& t, const float2* ghat, int pairs, float2* fhat, hipStream_t st) {
    TP_LP_DISPATCH(t.NA, launch_conv_t, t, ghat, pairs, fhat, st)
}

size_t lprec_ktable_bytes(int Ns, int NA) {
    return NA >= 8192 ? static_cast<size_t>(Ns) * NA * sizeof(float2) : 0;
}

hipError_t launch_lprec_ktable(const LprecTables& t, float2* kt, hipStream_t st) {
    TP_LP_DISPATCH(t.NA, launch_ktable_t, t, kt, st)
}

hipError_t launch_lprec_sigma(const LprecTables& t, const float2* fhat, int pairs, float2* F, hipStream_t st) {
    TP_LP_DISPATCH(t.Ns, launch_sigma_t, t, fhat, pairs, F, st)
}

hipError_t launch_lprec_interp(const LprecTables& t, const float2* F, int pairs, int rows, float* vol,
                               hipStream_t st) {
    const int tiles = (t.N + 15) / 16;
    hipLaunchKernelGGL(k_lp_interp, dim3(tiles * tiles), dim3(256), 0, st, F, t, pairs, rows, vol);
    return hipGetLastError();
}

}  // namespace tp
