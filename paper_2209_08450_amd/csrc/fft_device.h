// Device FFT building blocks shared by the filter kernels and the
// Fourier-domain backprojection: complex helpers, an LDS Stockham radix-4
// transform for any power-of-two length up to 16384, and a register-resident
// radix-16 transform for 1024 <= L <= 8192.  Everything has internal linkage
// (anonymous namespace), so each translation unit gets its own copy.
#pragma once

#include "tp_internal.h"

namespace tp {
namespace {

constexpr int kMaxPerThread4 = 4;  // radix-4 butterflies per thread (L / (4 B) with B = L / 16)

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// multiply by -i
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }

// In-place forward DFT X[k] = sum_m x[m] exp(-2 pi i k m / L) of buf[0..L),
// with at most PT4 radix-4 butterflies (2 PT4 radix-2 ones) per thread, so
// blockDim.x >= L / (4 PT4).  Caller must have synchronised after writing buf;
// returns synchronised.
template <int PT4 = kMaxPerThread4>
__device__ void fft_forward_lds(float2* buf, int L, int log2L, const float2* __restrict__ tw) {
    constexpr int PT2 = 2 * PT4;
    const int tid = threadIdx.x;
    const int B = blockDim.x;
    int Ns = 1;
    if (log2L & 1) {
        const int h = L >> 1;
        float2 v0[PT2], v1[PT2];
#pragma unroll
        for (int c = 0; c < PT2; ++c) {
            const int j = tid + c * B;
            if (j < h) { v0[c] = buf[j]; v1[c] = buf[j + h]; }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < PT2; ++c) {
            const int j = tid + c * B;
            if (j < h) { buf[2 * j] = cadd(v0[c], v1[c]); buf[2 * j + 1] = csub(v0[c], v1[c]); }
        }
        __syncthreads();
        Ns = 2;
    }
    const int q = L >> 2;
    for (; Ns < L; Ns <<= 2) {
        const int tstride = L / (Ns << 2);
        float2 v[PT4][4];
#pragma unroll
        for (int c = 0; c < PT4; ++c) {
            const int j = tid + c * B;
            if (j < q) {
                const int k = j & (Ns - 1);
                const int t1 = k * tstride;
                float2 x0 = buf[j];
                float2 x1 = buf[j + q];
                float2 x2 = buf[j + 2 * q];
                float2 x3 = buf[j + 3 * q];
                if (Ns > 1) {
                    x1 = cmul(x1, tw[t1]);
                    x2 = cmul(x2, tw[(2 * t1) & (L - 1)]);
                    x3 = cmul(x3, tw[(3 * t1) & (L - 1)]);
                }
                const float2 a0 = cadd(x0, x2), a1 = csub(x0, x2);
                const float2 a2 = cadd(x1, x3), a3 = cmul_mi(csub(x1, x3));
                v[c][0] = cadd(a0, a2);
                v[c][1] = cadd(a1, a3);
                v[c][2] = csub(a0, a2);
                v[c][3] = csub(a1, a3);
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < PT4; ++c) {
            const int j = tid + c * B;
            if (j < q) {
                const int k = j & (Ns - 1);
                const int d = ((j - k) << 2) + k;
                buf[d] = v[c][0];
                buf[d + Ns] = v[c][1];
                buf[d + 2 * Ns] = v[c][2];
                buf[d + 3 * Ns] = v[c][3];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Register-resident variant for 1024 <= L <= 8192 (16384 would spill): B = L/16 threads, thread t
// holds the 16 elements t + B*s (s = 0..15) in registers.  Stockham passes of
// radix 16 (and one radix 2/4/8 pass when log2 L is not a multiple of 4):
// in a radix-R pass thread t runs 16/R butterflies j = t + B*c; butterfly j
// needs elements j + (L/R) r = t + B*(c + (16/R) r), i.e. its own slots, so
// every pass reads registers, and only the pass outputs are exchanged
// through LDS (written at the Stockham destinations, read back at t + B*s).
// After the last pass the outputs j + (L/R) r are again the thread's own
// slots, in natural order, so the spectrum is multiplied by H and the
// inverse transform starts without an exchange; loading (with normalisation
// and edge padding) and the cropped store go straight between HBM and
// registers.
// ---------------------------------------------------------------------------
template <int R> struct Dft;
template <> struct Dft<2> {
    __device__ __forceinline__ static void run(float2* v) {
        const float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};
template <> struct Dft<4> {
    __device__ __forceinline__ static void run(float2* v) {
        const float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        const float2 a2 = cadd(v[1], v[3]), a3 = cmul_mi(csub(v[1], v[3]));
        v[0] = cadd(a0, a2);
        v[1] = cadd(a1, a3);
        v[2] = csub(a0, a2);
        v[3] = csub(a1, a3);
    }
};
// exp(-2 pi i k / R) for R in {8, 16}, k < R/2 (FP32 roundings of the exact values)
template <int R>
__device__ __forceinline__ float2 wconst(int k) {
    constexpr float c1 = 0.923879532511286756f, s1 = 0.382683432365089772f, h = 0.707106781186547524f;
    if (R == 8) {
        switch (k) {
            case 0: return make_float2(1.0f, 0.0f);
            case 1: return make_float2(h, -h);
            case 2: return make_float2(0.0f, -1.0f);
            default: return make_float2(-h, -h);
        }
    }
    switch (k) {
        case 0: return make_float2(1.0f, 0.0f);
        case 1: return make_float2(c1, -s1);
        case 2: return make_float2(h, -h);
        case 3: return make_float2(s1, -c1);
        case 4: return make_float2(0.0f, -1.0f);
        case 5: return make_float2(-s1, -c1);
        case 6: return make_float2(-h, -h);
        default: return make_float2(-c1, -s1);
    }
}
template <int R> struct Dft {
    __device__ __forceinline__ static void run(float2* v) {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        Dft<R / 2>::run(e);
        Dft<R / 2>::run(o);
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            const float2 t = (k == 0) ? o[k] : cmul(o[k], wconst<R>(k));
            v[k] = cadd(e[k], t);
            v[k + R / 2] = csub(e[k], t);
        }
    }
};

constexpr int kRegPts = 16;

__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }

// One Stockham pass of radix R over the 16 register slots; Ns = product of
// the previous radices.  If LAST, outputs stay in the slots; otherwise they
// are written to LDS at their Stockham destinations.
template <int L, int R, bool LAST>
__device__ __forceinline__ void reg_pass(float2 (&x)[kRegPts], float2* lds, int Ns, const float2* __restrict__ tw,
                                         int t) {
    constexpr int B = L / kRegPts;
    constexpr int NBF = kRegPts / R;
#pragma unroll
    for (int c = 0; c < NBF; ++c) {
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = x[c + NBF * r];
        const int j = t + B * c;
        const int k = j & (Ns - 1);
        if (Ns > 1) {
            const int step = k * (L / (Ns * R));
#pragma unroll
            for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[step * r]);
        }
        Dft<R>::run(v);
        if (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) x[c + NBF * r] = v[r];
        } else {
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[lds_pad(base + Ns * r)] = v[r];
        }
    }
}

template <int L>
__device__ __forceinline__ void reg_exchange(float2 (&x)[kRegPts], float2* lds, int t) {
    constexpr int B = L / kRegPts;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kRegPts; ++s) x[s] = lds[lds_pad(t + B * s)];
    __syncthreads();
}

// Forward DFT of the register-held sequence (slots: element t + B*s in, X[t + B*s] out).
template <int L>
__device__ __forceinline__ void reg_fft(float2 (&x)[kRegPts], float2* lds, const float2* __restrict__ tw, int t) {
    static_assert(L >= 1024 && L <= 16384, "register FFT covers 1024..16384");
    constexpr int log2L = (L == 1024) ? 10 : (L == 2048) ? 11 : (L == 4096) ? 12 : (L == 8192) ? 13 : 14;
    constexpr int rem = 1 << (log2L - 8 - ((log2L >= 12) ? 4 : 0));  // radix of the pass after the 16s
    if constexpr (log2L < 12) {
        // 16 x 16 x rem, rem in {4, 8}
        reg_pass<L, 16, false>(x, lds, 1, tw, t);
        reg_exchange<L>(x, lds, t);
        reg_pass<L, 16, false>(x, lds, 16, tw, t);
        reg_exchange<L>(x, lds, t);
        reg_pass<L, rem, true>(x, lds, 256, tw, t);
    } else if constexpr (log2L == 12) {
        reg_pass<L, 16, false>(x, lds, 1, tw, t);
        reg_exchange<L>(x, lds, t);
        reg_pass<L, 16, false>(x, lds, 16, tw, t);
        reg_exchange<L>(x, lds, t);
        reg_pass<L, 16, true>(x, lds, 256, tw, t);
    } else {
        // 16 x 16 x 16 x rem, rem in {2, 4}
        reg_pass<L, 16, false>(x, lds, 1, tw, t);
        reg_exchange<L>(x, lds, t);
        reg_pass<L, 16, false>(x, lds, 16, tw, t);
        reg_exchange<L>(x, lds, t);
        reg_pass<L, 16, false>(x, lds, 256, tw, t);
        reg_exchange<L>(x, lds, t);
        reg_pass<L, (L >> 12), true>(x, lds, 4096, tw, t);
    }
}

// ---------------------------------------------------------------------------
// The same register transform with every twiddle held in registers.  A
// thread's twiddles depend only on its index, so a kernel that runs many
// transforms loads them once (reg_tw_load) instead of reading the table in
// every pass of every transform.  Identical values and operation order as
// reg_fft, so the results are bitwise the same.  1024 <= L <= 8192.
// ---------------------------------------------------------------------------
template <int L>
struct RegTw {
    static constexpr int log2L = (L == 1024) ? 10 : (L == 2048) ? 11 : (L == 4096) ? 12 : 13;
    static constexpr int R3 = log2L == 10 ? 4 : (log2L == 11 ? 8 : 16);  // radix of the third pass
    static constexpr int N3 = (kRegPts / R3) * (R3 - 1);
    static constexpr int R4 = log2L == 13 ? 2 : 1;                        // fourth pass (L = 8192 only)
    static constexpr int N4 = log2L == 13 ? (kRegPts / 2) : 1;
    float2 p2[15];  // second pass: Ns = 16, radix 16, one butterfly per thread
    float2 p3[N3];  // third pass: Ns = 256
    float2 p4[N4];  // fourth pass: Ns = 4096
};

template <int L>
__device__ __forceinline__ void reg_tw_load(RegTw<L>& w, const float2* __restrict__ tw, int t) {
    static_assert(L >= 1024 && L <= 8192, "register twiddles cover 1024..8192");
    constexpr int B = L / kRegPts;
    {
        const int step = (t & 15) * (L / 256);
#pragma unroll
        for (int r = 1; r < 16; ++r) w.p2[r - 1] = tw[step * r];
    }
    constexpr int R3 = RegTw<L>::R3;
#pragma unroll
    for (int c = 0; c < kRegPts / R3; ++c) {
        const int step = ((t + B * c) & 255) * (L / (256 * R3));
#pragma unroll
        for (int r = 1; r < R3; ++r) w.p3[c * (R3 - 1) + r - 1] = tw[step * r];
    }
    if constexpr (RegTw<L>::R4 == 2) {
#pragma unroll
        for (int c = 0; c < kRegPts / 2; ++c) w.p4[c] = tw[((t + B * c) & 4095) * (L / 8192)];
    }
}

// reg_pass with the pass's twiddles from registers: w[c * (R - 1) + r - 1].
template <int L, int R, bool LAST>
__device__ __forceinline__ void reg_pass_w(float2 (&x)[kRegPts], float2* lds, int Ns, const float2* w, int t) {
    constexpr int B = L / kRegPts;
    constexpr int NBF = kRegPts / R;
#pragma unroll
    for (int c = 0; c < NBF; ++c) {
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = x[c + NBF * r];
        const int j = t + B * c;
        const int k = j & (Ns - 1);
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[c * (R - 1) + r - 1]);
        }
        Dft<R>::run(v);
        if (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) x[c + NBF * r] = v[r];
        } else {
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[lds_pad(base + Ns * r)] = v[r];
        }
    }
}

template <int L>
__device__ __forceinline__ void reg_fft_w(float2 (&x)[kRegPts], float2* lds, const RegTw<L>& w, int t) {
    constexpr int R3 = RegTw<L>::R3;
    reg_pass_w<L, 16, false>(x, lds, 1, w.p2, t);
    reg_exchange<L>(x, lds, t);
    reg_pass_w<L, 16, false>(x, lds, 16, w.p2, t);
    reg_exchange<L>(x, lds, t);
    if constexpr (RegTw<L>::R4 == 2) {
        reg_pass_w<L, R3, false>(x, lds, 256, w.p3, t);
        reg_exchange<L>(x, lds, t);
        reg_pass_w<L, 2, true>(x, lds, 4096, w.p4, t);
    } else {
        reg_pass_w<L, R3, true>(x, lds, 256, w.p3, t);
    }
}

}  // namespace
}  // namespace tp
