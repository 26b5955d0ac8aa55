// Internal declarations shared by the HIP translation units of libtp.so.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <string>

#include "../../include/tp.h"

namespace tp {

// Edge of the square voxel tiles whose origins carry the FP64-derived
// detector coordinate (integer + FP32 fraction).  Shared by the
// backprojector and the forward projector so both take identical
// floor/weight decisions.
constexpr int kGeoTile = 32;
// Detector window staged per (tile, angle): a 32x32 tile spans at most
// 31*sqrt(2) < 44 columns, so floor() takes at most 45 values and the two
// taps at most 46 bins.
constexpr int kWin = 48;
// Threads of the backprojection work-group (4 waves, 8x8 voxels per wave step).
constexpr int kBpThreads = 256;

struct GeoTables {
    const float* cs;   // [na]      FP32 cos(theta)
    const float* sn;   // [na]      FP32 sin(theta)
    const int* xi;     // [nb][na]  floor((bx*32 - N/2) cos)
    const float* xf;   // [nb][na]  fraction of the same, FP32
    const int* yi;     // [nb][na]  floor((by*32 - N/2) sin + center)
    const float* yf;   // [nb][na]
    int na, n, N, nb;
    float center_f;    // FP32 rotation axis (only for candidate search in the forward projector)
    const int* order;  // [n_order] forward-projector grouping: angle indices (-1 = padding), first
                       // n_rows_major entries for angles with |cos| >= |sin|, then the rest
    int n_rows_major;
    int n_order;
};

struct FilterTables {
    const float2* tw;  // [L]  exp(-2 pi i k / L)
    const float* H;    // [L]  H[k] / L (ramp response, inverse-FFT scale folded in)
    int L, log2L;
};

// Raw-count inputs of the normalisation (dev pointers, element strides).
struct RawInput {
    const uint16_t* proj;
    int64_t proj_stride;   // elements between consecutive projections
    const uint16_t* dark;
    const uint16_t* flat;
    int64_t frame_stride;  // elements between consecutive dark/flat frames
    int n_dark, n_flat;
};

// Tables of the Fourier-domain backprojection (one set per plan, filter
// window and truncation radius).  Spectra rows are stored per pair of slices
// and per angle in the order of the angles reduced modulo pi (sorted), each
// row holding the L + 1 samples of signed frequency k = -L/2 .. L/2 at index
// k + L/2 (reversed for angles whose reduction flipped the ray direction).
struct FourierTables {
    const float2* E;        // [L + 1] (pi / na) / L * w_k * H[k] * exp(2 pi i k pos0 / L)
    const float* D;         // [N]     1 / (FT of the 1-D Gaussian at (i - N/2) / M)
    const double* cbd;      // [na]    cos / sin of the sorted reduced angles, FP64
    const double* sbd;
    const float* cb;        // [na]    the same, FP32
    const float* sb;
    const float* beta;      // [na]    sorted reduced angles in [0, pi), FP32
    const int* slot;        // [na]    angle a -> 2 * (sorted position) + (direction reversed)
    const int* tile_order;  // [ntiles] 16x16 work tiles of the gather, nearest the origin first
    int na, n, N, L, log2L, M, log2M, SL;  // SL = L + 1 samples per row
    int nt;                 // gather taps per lane along the ray
    int sw;                 // staged samples per (tile, angle)
    int ntiles;
    int back;               // staged samples before the tile centre's sample: ceil((h + 1) / s) + nt / 2
    float s, inv_s;         // grid points per frequency sample (M / L, a power of two >= 1)
    float msp;              // truncation radius (grid points)
    float kappa;            // log2(e) / (4 tau)
    float ratio2;           // exp2(-2 kappa s^2): ratio of successive tap ratios
};

// Tables of the laminographic backprojection (one set per plan, tilt, row
// centre and slice count): the detector row coordinate of a tile origin,
// split into integer + FP32 fraction per tile edge and angle and per slice.
struct LaminoTables {
    const int* vxi;    // [nb][na] floor((bx*32 - N/2) * (-sin cos_phi))
    const float* vxf;  // [nb][na] fraction of the same
    const int* vyi;    // [nb][na] floor((by*32 - N/2) * (cos cos_phi))
    const float* vyf;
    const int* vzi;    // [Nz]     floor((iz - Nz/2) sin_phi + center_v)
    const float* vzf;
    const float* dvdx; // [na]     -sin(theta) cos(phi), FP32
    const float* dvdy; // [na]      cos(theta) cos(phi)
    float dvdz;        //          sin(phi)
    float dvdcos;      //          cos(phi)
    int Nz;            // slices of the whole volume
    int rows;          // detector rows of the projections (per call)
};

// Tables of the log-polar backprojection (one set per plan, filter window,
// span count, oversampling and origin margin).  Spans p < spans hold n_span
// angle slots each (slot k of span p is angle p * n_span + k, empty past the
// last angle), rotated by beta_p so that slot k sits at phi_k = phi0 + k dtheta.
// Grids: sigma_j = sigma0 + j delta (j < Ns), psi_m = phi0 + m dpsi,
// dpsi = dtheta / M, stored rows m_lo .. m_lo + rows - 1, stored sigma
// window j_lo .. j_lo + nj - 1.
struct LprecTables {
    const float* T0;        // [L]   H[k] / (L B(k~ / 2L)): row spline multiplier, even half-samples
    const float2* T1;       // [L]   T0[k] exp(i pi k~ / L), zero at L/2: odd half-samples
    const double* E;        // [Ns]  exp(sigma_j)
    const float* taper;     // [Ns]  raised-cosine window of the log-radial samples
    const double* A;        // [n_span] a0 cos(phi_k) - pos0
    const double* cd;       // [D]   log(cos((d_lo + d) dpsi)) / (delta Ns)
    const float* preA;      // [NA]  1 / B(nu / NA)
    const float* colscale;  // [Ns]  dtheta / (NA Ns B(eta / Ns))
    const double* cb;       // [spans] cos(beta_p), FP64
    const double* sb;       // [spans] sin(beta_p)
    const float2* twL;      // [L]   exp(-2 pi i k / L)
    const float2* twNs;     // [Ns]
    const float2* twNA;     // [NA]
    const float2* twNAc;    // [NAc]
    const float2* kt;       // [Ns][NA] transformed kernel columns, prefilter and scale folded in (NA >= 8192)
    int na, n, N, L, log2L, spans, n_span, Ns, NA, M, NAc, log2NAc, D, rows, nmb, m_lo, j_lo, nj;
    double a0, sigma0, delta, phi0, dpsi;
};

// ---- allocation-free normalisation ----
// Pixels (n_rows * n_det) whose D and 1/max(F - D, 1) fit the file-scope
// scratch array of the allocation-free normaliser (2 x 32 MiB of FP32).
constexpr int64_t kNoAllocPixels = int64_t(1) << 23;
// Addresses of that array's two halves on the current device, looked up once
// per device with hipGetSymbolAddress.
hipError_t normalize_scratch(float** dmean, float** den);

// ---- launchers (each returns hipError_t of the launch) ----
hipError_t launch_darkflat(const RawInput& in, int n_rows, int n_det, float* dmean, float* den,
                           hipStream_t st);
hipError_t launch_normalize(const RawInput& in, const float* dmean, const float* den, int n_angles,
                            int n_rows, int n_det, tp_dtype out_dtype, void* sino, hipStream_t st);
hipError_t launch_filter(const void* in, tp_dtype in_dt, void* out, tp_dtype out_dt, int64_t n_lines,
                         int n_det, const FilterTables& ft, hipStream_t st);
hipError_t launch_norm_filter(const RawInput& in, const float* dmean, const float* den, int n_angles,
                              int n_rows, int n_det, const FilterTables& ft, tp_dtype out_dt, void* out,
                              hipStream_t st);
// vol: FP32 slices (vol_dt TP_F32), or FP16 slices (TP_F16, FP16 rows only)
hipError_t launch_backproject(const GeoTables& g, const void* filt, tp_dtype dt, int n_rows, float scale,
                              void* vol, tp_dtype vol_dt, int accumulate, int slices_per_block, int angles_per_block,
                              hipStream_t st);
size_t backproject_lds_bytes(tp_dtype dt, int slices_per_block, int angles_per_block);
// Sets the dynamic-LDS limit of one backprojection kernel instance (no launch).
hipError_t prepare_backproject(tp_dtype dt, int slices_per_block, int angles_per_block);
size_t radon_workspace_bytes(const GeoTables& g, int n_rows);
hipError_t launch_radon(const GeoTables& g, const float* vol, int n_rows, float* sino, float* workspace,
                        hipStream_t st);

hipError_t launch_fourier_spectra(const RawInput& in, int rows, const float* dmean, const float* rden,
                                  const float2* tw_L, const FourierTables& t, float2* spec, hipStream_t st);
size_t fourier_grid_tiles(int M);  // work-groups per pair of the gather
hipError_t launch_fourier_grid(const FourierTables& t, const float2* spec, int pairs, float2* grid, hipStream_t st);
hipError_t launch_fourier_rows(const FourierTables& t, const float2* tw_M, const float2* grid, int pairs,
                               float2* cols, hipStream_t st);
hipError_t launch_fourier_cols(const FourierTables& t, const float2* tw_M, const float2* cols, int pairs, int rows,
                               void* vol, bool half_out, hipStream_t st);

int lamino_slices_per_block();

// log-polar backprojection (k_lprec.hip); `pairs` slice pairs per launch
hipError_t launch_lprec_rows(const RawInput& in, int rows, const float* dmean, const float* rden,
                             const LprecTables& t, float2* out, hipStream_t st);
hipError_t launch_lprec_logradial(const LprecTables& t, const float2* rows, int pairs, float2* ghat, hipStream_t st);
hipError_t launch_lprec_conv(const LprecTables& t, const float2* ghat, int pairs, float2* fhat, hipStream_t st);
hipError_t launch_lprec_sigma(const LprecTables& t, const float2* fhat, int pairs, float2* F, hipStream_t st);
hipError_t launch_lprec_interp(const LprecTables& t, const float2* F, int pairs, int rows, float* vol,
                               hipStream_t st);
// Sets the dynamic-LDS limits of the instances a table set uses (no launch).
hipError_t prepare_lprec(const LprecTables& t);
// The transformed kernel table of the long angle transforms: its size (0 when
// the convolution holds the columns in registers) and the launch that fills it.
size_t lprec_ktable_bytes(int Ns, int NA);
hipError_t launch_lprec_ktable(const LprecTables& t, float2* kt, hipStream_t st);

// measurement instruments (k_peak.hip)
hipError_t launch_peak_copy(const void* src, void* dst, int64_t bytes, hipStream_t st);
int64_t peak_valu_flop(int form, int blocks, int iters);
hipError_t launch_peak_valu(int form, float* out, int blocks, int iters, hipStream_t st);
int64_t peak_lds_bytes(int blocks, int iters);
hipError_t launch_peak_lds(uint32_t* out, int blocks, int iters, hipStream_t st);

// ---- backprojection tilings read from the autotuner's JSON table (tp_tune.cpp) ----
// Replaces the process-wide table with the file's entries (path null: clears
// it).  Returns the number of shapes held, or -1 with *err set (the table is
// then unchanged).
int tune_table_load(const char* path, std::string* err);
bool tune_table_lookup(const std::string& device, int storage, int na, int n, int N, int* k, int* a);
bool tune_table_empty();
hipError_t launch_lamino(const GeoTables& g, const LaminoTables& t, const void* filt, tp_dtype dt, int z0, int nz,
                         float scale, float* vol, hipStream_t st);

// ---- detector coordinate decisions shared by backprojection and radon ----
// Offset of voxel (dx, dy) within its 32x32 tile at one angle; bf is the
// FP32 fraction of the tile origin's coordinate.  Explicit FMAs: no
// reassociation, so both kernels round identically.
__device__ __forceinline__ float tile_offset(float dx, float dy, float cs, float sn, float bf) {
    return __builtin_fmaf(dx, cs, __builtin_fmaf(dy, sn, bf));
}
// floor(s) as an integer in one instruction.
__device__ __forceinline__ int coord_floor(float s) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(s));
    return r;
}
// Interpolation weight of the upper tap: s - floor(s), clamped below 1.0 by
// the hardware instruction (only differs for |s| < 2^-24 below an integer).
__device__ __forceinline__ float coord_frac(float s) { return __builtin_amdgcn_fractf(s); }

// ---- storage conversions (round to nearest even) ----
// Negative log of the flat/dark-corrected transmission (paper, Section 2.2):
// -ln(max((P - D) * rden, 1e-6)) with rden = 1 / max(F - D, 1) stored per
// pixel by the dark/flat pass (a multiply per sample instead of a divide).
// The clamp keeps the argument a normal number, so the hardware base-2
// logarithm needs none of the library's range handling: -ln t = -ln 2 * log2 t.
constexpr float kMinTransmission = 1e-6f;
constexpr float kNegLn2 = -0.693147180559945309f;
__device__ __forceinline__ float neglog_counts(float P, float d, float rden) {
    return kNegLn2 * __builtin_amdgcn_logf(fmaxf((P - d) * rden, kMinTransmission));
}

__device__ __forceinline__ float load_as_float(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float load_as_float(const __half* p, int64_t i) { return __half2float(p[i]); }
__device__ __forceinline__ float load_as_float(const uint16_t* p, int64_t i) {  // bfloat16 bits
    return __uint_as_float(static_cast<uint32_t>(p[i]) << 16);
}
__device__ __forceinline__ void store_from_float(float* p, int64_t i, float v) { p[i] = v; }
__device__ __forceinline__ void store_from_float(__half* p, int64_t i, float v) { p[i] = __float2half_rn(v); }
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float v) {
    uint32_t b = __float_as_uint(v);
    if ((b & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((b >> 16) | 0x40u);  // quiet NaN
    b += 0x7fffu + ((b >> 16) & 1u);
    return static_cast<uint16_t>(b >> 16);
}
__device__ __forceinline__ void store_from_float(uint16_t* p, int64_t i, float v) { p[i] = f32_to_bf16_rne(v); }

}  // namespace tp
