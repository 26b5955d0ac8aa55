// Host side of libtp.so: argument validation, FP64-derived tables, plans and
// dispatch to the HIP kernels.  Implements the C ABI declared in include/tp.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "tp_internal.h"

static_assert(TP_NOALLOC_MAX_PIXELS == tp::kNoAllocPixels, "header limit and scratch size disagree");

struct FourierEntry {
    void* block = nullptr;  // one allocation holding the tables
    tp::FourierTables t{};
};

struct LaminoEntry {
    void* block = nullptr;
    tp::LaminoTables t{};
};

struct LprecEntry {
    void* block = nullptr;
    tp::LprecTables t{};
};

struct tp_plan {
    int device = -1;
    int na = 0, n = 0, N = 0, nb = 0;
    double center = 0.0;
    std::vector<double> angles;  // FP64 copy for tables built later
    void* dev_block = nullptr;  // one allocation holding every geometry table
    tp::GeoTables geo{};
    tp::FilterTables filt{};
    // backprojection tuning per storage type (F32, F16, BF16)
    int bp_k[3] = {16, 16, 16};
    int bp_a[3] = {8, 8, 8};
    // Fourier-domain backprojection tables per (filter window, truncation radius)
    mutable std::mutex fr_mu;
    mutable std::map<std::pair<int, int>, FourierEntry> fr;
    // laminographic backprojection tables per (tilt, row centre, slice count)
    mutable std::map<std::tuple<double, double, int>, LaminoEntry> lam;
    // log-polar backprojection tables per (filter window, spans, oversampling, origin margin)
    mutable std::map<std::tuple<int, int, double, double>, LprecEntry> lp;
};

namespace {

constexpr const char* kVersion = "tp 0.1.0 (gfx950)";
constexpr int kMaxPadLen = 16384;
constexpr size_t kMaxLds = 160 * 1024;

thread_local std::string g_err;

tp_status fail(tp_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

tp_status hip_fail(hipError_t e, const char* what) {
    return fail(TP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(int64_t v) {
    int r = 0;
    while ((int64_t{1} << r) < v) ++r;
    return r;
}

int default_pad_len(int n) { return 1 << ilog2(2 * static_cast<int64_t>(n)); }

bool valid_dtype(tp_dtype d) { return d == TP_F32 || d == TP_F16 || d == TP_BF16; }

size_t dtype_size(tp_dtype d) { return d == TP_F32 ? 4 : 2; }

size_t align256(size_t v) { return (v + 255) & ~size_t{255}; }

// ---- filter tables, cached per (device, L, window) ----
struct FilterEntry {
    float2* tw = nullptr;
    float* H = nullptr;
};
std::mutex g_filter_mu;
std::map<std::tuple<int, int, int>, FilterEntry> g_filter_cache;
// plans created and not yet destroyed (tp_shutdown refuses while any exist:
// every plan points at the cached ramp tables of its pad length)
std::atomic<int> g_live_plans{0};

// Exact integral of p(x) cos(pi m x) over [x0, x1] for a polynomial p with
// coefficients c[0..deg] (p = sum c[i] x^i), using the antiderivative
//   F(x) = sum_k (-1)^k [ p^(2k)(x) sin(a x) / a^(2k+1) + p^(2k+1)(x) cos(a x) / a^(2k+2) ],  a = pi m.
// The end points are multiples of 1/2, so sin and cos of a x are taken
// exactly from the quarter-turn count (m x in half-integers).
double poly_cos_integral(std::vector<double> c, int m, double x0, double x1) {
    auto eval = [](const std::vector<double>& q, double x) {
        double v = 0.0;
        for (size_t i = q.size(); i-- > 0;) v = v * x + q[i];
        return v;
    };
    auto deriv = [](const std::vector<double>& q) {
        std::vector<double> d;
        for (size_t i = 1; i < q.size(); ++i) d.push_back(q[i] * static_cast<double>(i));
        return d;
    };
    if (m == 0) {
        double v = 0.0;
        for (size_t i = 0; i < c.size(); ++i)
            v += c[i] * (std::pow(x1, static_cast<double>(i + 1)) - std::pow(x0, static_cast<double>(i + 1))) /
                 static_cast<double>(i + 1);
        return v;
    }
    auto sin_cos = [m](double x, double* sv, double* cv) {
        // a x = (pi/2) * q with q = 2 m x an integer for x in {0, 1/2, 1}
        const int64_t q = static_cast<int64_t>(std::llround(2.0 * m * x));
        static const double S[4] = {0.0, 1.0, 0.0, -1.0}, C[4] = {1.0, 0.0, -1.0, 0.0};
        *sv = S[q & 3];
        *cv = C[q & 3];
    };
    const double a = M_PI * m;
    auto F = [&](double x) {
        double sv, cv;
        sin_cos(x, &sv, &cv);
        double total = 0.0, apow = a, sign = 1.0;
        std::vector<double> q = c;
        while (!q.empty()) {
            total += sign * eval(q, x) * sv / apow;
            q = deriv(q);
            if (q.empty()) break;
            total += sign * eval(q, x) * cv / (apow * a);
            q = deriv(q);
            apow *= a * a;
            sign = -sign;
        }
        return total;
    };
    return F(x1) - F(x0);
}

// Taps h[m], m = 0..L/2, of the windowed band-limited ramp
//   h[m] = integral over |w| <= 1/2 of |w| W(2|w|) exp(2 pi i w m) dw   (h is even),
// with the window W on x = 2|w| in [0, 1]:
//   ramp:   W = 1                      -> h[0] = 1/4, h[odd m] = -1/(pi^2 m^2), h[even m] = 0;
//   Shepp-Logan: W = sinc(x/2)         -> h[m] = 2 / (pi^2 (1 - 4 m^2));
//   Parzen: W = 1 - 6x^2 + 6x^3 (x <= 1/2), 2 (1 - x)^3 (x > 1/2)
//           -> h[m] = (1/2) integral_0^1 x W(x) cos(pi m x) dx, exact per polynomial piece.
void window_taps_fp64(int L, tp_filter_kind kind, std::vector<double>& h) {
    h.assign(L / 2 + 1, 0.0);
    const double inv_pi2 = 1.0 / (M_PI * M_PI);
    for (int m = 0; m <= L / 2; ++m) {
        const double dm = static_cast<double>(m);
        if (kind == TP_RAMP) {
            h[m] = m == 0 ? 0.25 : ((m & 1) ? -inv_pi2 / (dm * dm) : 0.0);
        } else if (kind == TP_SHEPP) {
            h[m] = 2.0 * inv_pi2 / (1.0 - 4.0 * dm * dm);
        } else {
            // x W(x) on each piece, as polynomial coefficients in x
            h[m] = 0.5 * (poly_cos_integral({0.0, 1.0, 0.0, -6.0, 6.0}, m, 0.0, 0.5) +
                          poly_cos_integral({0.0, 2.0, -6.0, 6.0, -2.0}, m, 0.5, 1.0));
        }
    }
}

// H[k] = sum_{m=-L/2}^{L/2-1} h[m] exp(-2 pi i k m / L), real and even: FP64
// direct sum over the non-zero lags with an exact integer phase index.
void filter_response_fp64(int L, tp_filter_kind kind, std::vector<double>& H) {
    std::vector<double> h;
    window_taps_fp64(L, kind, h);
    std::vector<double> c(L);
    for (int k = 0; k < L; ++k) c[k] = std::cos(2.0 * M_PI * static_cast<double>(k) / L);
    H.assign(L, h[0]);
    for (int m = -L / 2; m < L / 2; ++m) {
        const double hm = h[m < 0 ? -m : m];
        if (m == 0 || hm == 0.0) continue;
        const int64_t mm = ((m % L) + L) % L;
        for (int k = 0; k < L; ++k) H[k] += hm * c[(static_cast<int64_t>(k) * mm) % L];
    }
}

bool valid_kind(tp_filter_kind k) { return k == TP_RAMP || k == TP_SHEPP || k == TP_PARZEN; }

tp_status filter_tables(int L, tp_filter_kind kind, tp::FilterTables* out, hipStream_t st_for_capture_check) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_filter_mu);
    auto key = std::make_tuple(dev, L, static_cast<int>(kind));
    auto it = g_filter_cache.find(key);
    if (it == g_filter_cache.end()) {
        if (st_for_capture_check != nullptr) {
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(st_for_capture_check, &cs) == hipSuccess &&
                cs != hipStreamCaptureStatusNone)
                return fail(TP_EUNSUPPORTED,
                            "filter tables for pad length %d, window %d not built; call tp_filter_prepare before "
                            "capture", L, static_cast<int>(kind));
        }
        std::vector<double> H;
        filter_response_fp64(L, kind, H);
        std::vector<float2> tw(L);
        std::vector<float> hf(L);
        for (int k = 0; k < L; ++k) {
            const double ang = -2.0 * M_PI * static_cast<double>(k) / L;
            tw[k] = make_float2(static_cast<float>(std::cos(ang)), static_cast<float>(std::sin(ang)));
            hf[k] = static_cast<float>(H[k] / L);
        }
        FilterEntry fe;
        e = hipMalloc(&fe.tw, sizeof(float2) * L);
        if (e != hipSuccess) return fail(TP_ENOMEM, "hipMalloc(filter twiddles): %s", hipGetErrorString(e));
        e = hipMalloc(&fe.H, sizeof(float) * L);
        if (e != hipSuccess) {
            (void)hipFree(fe.tw);
            return fail(TP_ENOMEM, "hipMalloc(filter response): %s", hipGetErrorString(e));
        }
        e = hipMemcpy(fe.tw, tw.data(), sizeof(float2) * L, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(fe.H, hf.data(), sizeof(float) * L, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(fe.tw);
            (void)hipFree(fe.H);
            return hip_fail(e, "hipMemcpy(filter tables)");
        }
        it = g_filter_cache.emplace(key, fe).first;
    }
    out->tw = it->second.tw;
    out->H = it->second.H;
    out->L = L;
    out->log2L = ilog2(L);
    return TP_OK;
}

tp_status check_raw(const uint16_t* proj, const uint16_t* dark, int32_t n_dark, const uint16_t* flat,
                    int32_t n_flat, int64_t* proj_stride, int64_t* frame_stride, int32_t n_angles,
                    int32_t n_rows, int32_t n_det) {
    if (!proj || !dark || !flat) return fail(TP_EINVAL, "null raw-data pointer");
    if (n_angles <= 0 || n_rows <= 0 || n_det <= 0)
        return fail(TP_EINVAL, "sizes must be positive (n_angles=%d n_rows=%d n_det=%d)", n_angles, n_rows, n_det);
    if (n_rows > 65535) return fail(TP_EINVAL, "n_rows=%d exceeds 65535 per call", n_rows);
    if (n_dark < 1 || n_dark > 256 || n_flat < 1 || n_flat > 256)
        return fail(TP_EINVAL, "n_dark=%d n_flat=%d must be in [1, 256]", n_dark, n_flat);
    const int64_t slab = static_cast<int64_t>(n_rows) * n_det;
    if (*proj_stride == 0) *proj_stride = slab;
    if (*frame_stride == 0) *frame_stride = slab;
    if (*proj_stride < slab) return fail(TP_EINVAL, "proj_stride %lld < n_rows*n_det", (long long)*proj_stride);
    if (*frame_stride < slab)
        return fail(TP_EINVAL, "frame_stride %lld < n_rows*n_det", (long long)*frame_stride);
    return TP_OK;
}

// ---- Fourier-domain backprojection: sizes, tables, workspace layout ----
constexpr int kFourierDefaultHalfWidth = 6;
constexpr int kFourierMaxSide = 16384;
// Tile half-diagonal (7.5 sqrt(2)) of the gather's 16x16 tiles, as in the kernel.
constexpr double kFrHalfDiag = 10.606601717798213;

struct FrDims {
    int L, M, SL, ng;  // pad length, grid side, samples per spectrum row, 16-row column groups
    size_t spec_pair, cols_pair, grid_pair;
};

FrDims fr_dims(const tp_plan* plan) {
    FrDims d{};
    d.L = plan->filt.L;
    d.M = std::max({d.L, 1 << ilog2(2 * static_cast<int64_t>(plan->N)), 64});
    d.SL = d.L + 1;
    d.ng = (plan->N + 15) / 16;
    d.spec_pair = static_cast<size_t>(plan->na) * d.SL * sizeof(float2);
    d.cols_pair = static_cast<size_t>(d.ng) * 16 * d.M * sizeof(float2);
    d.grid_pair = static_cast<size_t>(d.M) * d.M * sizeof(float2);
    return d;
}

// Workspace: dark/flat tables of every row, then (per pass of P pairs) a
// region holding the spectra and later the column-group intermediate, then
// the Cartesian grid.
size_t fr_workspace(const tp_plan* plan, int32_t n_rows, int64_t P) {
    const FrDims d = fr_dims(plan);
    return tp_normalize_workspace_bytes(n_rows, plan->n) +
           align256(static_cast<size_t>(P) * std::max(d.spec_pair, d.cols_pair)) +
           align256(static_cast<size_t>(P) * d.grid_pair);
}

tp_status fourier_tables(const tp_plan* plan, tp_filter_kind kind, int msp, tp::FourierTables* out,
                         hipStream_t st_for_capture_check) {
    std::lock_guard<std::mutex> lk(plan->fr_mu);
    const auto key = std::make_pair(static_cast<int>(kind), msp);
    auto it = plan->fr.find(key);
    if (it != plan->fr.end()) {
        *out = it->second.t;
        return TP_OK;
    }
    if (st_for_capture_check != nullptr) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st_for_capture_check, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
            return fail(TP_EUNSUPPORTED,
                        "Fourier tables for window %d, half width %d not built; call tp_fourier_prepare before "
                        "capture", static_cast<int>(kind), msp);
    }
    const FrDims d = fr_dims(plan);
    const int na = plan->na, n = plan->n, N = plan->N, L = d.L, M = d.M, h = L / 2;
    const double s = static_cast<double>(M) / L;
    const double tau = msp / (2.0 * std::sqrt(2.0) * M_PI);
    const double kappa = 1.0 / (4.0 * tau * std::log(2.0));
    const int nt = 2 * static_cast<int>(std::ceil(msp / s));
    const int back = static_cast<int>(std::ceil((kFrHalfDiag + 1.0) / s)) + nt / 2;
    const int sw = static_cast<int>(std::ceil(2.0 * (kFrHalfDiag + 1.0) / s)) + nt + 4;
    if (s > 8.0 || sw > 64)
        return fail(TP_EUNSUPPORTED, "Fourier grid of %d points per side for pad length %d (more than 8 grid "
                    "points per frequency sample)", M, L);
    const double pos0 = plan->center + (L - n) / 2;
    // E[k + L/2] = (pi / na) / L * w_k * H[k] * exp(2 pi i k pos0 / L)
    std::vector<double> H;
    filter_response_fp64(L, kind, H);
    std::vector<float2> E(static_cast<size_t>(L) + 1);
    for (int k = -h; k <= h; ++k) {
        const double wk = (k == -h || k == h) ? 0.5 : 1.0;
        const double amp = (M_PI / na) / L * wk * H[static_cast<size_t>((k + L) % L)];
        double fr = static_cast<double>(k) * pos0 / L;
        fr -= std::floor(fr);
        const double ph = 2.0 * M_PI * fr;
        E[static_cast<size_t>(k + h)] =
            make_float2(static_cast<float>(amp * std::cos(ph)), static_cast<float>(amp * std::sin(ph)));
    }
    // D[i] = 1 / phi_hat((i - N/2) / M), phi_hat(v) = sqrt(4 pi tau) exp(-4 pi^2 tau v^2)
    std::vector<float> D(N);
    for (int i = 0; i < N; ++i) {
        const double v = static_cast<double>(i - N / 2) / M;
        D[i] = static_cast<float>(std::exp(4.0 * M_PI * M_PI * tau * v * v) / std::sqrt(4.0 * M_PI * tau));
    }
    // angles reduced modulo pi into [0, pi), sorted; reversed when the reduction was by an odd multiple of pi
    std::vector<double> beta(na);
    std::vector<int> rev(na), idx(na);
    for (int a = 0; a < na; ++a) {
        double t2 = std::fmod(plan->angles[a], 2.0 * M_PI);
        if (t2 < 0) t2 += 2.0 * M_PI;
        if (t2 >= 2.0 * M_PI) t2 = 0.0;
        rev[a] = t2 >= M_PI;
        beta[a] = rev[a] ? t2 - M_PI : t2;
        if (beta[a] >= M_PI) beta[a] = 0.0;
        idx[a] = a;
    }
    std::sort(idx.begin(), idx.end(), [&](int p, int q) { return beta[p] < beta[q] || (beta[p] == beta[q] && p < q); });
    std::vector<double> cbd(na), sbd(na);
    std::vector<float> cb(na), sb(na), bf(na);
    std::vector<int> slot(na);
    for (int j = 0; j < na; ++j) {
        const int a = idx[j];
        cbd[j] = std::cos(beta[a]);
        sbd[j] = std::sin(beta[a]);
        cb[j] = static_cast<float>(cbd[j]);
        sb[j] = static_cast<float>(sbd[j]);
        bf[j] = static_cast<float>(beta[a]);
        slot[a] = 2 * j + rev[a];
    }
    // The gather's 16x16 work tiles: the tile rows with uy >= 0 (each also
    // produces the mirror points -u) and tile row 0 (for the grid row
    // uy = -M/2), nearest the origin first: their angle lists are the longest.
    const int tps = M / 16;
    std::vector<int> tiles;
    tiles.reserve(tp::fourier_grid_tiles(M));
    for (int ty = 0; ty < tps; ++ty) {
        if (ty != 0 && ty < tps / 2) continue;
        for (int tx = 0; tx < tps; ++tx) tiles.push_back(ty * tps + tx);
    }
    const int ntiles = static_cast<int>(tiles.size());
    auto dist = [&](int i) {
        const double cx = (i % tps) * 16 - M / 2 + 7.5, cy = (i / tps) * 16 - M / 2 + 7.5;
        return cx * cx + cy * cy;
    };
    std::sort(tiles.begin(), tiles.end(),
              [&](int p, int q) { return dist(p) < dist(q) || (dist(p) == dist(q) && p < q); });

    const size_t sE = align256(sizeof(float2) * E.size()), sD = align256(sizeof(float) * N);
    const size_t sd = align256(sizeof(double) * na), sf = align256(sizeof(float) * na);
    const size_t sT = align256(sizeof(int) * ntiles);
    const size_t total = sE + sD + 2 * sd + 4 * sf + sT;
    FourierEntry fe;
    hipError_t e = hipMalloc(&fe.block, total);
    if (e != hipSuccess) return fail(TP_ENOMEM, "hipMalloc(Fourier tables, %zu bytes): %s", total, hipGetErrorString(e));
    char* b = static_cast<char*>(fe.block);
    char* dE = b;
    char* dD = dE + sE;
    char* dcbd = dD + sD;
    char* dsbd = dcbd + sd;
    char* dcb = dsbd + sd;
    char* dsb = dcb + sf;
    char* dbeta = dsb + sf;
    char* dslot = dbeta + sf;
    char* dtile = dslot + sf;
    e = hipMemcpy(dE, E.data(), sizeof(float2) * E.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dD, D.data(), sizeof(float) * N, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dcbd, cbd.data(), sizeof(double) * na, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dsbd, sbd.data(), sizeof(double) * na, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dcb, cb.data(), sizeof(float) * na, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dsb, sb.data(), sizeof(float) * na, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dbeta, bf.data(), sizeof(float) * na, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dslot, slot.data(), sizeof(int) * na, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dtile, tiles.data(), sizeof(int) * ntiles, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(fe.block);
        return hip_fail(e, "hipMemcpy(Fourier tables)");
    }
    tp::FourierTables& t = fe.t;
    t.E = reinterpret_cast<const float2*>(dE);
    t.D = reinterpret_cast<const float*>(dD);
    t.cbd = reinterpret_cast<const double*>(dcbd);
    t.sbd = reinterpret_cast<const double*>(dsbd);
    t.cb = reinterpret_cast<const float*>(dcb);
    t.sb = reinterpret_cast<const float*>(dsb);
    t.beta = reinterpret_cast<const float*>(dbeta);
    t.slot = reinterpret_cast<const int*>(dslot);
    t.tile_order = reinterpret_cast<const int*>(dtile);
    t.na = na;
    t.n = n;
    t.N = N;
    t.L = L;
    t.log2L = ilog2(L);
    t.M = M;
    t.log2M = ilog2(M);
    t.SL = d.SL;
    t.nt = nt;
    t.sw = sw;
    t.ntiles = ntiles;
    t.back = back;
    t.s = static_cast<float>(s);
    t.inv_s = static_cast<float>(1.0 / s);
    t.msp = static_cast<float>(msp);
    t.kappa = static_cast<float>(kappa);
    t.ratio2 = static_cast<float>(std::exp2(-2.0 * kappa * s * s));
    plan->fr.emplace(key, fe);
    *out = t;
    return TP_OK;
}

tp_status lamino_tables(const tp_plan* plan, double tilt, double center_v, int Nz, tp::LaminoTables* out,
                        hipStream_t st_for_capture_check) {
    std::lock_guard<std::mutex> lk(plan->fr_mu);
    const auto key = std::make_tuple(tilt, center_v, Nz);
    auto it = plan->lam.find(key);
    if (it != plan->lam.end()) {
        *out = it->second.t;
        return TP_OK;
    }
    if (st_for_capture_check != nullptr) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st_for_capture_check, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
            return fail(TP_EUNSUPPORTED, "laminography tables not built; call tp_lamino_prepare before capture");
    }
    const int na = plan->na, nb = plan->nb, N = plan->N;
    const double cphi = std::cos(tilt), sphi = std::sin(tilt);
    std::vector<int> vxi(static_cast<size_t>(nb) * na), vyi(static_cast<size_t>(nb) * na), vzi(Nz);
    std::vector<float> vxf(vxi.size()), vyf(vyi.size()), vzf(Nz), dvdx(na), dvdy(na);
    for (int a = 0; a < na; ++a) {
        const double c = std::cos(plan->angles[a]), sn = std::sin(plan->angles[a]);
        dvdx[a] = static_cast<float>(-sn * cphi);
        dvdy[a] = static_cast<float>(c * cphi);
        for (int b = 0; b < nb; ++b) {
            const double o = static_cast<double>(b * tp::kGeoTile - N / 2);
            const double X = o * (-sn * cphi), Y = o * (c * cphi);
            const double fx = std::floor(X), fy = std::floor(Y);
            const size_t i = static_cast<size_t>(b) * na + a;
            vxi[i] = static_cast<int>(fx);
            vxf[i] = static_cast<float>(X - fx);
            vyi[i] = static_cast<int>(fy);
            vyf[i] = static_cast<float>(Y - fy);
        }
    }
    for (int z = 0; z < Nz; ++z) {
        const double Z = static_cast<double>(z - Nz / 2) * sphi + center_v;
        const double fz = std::floor(Z);
        vzi[z] = static_cast<int>(fz);
        vzf[z] = static_cast<float>(Z - fz);
    }
    const size_t sT = align256(sizeof(int) * vxi.size()), sZ = align256(sizeof(int) * Nz), sA = align256(sizeof(float) * na);
    const size_t total = 4 * sT + 2 * sZ + 2 * sA;
    LaminoEntry le;
    hipError_t e = hipMalloc(&le.block, total);
    if (e != hipSuccess) return fail(TP_ENOMEM, "hipMalloc(laminography tables, %zu bytes): %s", total, hipGetErrorString(e));
    char* p = static_cast<char*>(le.block);
    char* d_vxi = p;
    char* d_vxf = d_vxi + sT;
    char* d_vyi = d_vxf + sT;
    char* d_vyf = d_vyi + sT;
    char* d_vzi = d_vyf + sT;
    char* d_vzf = d_vzi + sZ;
    char* d_dx = d_vzf + sZ;
    char* d_dy = d_dx + sA;
    const size_t tb = sizeof(int) * vxi.size();
    e = hipMemcpy(d_vxi, vxi.data(), tb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_vxf, vxf.data(), tb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_vyi, vyi.data(), tb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_vyf, vyf.data(), tb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_vzi, vzi.data(), sizeof(int) * Nz, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_vzf, vzf.data(), sizeof(float) * Nz, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_dx, dvdx.data(), sizeof(float) * na, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_dy, dvdy.data(), sizeof(float) * na, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(le.block);
        return hip_fail(e, "hipMemcpy(laminography tables)");
    }
    tp::LaminoTables& t = le.t;
    t.vxi = reinterpret_cast<const int*>(d_vxi);
    t.vxf = reinterpret_cast<const float*>(d_vxf);
    t.vyi = reinterpret_cast<const int*>(d_vyi);
    t.vyf = reinterpret_cast<const float*>(d_vyf);
    t.vzi = reinterpret_cast<const int*>(d_vzi);
    t.vzf = reinterpret_cast<const float*>(d_vzf);
    t.dvdx = reinterpret_cast<const float*>(d_dx);
    t.dvdy = reinterpret_cast<const float*>(d_dy);
    t.dvdz = static_cast<float>(sphi);
    t.dvdcos = static_cast<float>(cphi);
    t.Nz = Nz;
    t.rows = 0;
    plan->lam.emplace(key, le);
    *out = t;
    return TP_OK;
}

tp_status lamino_check(const tp_plan* plan, double tilt, double center_v, int32_t n_slices) {
    if (!plan) return fail(TP_EINVAL, "plan is null");
    if (!std::isfinite(tilt) || tilt <= 0.0 || tilt >= M_PI)
        return fail(TP_EINVAL, "tilt %g must lie in (0, pi)", tilt);
    if (!std::isfinite(center_v) || std::fabs(center_v) > 1e6) return fail(TP_EINVAL, "center_v %g out of range", center_v);
    if (n_slices <= 0 || n_slices > 1000000) return fail(TP_EINVAL, "n_slices=%d out of range", n_slices);
    return TP_OK;
}

tp_status fourier_half_width(int32_t half_width, int* msp) {
    if (half_width == 0) {
        *msp = kFourierDefaultHalfWidth;
        return TP_OK;
    }
    if (half_width < 3 || half_width > 8) return fail(TP_EINVAL, "half_width=%d not in 3..8 (or 0)", half_width);
    *msp = half_width;
    return TP_OK;
}

// ---- log-polar backprojection: grid sizing, tables, workspace ----
constexpr int kLpSigmaMargin = 12;   // sigma points of taper beyond the data range
constexpr int kLpAngleMargin = 16;   // psi rows beyond the image sector
constexpr int kLpWindowMargin = 4;   // sigma points kept beyond the image's rho range
constexpr int kLpMinFft = 1024;
constexpr int kLpMaxFft = 16384;
constexpr int kLpMaxSpans = 4;       // the evaluation kernel holds every span's weights in registers
constexpr int kLpDefaultSpans = 3;
constexpr double kLpDefaultOs = 1.0;
constexpr double kLpDefaultEps = 1.0;

int pow2_at_least(int64_t v) {
    int r = 0;
    while ((int64_t{1} << r) < v) ++r;
    return 1 << r;
}

// Sizing rule of the log-polar grids (see tp.h, tp_lprec_grid_query).
tp_status lp_grid(int na, int N, int spans, double os, double eps, tp_lprec_grid* g) {
    if (spans == 0) spans = kLpDefaultSpans;
    if (os == 0.0) os = kLpDefaultOs;
    if (eps == 0.0) eps = kLpDefaultEps;
    if (spans < 2 || spans > kLpMaxSpans) return fail(TP_EINVAL, "spans=%d not in 2..%d", spans, kLpMaxSpans);
    if (!(os >= 0.25 && os <= 8.0)) return fail(TP_EINVAL, "oversampling %g not in [0.25, 8]", os);
    if (!(eps >= 0.05 && eps <= 4.0)) return fail(TP_EINVAL, "origin margin %g not in [0.05, 4]", eps);
    if (na < 2 * spans) return fail(TP_EUNSUPPORTED, "%d angles for %d spans", na, spans);
    if (N < 2) return fail(TP_EUNSUPPORTED, "slice side %d", N);
    tp_lprec_grid r{};
    r.spans = spans;
    r.os = os;
    r.eps = eps;
    r.dtheta = M_PI / na;
    const int half = N / 2;
    r.R = std::sqrt(2.0) * half + 2.0;
    r.n_span = (na + spans - 1) / spans;
    const double phi_max = 0.5 * (r.n_span - 1) * r.dtheta;
    r.phi0 = -phi_max;
    r.a0 = (1.0 + eps) * r.R / std::cos(phi_max);
    r.s_min = r.a0 * std::cos(phi_max) - r.R;
    r.s_max = r.a0 + r.R;
    const double lo = std::log(r.s_min), hi = std::log(r.s_max);
    const int64_t n_need = static_cast<int64_t>(std::ceil((hi - lo) * os * r.s_max)) + 2 * kLpSigmaMargin + 1;
    r.Ns = std::max(kLpMinFft, pow2_at_least(n_need));
    if (r.Ns > kLpMaxFft)
        return fail(TP_EUNSUPPORTED, "log-polar grid needs %lld sigma points (> %d); lower the oversampling",
                    static_cast<long long>(n_need), kLpMaxFft);
    r.delta = (hi - lo) / (r.Ns - 1 - 2 * kLpSigmaMargin);
    r.sigma0 = lo - kLpSigmaMargin * r.delta;
    r.M = pow2_at_least(static_cast<int64_t>(std::ceil(os * r.dtheta * r.s_max)));
    r.dpsi = r.dtheta / r.M;
    const double psi_max = std::asin(r.R / r.a0);
    r.m_lo = static_cast<int32_t>(std::floor((-psi_max - r.phi0) / r.dpsi)) - kLpAngleMargin;
    const int m_hi = static_cast<int32_t>(std::ceil((psi_max - r.phi0) / r.dpsi)) + kLpAngleMargin;
    r.rows = m_hi - r.m_lo + 1;
    r.D = r.rows + r.M * (r.n_span - 1);
    r.NA = std::max(kLpMinFft, pow2_at_least(r.D));
    if (r.NA > kLpMaxFft)
        return fail(TP_EUNSUPPORTED, "log-polar grid needs %d angle points (> %d); lower the oversampling", r.D,
                    kLpMaxFft);
    r.d_lo = r.m_lo - r.M * (r.n_span - 1);
    if (!(std::fabs(r.d_lo * r.dpsi) < M_PI / 2) || !(std::fabs((r.d_lo + r.D - 1) * r.dpsi) < M_PI / 2))
        return fail(TP_EUNSUPPORTED, "angular margin reaches 90 degrees; increase the origin margin");
    r.j_lo = static_cast<int32_t>(std::floor((std::log(r.a0 - r.R) - r.sigma0) / r.delta)) - kLpWindowMargin;
    const int j_hi = static_cast<int32_t>(std::ceil((std::log(r.a0 + r.R) - r.sigma0) / r.delta)) + kLpWindowMargin;
    r.nj = j_hi - r.j_lo + 1;
    *g = r;
    return TP_OK;
}

double bspline5_hat(double nu) {  // sampled transform of the centred quintic B-spline, nu in cycles per sample
    const double w = 2.0 * M_PI * nu;
    return (66.0 + 52.0 * std::cos(w) + 2.0 * std::cos(2.0 * w)) / 120.0;
}

bool lp_angles_uniform(const tp_plan* plan) {
    const double d = M_PI / plan->na;
    for (int a = 0; a < plan->na; ++a)
        if (std::fabs(plan->angles[a] - (plan->angles[0] + a * d)) > 1e-9) return false;
    return true;
}

struct LpSizes {
    size_t rows, ghat, fhat, F;  // bytes per pair of slices
};

LpSizes lp_sizes(const tp_plan* plan, const tp_lprec_grid& g) {
    const int L = plan->filt.L;
    const size_t nmb = static_cast<size_t>((g.rows + 15) / 16);
    LpSizes z;
    z.rows = sizeof(float2) * static_cast<size_t>(plan->na) * 2 * L;
    z.ghat = sizeof(float2) * static_cast<size_t>(g.spans) * g.Ns * g.n_span;
    z.fhat = sizeof(float2) * static_cast<size_t>(g.spans) * nmb * g.Ns * 16;
    z.F = sizeof(float2) * static_cast<size_t>(g.spans) * g.rows * g.nj;
    return z;
}

size_t lp_workspace(const tp_plan* plan, const tp_lprec_grid& g, int32_t n_rows, int64_t P) {
    const LpSizes z = lp_sizes(plan, g);
    return tp_normalize_workspace_bytes(n_rows, plan->n) + align256(static_cast<size_t>(P) * std::max(z.rows, z.fhat)) +
           align256(static_cast<size_t>(P) * std::max(z.ghat, z.F));
}

tp_status lprec_tables(const tp_plan* plan, tp_filter_kind kind, const tp_lprec_grid& g, tp::LprecTables* out,
                       hipStream_t st_for_capture_check) {
    std::lock_guard<std::mutex> lk(plan->fr_mu);
    const auto key = std::make_tuple(static_cast<int>(kind), g.spans, g.os, g.eps);
    auto it = plan->lp.find(key);
    if (it != plan->lp.end()) {
        *out = it->second.t;
        return TP_OK;
    }
    if (st_for_capture_check != nullptr) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st_for_capture_check, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
            return fail(TP_EUNSUPPORTED, "log-polar tables not built; call tp_lprec_prepare before capture");
    }
    const int na = plan->na, n = plan->n, L = plan->filt.L, Ns = g.Ns, NA = g.NA, NAc = g.NA / g.M;
    const double pos0 = plan->center + (L - n) / 2;
    std::vector<double> H;
    filter_response_fp64(L, kind, H);
    std::vector<float> T0(L), taper(Ns), preA(NA), colscale(Ns);
    std::vector<float2> T1(L);
    for (int k = 0; k < L; ++k) {
        const int ks = k < L / 2 ? k : k - L;
        const double t0 = H[k] / (L * bspline5_hat(static_cast<double>(ks) / (2.0 * L)));
        T0[k] = static_cast<float>(t0);
        const double ph = M_PI * ks / L;
        T1[k] = k == L / 2 ? make_float2(0.0f, 0.0f)
                           : make_float2(static_cast<float>(t0 * std::cos(ph)), static_cast<float>(t0 * std::sin(ph)));
    }
    std::vector<double> E(Ns), A(g.n_span), cd(g.D), cbp(g.spans), sbp(g.spans);
    const double ramp = kLpSigmaMargin - 2;
    for (int j = 0; j < Ns; ++j) {
        E[j] = std::exp(g.sigma0 + g.delta * j);
        const double tl = std::min(std::max((j - 2.0) / ramp, 0.0), 1.0);
        const double th = std::min(std::max((Ns - 3.0 - j) / ramp, 0.0), 1.0);
        taper[j] = static_cast<float>(std::min(0.5 - 0.5 * std::cos(M_PI * tl), 0.5 - 0.5 * std::cos(M_PI * th)));
        colscale[j] = static_cast<float>(g.dtheta / (static_cast<double>(NA) * Ns * bspline5_hat(static_cast<double>(j) / Ns)));
    }
    for (int k = 0; k < g.n_span; ++k) A[k] = g.a0 * std::cos((k - 0.5 * (g.n_span - 1)) * g.dtheta) - pos0;
    for (int d = 0; d < g.D; ++d) cd[d] = std::log(std::cos((g.d_lo + d) * g.dpsi)) / (g.delta * Ns);
    for (int v = 0; v < NA; ++v) preA[v] = static_cast<float>(1.0 / bspline5_hat(static_cast<double>(v) / NA));
    for (int p = 0; p < g.spans; ++p) {
        const double beta = plan->angles[0] + (p * g.n_span + 0.5 * (g.n_span - 1)) * g.dtheta;
        cbp[p] = std::cos(beta);
        sbp[p] = std::sin(beta);
    }
    auto twiddles = [](int len) {
        std::vector<float2> tw(len);
        for (int k = 0; k < len; ++k) {
            const double ang = -2.0 * M_PI * static_cast<double>(k) / len;
            tw[k] = make_float2(static_cast<float>(std::cos(ang)), static_cast<float>(std::sin(ang)));
        }
        return tw;
    };
    const std::vector<float2> twL = twiddles(L), twNs = twiddles(Ns), twNA = twiddles(NA), twNAc = twiddles(NAc);
    struct Part {
        const void* src;
        size_t bytes;
        char* dst;
    };
    std::vector<Part> parts = {{T0.data(), sizeof(float) * L, nullptr},        {T1.data(), sizeof(float2) * L, nullptr},
                               {E.data(), sizeof(double) * Ns, nullptr},        {taper.data(), sizeof(float) * Ns, nullptr},
                               {A.data(), sizeof(double) * g.n_span, nullptr},  {cd.data(), sizeof(double) * g.D, nullptr},
                               {preA.data(), sizeof(float) * NA, nullptr},      {colscale.data(), sizeof(float) * Ns, nullptr},
                               {cbp.data(), sizeof(double) * g.spans, nullptr}, {sbp.data(), sizeof(double) * g.spans, nullptr},
                               {twL.data(), sizeof(float2) * L, nullptr},       {twNs.data(), sizeof(float2) * Ns, nullptr},
                               {twNA.data(), sizeof(float2) * NA, nullptr},     {twNAc.data(), sizeof(float2) * NAc, nullptr}};
    size_t total = 0;
    for (const Part& q : parts) total += align256(q.bytes);
    const size_t kt_bytes = tp::lprec_ktable_bytes(Ns, NA);
    total += align256(kt_bytes);
    LprecEntry le;
    hipError_t e = hipMalloc(&le.block, total);
    if (e != hipSuccess) return fail(TP_ENOMEM, "hipMalloc(log-polar tables, %zu bytes): %s", total, hipGetErrorString(e));
    char* b = static_cast<char*>(le.block);
    for (Part& q : parts) {
        q.dst = b;
        b += align256(q.bytes);
        if (e == hipSuccess) e = hipMemcpy(q.dst, q.src, q.bytes, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        (void)hipFree(le.block);
        return hip_fail(e, "hipMemcpy(log-polar tables)");
    }
    tp::LprecTables& t = le.t;
    t.T0 = reinterpret_cast<const float*>(parts[0].dst);
    t.T1 = reinterpret_cast<const float2*>(parts[1].dst);
    t.E = reinterpret_cast<const double*>(parts[2].dst);
    t.taper = reinterpret_cast<const float*>(parts[3].dst);
    t.A = reinterpret_cast<const double*>(parts[4].dst);
    t.cd = reinterpret_cast<const double*>(parts[5].dst);
    t.preA = reinterpret_cast<const float*>(parts[6].dst);
    t.colscale = reinterpret_cast<const float*>(parts[7].dst);
    t.cb = reinterpret_cast<const double*>(parts[8].dst);
    t.sb = reinterpret_cast<const double*>(parts[9].dst);
    t.twL = reinterpret_cast<const float2*>(parts[10].dst);
    t.twNs = reinterpret_cast<const float2*>(parts[11].dst);
    t.twNA = reinterpret_cast<const float2*>(parts[12].dst);
    t.twNAc = reinterpret_cast<const float2*>(parts[13].dst);
    t.kt = kt_bytes ? reinterpret_cast<const float2*>(b) : nullptr;
    t.na = na;
    t.n = n;
    t.N = plan->N;
    t.L = L;
    t.log2L = ilog2(L);
    t.spans = g.spans;
    t.n_span = g.n_span;
    t.Ns = Ns;
    t.NA = NA;
    t.M = g.M;
    t.NAc = NAc;
    t.log2NAc = ilog2(NAc);
    t.D = g.D;
    t.rows = g.rows;
    t.nmb = (g.rows + 15) / 16;
    t.m_lo = g.m_lo;
    t.j_lo = g.j_lo;
    t.nj = g.nj;
    t.a0 = g.a0;
    t.sigma0 = g.sigma0;
    t.delta = g.delta;
    t.phi0 = g.phi0;
    t.dpsi = g.dpsi;
    e = tp::prepare_lprec(t);
    if (e == hipSuccess && kt_bytes) {
        e = tp::launch_lprec_ktable(t, reinterpret_cast<float2*>(b), nullptr);
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    }
    if (e != hipSuccess) {
        (void)hipFree(le.block);
        return hip_fail(e, "log-polar kernel attributes or kernel table");
    }
    plan->lp.emplace(key, le);
    *out = t;
    return TP_OK;
}

tp_status lp_plan_grid(const tp_plan* plan, int32_t spans, double os, double eps, tp_lprec_grid* g) {
    if (!lp_angles_uniform(plan))
        return fail(TP_EUNSUPPORTED, "the log-polar method needs angles theta_0 + a pi / n_angles (equally spaced "
                    "over a half turn, increasing)");
    if (plan->filt.L > 8192) return fail(TP_EUNSUPPORTED, "pad length %d > 8192", plan->filt.L);
    return lp_grid(plan->na, plan->N, spans, os, eps, g);
}

}  // namespace

extern "C" {

const char* tp_last_error(void) { return g_err.c_str(); }

const char* tp_version(void) { return kVersion; }

tp_status tp_plan_create(const tp_geometry* g, tp_plan** out) {
    if (!out) return fail(TP_EINVAL, "out is null");
    *out = nullptr;
    if (!g) return fail(TP_EINVAL, "geometry is null");
    if (g->n_angles <= 0 || g->n_det <= 0 || g->n_vox < 0)
        return fail(TP_EINVAL, "bad geometry sizes (n_angles=%d n_det=%d n_vox=%d)", g->n_angles, g->n_det,
                    g->n_vox);
    if (!g->angles) return fail(TP_EINVAL, "angles is null");
    if (!std::isfinite(g->center)) return fail(TP_EINVAL, "center is not finite");
    const int N = g->n_vox ? g->n_vox : g->n_det;
    if (default_pad_len(g->n_det) > kMaxPadLen)
        return fail(TP_EUNSUPPORTED, "n_det=%d needs pad length > %d", g->n_det, kMaxPadLen);
    if (N > 32768) return fail(TP_EUNSUPPORTED, "n_vox=%d too large (limit 32768)", N);
    for (int a = 0; a < g->n_angles; ++a)
        if (!std::isfinite(g->angles[a])) return fail(TP_EINVAL, "angle %d is not finite", a);
    // the detector coordinate must stay well inside int32 and the FP32 offset small
    if (std::fabs(g->center) > 1e6) return fail(TP_EINVAL, "center %g out of range", g->center);

    const int na = g->n_angles;
    const int nb = (N + tp::kGeoTile - 1) / tp::kGeoTile;
    const int half = N / 2;
    std::vector<float> cs(na), sn(na), xf(static_cast<size_t>(nb) * na), yf(static_cast<size_t>(nb) * na);
    std::vector<int> xi(static_cast<size_t>(nb) * na), yi(static_cast<size_t>(nb) * na);
    for (int a = 0; a < na; ++a) {
        const double c = std::cos(g->angles[a]), s = std::sin(g->angles[a]);
        cs[a] = static_cast<float>(c);
        sn[a] = static_cast<float>(s);
        for (int b = 0; b < nb; ++b) {
            const double o = static_cast<double>(b * tp::kGeoTile - half);
            const double X = o * c;
            const double Y = o * s + g->center;
            const double fx = std::floor(X), fy = std::floor(Y);
            xi[static_cast<size_t>(b) * na + a] = static_cast<int>(fx);
            xf[static_cast<size_t>(b) * na + a] = static_cast<float>(X - fx);
            yi[static_cast<size_t>(b) * na + a] = static_cast<int>(fy);
            yf[static_cast<size_t>(b) * na + a] = static_cast<float>(Y - fy);
        }
    }
    // Forward-projector grouping.  Angles sweep rows (|cos| >= |sin|) or
    // columns; within each class the sign of the swept coefficient decides on
    // which side of the image a bin's strip lies (angles near 0 and near pi
    // are mirror images), so each class is split by that sign.  Each of the 4
    // segments is sorted by the angle reduced modulo pi into [-pi/4, 3pi/4)
    // (neighbours share a work-group) and padded with -1 to a multiple of 8
    // entries, so no work-group of 4 or 8 angles straddles two segments.
    auto key = [&](int a) {
        double t = std::fmod(g->angles[a] + M_PI / 4, M_PI);
        if (t < 0) t += M_PI;
        return t - M_PI / 4;
    };
    auto by_angle = [&](int p, int q) { return key(p) < key(q) || (key(p) == key(q) && p < q); };
    std::vector<int> seg[4];
    for (int a = 0; a < na; ++a) {
        const bool rows = std::fabs(cs[a]) >= std::fabs(sn[a]);
        const bool neg = rows ? cs[a] < 0.0f : sn[a] < 0.0f;
        seg[(rows ? 0 : 2) + (neg ? 1 : 0)].push_back(a);
    }
    std::vector<int> order;
    order.reserve(na + 16);
    int n_rows_major = 0;
    for (int q = 0; q < 4; ++q) {
        std::sort(seg[q].begin(), seg[q].end(), by_angle);
        order.insert(order.end(), seg[q].begin(), seg[q].end());
        while (order.size() % 8) order.push_back(-1);
        if (q == 1) n_rows_major = static_cast<int>(order.size());
    }
    const int n_order = static_cast<int>(order.size());
    const size_t s_ang = align256(sizeof(float) * na);
    const size_t s_tab = align256(sizeof(float) * static_cast<size_t>(nb) * na);
    const size_t s_ord = align256(sizeof(int) * static_cast<size_t>(n_order));
    const size_t total = 2 * s_ang + 4 * s_tab + s_ord;

    tp_plan* p = new (std::nothrow) tp_plan();
    if (!p) return fail(TP_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipGetDevice");
    }
    e = hipMalloc(&p->dev_block, total);
    if (e != hipSuccess) {
        delete p;
        return fail(TP_ENOMEM, "hipMalloc(plan tables, %zu bytes): %s", total, hipGetErrorString(e));
    }
    char* base = static_cast<char*>(p->dev_block);
    char* d_cs = base;
    char* d_sn = d_cs + s_ang;
    char* d_xi = d_sn + s_ang;
    char* d_xf = d_xi + s_tab;
    char* d_yi = d_xf + s_tab;
    char* d_yf = d_yi + s_tab;
    char* d_order = d_yf + s_tab;
    const size_t tb = sizeof(float) * static_cast<size_t>(nb) * na;
    e = hipMemcpy(d_cs, cs.data(), sizeof(float) * na, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_sn, sn.data(), sizeof(float) * na, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_xi, xi.data(), tb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_xf, xf.data(), tb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_yi, yi.data(), tb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_yf, yf.data(), tb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_order, order.data(), sizeof(int) * n_order, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p->dev_block);
        delete p;
        return hip_fail(e, "hipMemcpy(plan tables)");
    }
    p->angles.assign(g->angles, g->angles + na);
    p->na = na;
    p->n = g->n_det;
    p->N = N;
    p->nb = nb;
    p->center = g->center;
    p->geo.cs = reinterpret_cast<const float*>(d_cs);
    p->geo.sn = reinterpret_cast<const float*>(d_sn);
    p->geo.xi = reinterpret_cast<const int*>(d_xi);
    p->geo.xf = reinterpret_cast<const float*>(d_xf);
    p->geo.yi = reinterpret_cast<const int*>(d_yi);
    p->geo.yf = reinterpret_cast<const float*>(d_yf);
    p->geo.na = na;
    p->geo.n = g->n_det;
    p->geo.N = N;
    p->geo.nb = nb;
    p->geo.center_f = static_cast<float>(g->center);
    p->geo.order = reinterpret_cast<const int*>(d_order);
    p->geo.n_rows_major = n_rows_major;
    p->geo.n_order = n_order;
    tp_status st = filter_tables(default_pad_len(g->n_det), TP_RAMP, &p->filt, nullptr);
    if (st != TP_OK) {
        (void)hipFree(p->dev_block);
        delete p;
        return st;
    }
    if (!tp::tune_table_empty()) {
        // tilings recorded by the autotuner for this device and shape (tp_tune_load)
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
            for (int d = TP_F32; d <= TP_BF16; ++d) {
                int k = 0, a = 0;
                if (tp::tune_table_lookup(prop.name, d, na, g->n_det, N, &k, &a)) {
                    p->bp_k[d] = k;
                    p->bp_a[d] = a;
                }
            }
        }
    }
    g_live_plans.fetch_add(1);
    *out = p;
    return TP_OK;
}

tp_status tp_plan_destroy(tp_plan* plan) {
    if (!plan) return TP_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != plan->device) (void)hipSetDevice(plan->device);
    hipError_t e = hipFree(plan->dev_block);
    for (auto& kv : plan->fr) {
        const hipError_t e2 = hipFree(kv.second.block);
        if (e == hipSuccess) e = e2;
    }
    for (auto& kv : plan->lam) {
        const hipError_t e2 = hipFree(kv.second.block);
        if (e == hipSuccess) e = e2;
    }
    for (auto& kv : plan->lp) {
        const hipError_t e2 = hipFree(kv.second.block);
        if (e == hipSuccess) e = e2;
    }
    if (cur != plan->device) (void)hipSetDevice(cur);
    delete plan;
    g_live_plans.fetch_sub(1);
    if (e != hipSuccess) return hip_fail(e, "hipFree(plan tables)");
    return TP_OK;
}

tp_status tp_prepare(const tp_plan* plan, tp_filter_kind kind, tp_dtype storage) {
    if (!plan) return fail(TP_EINVAL, "plan is null");
    if (!valid_kind(kind)) return fail(TP_EUNSUPPORTED, "unknown filter kind %d", static_cast<int>(kind));
    if (!valid_dtype(storage)) return fail(TP_EINVAL, "bad storage dtype %d", storage);
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != plan->device)
        return fail(TP_EINVAL, "plan belongs to device %d, current device is %d", plan->device, cur);
    tp::FilterTables ft;
    tp_status s = filter_tables(plan->filt.L, kind, &ft, nullptr);
    if (s != TP_OK) return s;
    e = tp::prepare_backproject(storage, plan->bp_k[storage], plan->bp_a[storage]);
    if (e != hipSuccess) return hip_fail(e, "backprojection kernel attribute");
    return TP_OK;
}

tp_status tp_tune_load(const char* json_path) {
    std::string err;
    if (tp::tune_table_load(json_path, &err) < 0) return fail(TP_EINVAL, "%s", err.c_str());
    return TP_OK;
}

tp_status tp_tune_lookup(const char* device_name, tp_dtype storage, int32_t n_angles, int32_t n_det, int32_t n_vox,
                         int32_t* slices_per_block, int32_t* angles_per_block) {
    if (!device_name || !slices_per_block || !angles_per_block) return fail(TP_EINVAL, "null argument");
    if (!valid_dtype(storage)) return fail(TP_EINVAL, "bad storage dtype %d", storage);
    const int N = n_vox ? n_vox : n_det;
    int k = 0, a = 0;
    if (!tp::tune_table_lookup(device_name, storage, n_angles, n_det, N, &k, &a))
        return fail(TP_EINVAL, "no tiling recorded for %s storage %d, %d angles, %d columns, %d voxels", device_name,
                    static_cast<int>(storage), n_angles, n_det, N);
    *slices_per_block = k;
    *angles_per_block = a;
    return TP_OK;
}

tp_status tp_shutdown(void) {
    const int live = g_live_plans.load();
    if (live > 0) return fail(TP_EINVAL, "%d plan(s) still exist; destroy them before tp_shutdown", live);
    std::string ignore;
    (void)tp::tune_table_load(nullptr, &ignore);
    std::lock_guard<std::mutex> lk(g_filter_mu);
    if (g_filter_cache.empty()) return TP_OK;
    int cur = 0;
    hipError_t first = hipGetDevice(&cur);
    for (auto& kv : g_filter_cache) {
        const int dev = std::get<0>(kv.first);
        hipError_t e = hipSetDevice(dev);
        if (e == hipSuccess) e = hipFree(kv.second.tw);
        const hipError_t e2 = hipFree(kv.second.H);
        if (first == hipSuccess) first = e != hipSuccess ? e : e2;
    }
    g_filter_cache.clear();
    (void)hipSetDevice(cur);
    if (first != hipSuccess) return hip_fail(first, "freeing the filter tables");
    return TP_OK;
}

tp_status tp_plan_set_tuning(tp_plan* plan, tp_dtype storage, int32_t slices_per_block,
                             int32_t angles_per_block) {
    if (!plan) return fail(TP_EINVAL, "plan is null");
    if (!valid_dtype(storage)) return fail(TP_EINVAL, "bad storage dtype %d", storage);
    const int k = slices_per_block, a = angles_per_block;
    if (!(k == 1 || k == 2 || k == 4 || k == 8 || k == 16))
        return fail(TP_EINVAL, "slices_per_block=%d not in {1,2,4,8,16}", k);
    if (!(a == 8 || a == 16 || a == 32 || a == 64))
        return fail(TP_EINVAL, "angles_per_block=%d not in {8,16,32,64}", a);
    if (tp::backproject_lds_bytes(storage, k, a) > kMaxLds)
        return fail(TP_EINVAL, "slices_per_block=%d x angles_per_block=%d exceeds LDS", k, a);
    plan->bp_k[storage] = k;
    plan->bp_a[storage] = a;
    return TP_OK;
}

tp_status tp_plan_get_tuning(const tp_plan* plan, tp_dtype storage, int32_t* slices_per_block,
                             int32_t* angles_per_block) {
    if (!plan || !slices_per_block || !angles_per_block) return fail(TP_EINVAL, "null argument");
    if (!valid_dtype(storage)) return fail(TP_EINVAL, "bad storage dtype %d", storage);
    *slices_per_block = plan->bp_k[storage];
    *angles_per_block = plan->bp_a[storage];
    return TP_OK;
}

tp_status tp_filter_prepare(int32_t pad_len, tp_filter_kind kind) {
    if (!valid_kind(kind)) return fail(TP_EUNSUPPORTED, "unknown filter kind %d", static_cast<int>(kind));
    if (!is_pow2(pad_len) || pad_len < 2 || pad_len > kMaxPadLen)
        return fail(TP_EINVAL, "pad_len=%d must be a power of two in [2, %d]", pad_len, kMaxPadLen);
    tp::FilterTables ft;
    return filter_tables(pad_len, kind, &ft, nullptr);
}

tp_status tp_filter_response(int32_t pad_len, tp_filter_kind kind, double* H) {
    if (!valid_kind(kind)) return fail(TP_EUNSUPPORTED, "unknown filter kind %d", static_cast<int>(kind));
    if (!H) return fail(TP_EINVAL, "H is null");
    if (!is_pow2(pad_len) || pad_len < 2 || pad_len > kMaxPadLen)
        return fail(TP_EINVAL, "pad_len=%d must be a power of two in [2, %d]", pad_len, kMaxPadLen);
    std::vector<double> r;
    filter_response_fp64(pad_len, kind, r);
    std::copy(r.begin(), r.end(), H);
    return TP_OK;
}

size_t tp_normalize_workspace_bytes(int32_t n_rows, int32_t n_det) {
    if (n_rows <= 0 || n_det <= 0) return 0;
    return 2 * align256(sizeof(float) * static_cast<size_t>(n_rows) * n_det);
}

tp_status tp_normalize(const uint16_t* proj, int64_t proj_stride, const uint16_t* dark, int32_t n_dark,
                       const uint16_t* flat, int32_t n_flat, int64_t frame_stride, int32_t n_angles,
                       int32_t n_rows, int32_t n_det, tp_dtype out_dtype, void* sino, void* workspace,
                       size_t workspace_bytes, void* stream) {
    tp_status s = check_raw(proj, dark, n_dark, flat, n_flat, &proj_stride, &frame_stride, n_angles, n_rows,
                            n_det);
    if (s != TP_OK) return s;
    if (!valid_dtype(out_dtype)) return fail(TP_EINVAL, "bad out_dtype %d", out_dtype);
    if (!sino) return fail(TP_EINVAL, "sino is null");
    if (!workspace) return fail(TP_EINVAL, "workspace is null");
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(TP_EINVAL, "workspace not 256-byte aligned");
    const size_t need = tp_normalize_workspace_bytes(n_rows, n_det);
    if (workspace_bytes < need) return fail(TP_EINVAL, "workspace %zu < %zu bytes", workspace_bytes, need);
    auto st = static_cast<hipStream_t>(stream);
    float* dmean = static_cast<float*>(workspace);
    float* den = reinterpret_cast<float*>(static_cast<char*>(workspace) + need / 2);
    tp::RawInput in{proj, proj_stride, dark, flat, frame_stride, n_dark, n_flat};
    hipError_t e = tp::launch_darkflat(in, n_rows, n_det, dmean, den, st);
    if (e != hipSuccess) return hip_fail(e, "darkflat launch");
    e = tp::launch_normalize(in, dmean, den, n_angles, n_rows, n_det, out_dtype, sino, st);
    if (e != hipSuccess) return hip_fail(e, "normalize launch");
    return TP_OK;
}

tp_status tp_normalize_noalloc(const uint16_t* proj, int64_t proj_stride, const uint16_t* dark, int32_t n_dark,
                               const uint16_t* flat, int32_t n_flat, int64_t frame_stride, int32_t n_angles,
                               int32_t n_rows, int32_t n_det, tp_dtype out_dtype, void* sino, void* stream) {
    tp_status s = check_raw(proj, dark, n_dark, flat, n_flat, &proj_stride, &frame_stride, n_angles, n_rows,
                            n_det);
    if (s != TP_OK) return s;
    if (!valid_dtype(out_dtype)) return fail(TP_EINVAL, "bad out_dtype %d", out_dtype);
    if (!sino) return fail(TP_EINVAL, "sino is null");
    const int64_t pixels = static_cast<int64_t>(n_rows) * n_det;
    if (pixels > TP_NOALLOC_MAX_PIXELS)
        return fail(TP_EINVAL, "n_rows*n_det=%lld exceeds the allocation-free limit of %lld pixels",
                    static_cast<long long>(pixels), static_cast<long long>(TP_NOALLOC_MAX_PIXELS));
    float* dmean = nullptr;
    float* den = nullptr;
    hipError_t e = tp::normalize_scratch(&dmean, &den);
    if (e != hipSuccess) return hip_fail(e, "scratch address of the allocation-free normaliser");
    auto st = static_cast<hipStream_t>(stream);
    tp::RawInput in{proj, proj_stride, dark, flat, frame_stride, n_dark, n_flat};
    e = tp::launch_darkflat(in, n_rows, n_det, dmean, den, st);
    if (e != hipSuccess) return hip_fail(e, "darkflat launch");
    e = tp::launch_normalize(in, dmean, den, n_angles, n_rows, n_det, out_dtype, sino, st);
    if (e != hipSuccess) return hip_fail(e, "normalize launch");
    return TP_OK;
}

tp_status tp_filter(const void* sino, tp_dtype in_dtype, void* filt, tp_dtype out_dtype, int64_t n_lines,
                    int32_t n_det, int32_t pad_len, tp_filter_kind kind, void* stream) {
    if (!valid_kind(kind)) return fail(TP_EUNSUPPORTED, "unknown filter kind %d", static_cast<int>(kind));
    if (!sino || !filt) return fail(TP_EINVAL, "null buffer");
    if (!valid_dtype(in_dtype) || !valid_dtype(out_dtype)) return fail(TP_EINVAL, "bad dtype");
    if (n_lines <= 0 || n_det <= 0) return fail(TP_EINVAL, "n_lines and n_det must be positive");
    if ((n_lines + 1) / 2 > 0x7fffffffLL) return fail(TP_EINVAL, "n_lines too large");
    const int L = pad_len == 0 ? default_pad_len(n_det) : pad_len;
    if (!is_pow2(L) || L < n_det || L > kMaxPadLen)
        return fail(pad_len == 0 ? TP_EUNSUPPORTED : TP_EINVAL,
                    "pad_len=%d must be a power of two with n_det <= pad_len <= %d", L, kMaxPadLen);
    const size_t in_bytes = static_cast<size_t>(n_lines) * n_det * dtype_size(in_dtype);
    const size_t out_bytes = static_cast<size_t>(n_lines) * n_det * dtype_size(out_dtype);
    const char* a0 = static_cast<const char*>(sino);
    const char* b0 = static_cast<const char*>(filt);
    const bool overlap = a0 < b0 + out_bytes && b0 < a0 + in_bytes;
    if (overlap && !(a0 == b0 && in_dtype == out_dtype))
        return fail(TP_EINVAL, "filt overlaps sino (in place only with identical pointers and dtypes)");
    auto st = static_cast<hipStream_t>(stream);
    tp::FilterTables ft;
    tp_status s = filter_tables(L, kind, &ft, st);
    if (s != TP_OK) return s;
    hipError_t e = tp::launch_filter(sino, in_dtype, filt, out_dtype, n_lines, n_det, ft, st);
    if (e != hipSuccess) return hip_fail(e, "filter launch");
    return TP_OK;
}

tp_status tp_backproject(const tp_plan* plan, const void* filt, tp_dtype in_dtype, int32_t n_rows, float scale,
                         float* vol, int32_t accumulate, void* stream) {
    if (!plan) return fail(TP_EINVAL, "plan is null");
    if (!filt || !vol) return fail(TP_EINVAL, "null buffer");
    if (!valid_dtype(in_dtype)) return fail(TP_EINVAL, "bad dtype %d", in_dtype);
    if (n_rows <= 0 || n_rows > 65535 * 8) return fail(TP_EINVAL, "n_rows=%d out of range", n_rows);
    if (!(accumulate == 0 || accumulate == 1)) return fail(TP_EINVAL, "accumulate must be 0 or 1");
    if (!std::isfinite(scale)) return fail(TP_EINVAL, "scale is not finite");
    const int K = plan->bp_k[in_dtype], A = plan->bp_a[in_dtype];
    if ((n_rows + K - 1) / K > 65535)
        return fail(TP_EINVAL, "n_rows=%d too large for slices_per_block=%d", n_rows, K);
    hipError_t e = tp::launch_backproject(plan->geo, filt, in_dtype, n_rows, scale, vol, TP_F32, accumulate, K, A,
                                          static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "backproject launch");
    return TP_OK;
}

size_t tp_radon_workspace_bytes(const tp_plan* plan, int32_t n_rows) {
    if (!plan || n_rows <= 0) return 0;
    return tp::radon_workspace_bytes(plan->geo, n_rows);
}

tp_status tp_radon(const tp_plan* plan, const float* vol, int32_t n_rows, float* sino, void* workspace,
                   size_t workspace_bytes, void* stream) {
    if (!plan) return fail(TP_EINVAL, "plan is null");
    if (!vol || !sino) return fail(TP_EINVAL, "null buffer");
    if (n_rows <= 0 || n_rows > 65535) return fail(TP_EINVAL, "n_rows=%d out of range [1, 65535]", n_rows);
    const size_t need = tp::radon_workspace_bytes(plan->geo, n_rows);
    if (need > 0) {
        if (!workspace) return fail(TP_EINVAL, "workspace is null (%zu bytes needed)", need);
        if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(TP_EINVAL, "workspace not 256-byte aligned");
        if (workspace_bytes < need) return fail(TP_EINVAL, "workspace %zu < %zu bytes", workspace_bytes, need);
        const char* w0 = static_cast<const char*>(workspace);
        const char* v0 = reinterpret_cast<const char*>(vol);
        const char* s0 = reinterpret_cast<const char*>(sino);
        const size_t vb = need, sb = sizeof(float) * static_cast<size_t>(n_rows) * plan->na * plan->n;
        if ((w0 < v0 + vb && v0 < w0 + need) || (w0 < s0 + sb && s0 < w0 + need))
            return fail(TP_EINVAL, "workspace overlaps vol or sino");
    }
    hipError_t e = tp::launch_radon(plan->geo, vol, n_rows, sino, static_cast<float*>(workspace),
                                    static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "radon launch");
    return TP_OK;
}

size_t tp_fbp_workspace_bytes(const tp_plan* plan, int32_t n_rows, tp_dtype storage) {
    if (!plan || n_rows <= 0 || !valid_dtype(storage)) return 0;
    return tp_normalize_workspace_bytes(n_rows, plan->n) +
           align256(static_cast<size_t>(n_rows) * plan->na * plan->n * dtype_size(storage));
}

tp_status tp_fbp_chunk(const tp_plan* plan, const uint16_t* proj, int64_t proj_stride, const uint16_t* dark,
                       int32_t n_dark, const uint16_t* flat, int32_t n_flat, int64_t frame_stride, int32_t n_rows,
                       tp_filter_kind kind, tp_dtype storage, void* workspace, size_t workspace_bytes, float* vol,
                       void* stream) {
    return tp_fbp_chunk_events(plan, proj, proj_stride, dark, n_dark, flat, n_flat, frame_stride, n_rows, kind,
                               storage, workspace, workspace_bytes, vol, stream, nullptr);
}

tp_status tp_fbp_chunk_events(const tp_plan* plan, const uint16_t* proj, int64_t proj_stride, const uint16_t* dark,
                              int32_t n_dark, const uint16_t* flat, int32_t n_flat, int64_t frame_stride,
                              int32_t n_rows, tp_filter_kind kind, tp_dtype storage, void* workspace,
                              size_t workspace_bytes, float* vol, void* stream, void* const* events) {
    return tp_fbp_chunk_out(plan, proj, proj_stride, dark, n_dark, flat, n_flat, frame_stride, n_rows, kind, storage,
                            workspace, workspace_bytes, TP_F32, vol, stream, events);
}

tp_status tp_fbp_chunk_out(const tp_plan* plan, const uint16_t* proj, int64_t proj_stride, const uint16_t* dark,
                           int32_t n_dark, const uint16_t* flat, int32_t n_flat, int64_t frame_stride, int32_t n_rows,
                           tp_filter_kind kind, tp_dtype storage, void* workspace, size_t workspace_bytes,
                           tp_dtype vol_dtype, void* vol, void* stream, void* const* events) {
    if (!plan) return fail(TP_EINVAL, "plan is null");
    tp_status s = check_raw(proj, dark, n_dark, flat, n_flat, &proj_stride, &frame_stride, plan->na, n_rows,
                            plan->n);
    if (s != TP_OK) return s;
    if (!valid_kind(kind)) return fail(TP_EUNSUPPORTED, "unknown filter kind %d", static_cast<int>(kind));
    if (!valid_dtype(storage)) return fail(TP_EINVAL, "bad storage dtype %d", storage);
    if (vol_dtype != TP_F32 && vol_dtype != TP_F16) return fail(TP_EINVAL, "bad volume dtype %d", vol_dtype);
    if (vol_dtype == TP_F16 && storage != TP_F16)
        return fail(TP_EUNSUPPORTED, "FP16 slices need FP16 storage (the 16-bit mode)");
    if (!vol) return fail(TP_EINVAL, "vol is null");
    if (!workspace) return fail(TP_EINVAL, "workspace is null");
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(TP_EINVAL, "workspace not 256-byte aligned");
    const size_t need = tp_fbp_workspace_bytes(plan, n_rows, storage);
    if (workspace_bytes < need) return fail(TP_EINVAL, "workspace %zu < %zu bytes", workspace_bytes, need);
    const int K = plan->bp_k[storage], A = plan->bp_a[storage];
    if ((n_rows + K - 1) / K > 65535)
        return fail(TP_EINVAL, "n_rows=%d too large for slices_per_block=%d", n_rows, K);
    if (static_cast<int64_t>(n_rows) * ((plan->na + 1) / 2) > 0x7fffffffLL)
        return fail(TP_EINVAL, "n_rows=%d x n_angles=%d too large for one call", n_rows, plan->na);
    auto st = static_cast<hipStream_t>(stream);
    tp::FilterTables ft = plan->filt;
    if (kind != TP_RAMP && (s = filter_tables(plan->filt.L, kind, &ft, st)) != TP_OK) return s;
    const size_t dfb = tp_normalize_workspace_bytes(n_rows, plan->n);
    float* dmean = static_cast<float*>(workspace);
    float* den = reinterpret_cast<float*>(static_cast<char*>(workspace) + dfb / 2);
    void* filt = static_cast<char*>(workspace) + dfb;
    tp::RawInput in{proj, proj_stride, dark, flat, frame_stride, n_dark, n_flat};
    auto mark = [&](int i) -> hipError_t {
        if (!events || !events[i]) return hipSuccess;
        return hipEventRecord(static_cast<hipEvent_t>(events[i]), st);
    };
    hipError_t e = mark(0);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    e = tp::launch_darkflat(in, n_rows, plan->n, dmean, den, st);
    if (e != hipSuccess) return hip_fail(e, "darkflat launch");
    if ((e = mark(1)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    e = tp::launch_norm_filter(in, dmean, den, plan->na, n_rows, plan->n, ft, storage, filt, st);
    if (e != hipSuccess) return hip_fail(e, "norm_filter launch");
    if ((e = mark(2)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    e = tp::launch_backproject(plan->geo, filt, storage, n_rows, static_cast<float>(M_PI / plan->na), vol, vol_dtype,
                               0, K, A, st);
    if (e != hipSuccess) return hip_fail(e, "backproject launch");
    if ((e = mark(3)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    return TP_OK;
}

tp_status tp_lamino_prepare(const tp_plan* plan, double tilt, double center_v, int32_t n_slices) {
    tp_status s = lamino_check(plan, tilt, center_v, n_slices);
    if (s != TP_OK) return s;
    tp::LaminoTables t;
    return lamino_tables(plan, tilt, center_v, n_slices, &t, nullptr);
}

tp_status tp_lamino_backproject(const tp_plan* plan, const void* filt, tp_dtype in_dtype, int32_t det_rows,
                                double tilt, double center_v, int32_t n_slices, int32_t z0, int32_t nz, float scale,
                                float* vol, void* stream) {
    tp_status s = lamino_check(plan, tilt, center_v, n_slices);
    if (s != TP_OK) return s;
    if (!filt || !vol) return fail(TP_EINVAL, "null filt or vol");
    if (!valid_dtype(in_dtype)) return fail(TP_EINVAL, "bad dtype %d", in_dtype);
    if (det_rows <= 0) return fail(TP_EINVAL, "det_rows=%d must be positive", det_rows);
    if (static_cast<int64_t>(det_rows) * plan->n >= (int64_t{1} << 31))
        return fail(TP_EINVAL, "det_rows=%d x n_det=%d samples per projection exceed 2^31", det_rows, plan->n);
    if (z0 < 0 || nz <= 0 || z0 + static_cast<int64_t>(nz) > n_slices)
        return fail(TP_EINVAL, "slices [%d, %d) outside [0, %d)", z0, z0 + nz, n_slices);
    const int kb = tp::lamino_slices_per_block();  // slice blocks are aligned to multiples of kb
    const int64_t lam_blocks = static_cast<int64_t>(plan->geo.nb) * plan->geo.nb *
                               ((static_cast<int64_t>(z0) + nz - 1) / kb - z0 / kb + 1);
    if (lam_blocks >= (int64_t{1} << 31)) return fail(TP_EINVAL, "nz=%d too large for one call", nz);
    if (!std::isfinite(scale)) return fail(TP_EINVAL, "scale is not finite");
    auto st = static_cast<hipStream_t>(stream);
    tp::LaminoTables t;
    if ((s = lamino_tables(plan, tilt, center_v, n_slices, &t, st)) != TP_OK) return s;
    t.rows = det_rows;
    const hipError_t e = tp::launch_lamino(plan->geo, t, filt, in_dtype, z0, nz, scale, vol, st);
    if (e != hipSuccess) return hip_fail(e, "laminography launch");
    return TP_OK;
}

size_t tp_fourier_workspace_bytes(const tp_plan* plan, int32_t n_rows) {
    if (!plan || n_rows <= 0) return 0;
    return fr_workspace(plan, n_rows, (n_rows + 1) / 2);
}

tp_status tp_fourier_prepare(const tp_plan* plan, tp_filter_kind kind, int32_t half_width) {
    if (!plan) return fail(TP_EINVAL, "plan is null");
    if (!valid_kind(kind)) return fail(TP_EUNSUPPORTED, "unknown filter kind %d", static_cast<int>(kind));
    int msp = 0;
    tp_status s = fourier_half_width(half_width, &msp);
    if (s != TP_OK) return s;
    const FrDims d = fr_dims(plan);
    if (d.M > kFourierMaxSide) return fail(TP_EUNSUPPORTED, "Fourier grid side %d > %d", d.M, kFourierMaxSide);
    tp::FourierTables t;
    if ((s = fourier_tables(plan, kind, msp, &t, nullptr)) != TP_OK) return s;
    tp::FilterTables fm;
    return filter_tables(d.M, TP_RAMP, &fm, nullptr);
}

tp_status tp_fourier_fbp_chunk(const tp_plan* plan, const uint16_t* proj, int64_t proj_stride, const uint16_t* dark,
                               int32_t n_dark, const uint16_t* flat, int32_t n_flat, int64_t frame_stride,
                               int32_t n_rows, tp_filter_kind kind, int32_t half_width, void* workspace,
                               size_t workspace_bytes, float* vol, void* stream) {
    return tp_fourier_fbp_chunk_events(plan, proj, proj_stride, dark, n_dark, flat, n_flat, frame_stride, n_rows,
                                       kind, half_width, workspace, workspace_bytes, vol, stream, nullptr);
}

tp_status tp_fourier_fbp_chunk_events(const tp_plan* plan, const uint16_t* proj, int64_t proj_stride,
                                      const uint16_t* dark, int32_t n_dark, const uint16_t* flat, int32_t n_flat,
                                      int64_t frame_stride, int32_t n_rows, tp_filter_kind kind, int32_t half_width,
                                      void* workspace, size_t workspace_bytes, float* vol, void* stream,
                                      void* const* events) {
    return tp_fourier_fbp_chunk_out(plan, proj, proj_stride, dark, n_dark, flat, n_flat, frame_stride, n_rows, kind,
                                    half_width, workspace, workspace_bytes, TP_F32, vol, stream, events);
}

tp_status tp_fourier_fbp_chunk_out(const tp_plan* plan, const uint16_t* proj, int64_t proj_stride,
                                   const uint16_t* dark, int32_t n_dark, const uint16_t* flat, int32_t n_flat,
                                   int64_t frame_stride, int32_t n_rows, tp_filter_kind kind, int32_t half_width,
                                   void* workspace, size_t workspace_bytes, tp_dtype vol_dtype, void* vol,
                                   void* stream, void* const* events) {
    if (!plan) return fail(TP_EINVAL, "plan is null");
    if (vol_dtype != TP_F32 && vol_dtype != TP_F16)
        return fail(TP_EUNSUPPORTED, "vol_dtype %d: FP32 or FP16 slices only", static_cast<int>(vol_dtype));
    tp_status s = check_raw(proj, dark, n_dark, flat, n_flat, &proj_stride, &frame_stride, plan->na, n_rows,
                            plan->n);
    if (s != TP_OK) return s;
    if (!valid_kind(kind)) return fail(TP_EUNSUPPORTED, "unknown filter kind %d", static_cast<int>(kind));
    int msp = 0;
    if ((s = fourier_half_width(half_width, &msp)) != TP_OK) return s;
    if (!vol) return fail(TP_EINVAL, "vol is null");
    if (!workspace) return fail(TP_EINVAL, "workspace is null");
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(TP_EINVAL, "workspace not 256-byte aligned");
    const FrDims d = fr_dims(plan);
    if (d.M > kFourierMaxSide) return fail(TP_EUNSUPPORTED, "Fourier grid side %d > %d", d.M, kFourierMaxSide);
    const int pairs = (n_rows + 1) / 2;
    const size_t df = tp_normalize_workspace_bytes(n_rows, plan->n);
    if (workspace_bytes < fr_workspace(plan, n_rows, 1))
        return fail(TP_EINVAL, "workspace %zu < %zu bytes (one pair of rows)", workspace_bytes,
                    fr_workspace(plan, n_rows, 1));
    int64_t P = static_cast<int64_t>((workspace_bytes - df) / (std::max(d.spec_pair, d.cols_pair) + d.grid_pair));
    P = std::min<int64_t>(std::max<int64_t>(P, 1), pairs);
    const int64_t ntiles = static_cast<int64_t>(tp::fourier_grid_tiles(d.M));
    P = std::min<int64_t>(P, 0x7fffffffLL / std::max<int64_t>({ntiles, plan->na, d.M}));
    while (P > 1 && fr_workspace(plan, n_rows, P) > workspace_bytes) --P;
    if (P < 1) return fail(TP_EINVAL, "grid too large for one launch");
    auto st = static_cast<hipStream_t>(stream);
    tp::FourierTables t;
    if ((s = fourier_tables(plan, kind, msp, &t, st)) != TP_OK) return s;
    tp::FilterTables fm;
    if ((s = filter_tables(d.M, TP_RAMP, &fm, st)) != TP_OK) return s;
    float* dmean = static_cast<float*>(workspace);
    float* den = reinterpret_cast<float*>(static_cast<char*>(workspace) + df / 2);
    char* regA = static_cast<char*>(workspace) + df;
    char* regB = regA + align256(static_cast<size_t>(P) * std::max(d.spec_pair, d.cols_pair));
    float2* spec = reinterpret_cast<float2*>(regA);
    float2* cols = reinterpret_cast<float2*>(regA);
    float2* grid = reinterpret_cast<float2*>(regB);
    tp::RawInput in{proj, proj_stride, dark, flat, frame_stride, n_dark, n_flat};
    bool first = true;
    auto mark = [&](int i) -> hipError_t {
        if (!first || !events || !events[i]) return hipSuccess;
        return hipEventRecord(static_cast<hipEvent_t>(events[i]), st);
    };
    hipError_t e = mark(0);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    e = tp::launch_darkflat(in, n_rows, plan->n, dmean, den, st);
    if (e != hipSuccess) return hip_fail(e, "darkflat launch");
    for (int r0 = 0; r0 < n_rows; r0 += static_cast<int>(2 * P)) {
        const int rows = std::min(static_cast<int>(2 * P), n_rows - r0);
        const int pp = (rows + 1) / 2;
        tp::RawInput ip = in;
        ip.proj = proj + static_cast<int64_t>(r0) * plan->n;
        const int64_t roff = static_cast<int64_t>(r0) * plan->n;
        if ((e = mark(1)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        e = tp::launch_fourier_spectra(ip, rows, dmean + roff, den + roff, plan->filt.tw, t, spec, st);
        if (e != hipSuccess) return hip_fail(e, "Fourier spectra launch");
        if ((e = mark(2)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        e = tp::launch_fourier_grid(t, spec, pp, grid, st);
        if (e != hipSuccess) return hip_fail(e, "Fourier grid launch");
        if ((e = mark(3)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        e = tp::launch_fourier_rows(t, fm.tw, grid, pp, cols, st);
        if (e != hipSuccess) return hip_fail(e, "Fourier row-transform launch");
        if ((e = mark(4)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        const size_t esize = vol_dtype == TP_F16 ? 2 : 4;
        e = tp::launch_fourier_cols(t, fm.tw, cols, pp, rows,
                                    static_cast<char*>(vol) + static_cast<int64_t>(r0) * plan->N * plan->N * esize,
                                    vol_dtype == TP_F16, st);
        if (e != hipSuccess) return hip_fail(e, "Fourier column-transform launch");
        if ((e = mark(5)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        first = false;
    }
    return TP_OK;
}

tp_status tp_lprec_grid_query(int32_t n_angles, int32_t n_vox, int32_t spans, double os, double eps,
                              tp_lprec_grid* out) {
    if (!out) return fail(TP_EINVAL, "out is null");
    if (n_angles <= 0 || n_vox <= 0) return fail(TP_EINVAL, "n_angles=%d n_vox=%d must be positive", n_angles, n_vox);
    return lp_grid(n_angles, n_vox, spans, os, eps, out);
}

size_t tp_lprec_workspace_bytes(const tp_plan* plan, int32_t n_rows, int32_t spans, double os, double eps) {
    if (!plan || n_rows <= 0) return 0;
    tp_lprec_grid g;
    if (lp_plan_grid(plan, spans, os, eps, &g) != TP_OK) return 0;
    return lp_workspace(plan, g, n_rows, (n_rows + 1) / 2);
}

tp_status tp_lprec_prepare(const tp_plan* plan, tp_filter_kind kind, int32_t spans, double os, double eps) {
    if (!plan) return fail(TP_EINVAL, "plan is null");
    if (!valid_kind(kind)) return fail(TP_EUNSUPPORTED, "unknown filter kind %d", static_cast<int>(kind));
    tp_lprec_grid g;
    tp_status s = lp_plan_grid(plan, spans, os, eps, &g);
    if (s != TP_OK) return s;
    tp::LprecTables t;
    return lprec_tables(plan, kind, g, &t, nullptr);
}

tp_status tp_lprec_fbp_chunk(const tp_plan* plan, const uint16_t* proj, int64_t proj_stride, const uint16_t* dark,
                             int32_t n_dark, const uint16_t* flat, int32_t n_flat, int64_t frame_stride,
                             int32_t n_rows, tp_filter_kind kind, int32_t spans, double os, double eps,
                             void* workspace, size_t workspace_bytes, float* vol, void* stream) {
    return tp_lprec_fbp_chunk_events(plan, proj, proj_stride, dark, n_dark, flat, n_flat, frame_stride, n_rows, kind,
                                     spans, os, eps, workspace, workspace_bytes, vol, stream, nullptr);
}

tp_status tp_lprec_fbp_chunk_events(const tp_plan* plan, const uint16_t* proj, int64_t proj_stride,
                                    const uint16_t* dark, int32_t n_dark, const uint16_t* flat, int32_t n_flat,
                                    int64_t frame_stride, int32_t n_rows, tp_filter_kind kind, int32_t spans,
                                    double os, double eps, void* workspace, size_t workspace_bytes, float* vol,
                                    void* stream, void* const* events) {
    if (!plan) return fail(TP_EINVAL, "plan is null");
    tp_status s = check_raw(proj, dark, n_dark, flat, n_flat, &proj_stride, &frame_stride, plan->na, n_rows,
                            plan->n);
    if (s != TP_OK) return s;
    if (!valid_kind(kind)) return fail(TP_EUNSUPPORTED, "unknown filter kind %d", static_cast<int>(kind));
    if (!vol) return fail(TP_EINVAL, "vol is null");
    if (!workspace) return fail(TP_EINVAL, "workspace is null");
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(TP_EINVAL, "workspace not 256-byte aligned");
    tp_lprec_grid g;
    if ((s = lp_plan_grid(plan, spans, os, eps, &g)) != TP_OK) return s;
    const int pairs = (n_rows + 1) / 2;
    const size_t df = tp_normalize_workspace_bytes(n_rows, plan->n);
    if (workspace_bytes < lp_workspace(plan, g, n_rows, 1))
        return fail(TP_EINVAL, "workspace %zu < %zu bytes (one pair of rows)", workspace_bytes,
                    lp_workspace(plan, g, n_rows, 1));
    const LpSizes z = lp_sizes(plan, g);
    int64_t P = static_cast<int64_t>((workspace_bytes - df) / (std::max(z.rows, z.fhat) + std::max(z.ghat, z.F)));
    P = std::min<int64_t>(std::max<int64_t>(P, 1), pairs);
    P = std::min<int64_t>(P, 65535);
    while (P > 1 && lp_workspace(plan, g, n_rows, P) > workspace_bytes) --P;
    auto st = static_cast<hipStream_t>(stream);
    tp::LprecTables t;
    if ((s = lprec_tables(plan, kind, g, &t, st)) != TP_OK) return s;
    float* dmean = static_cast<float*>(workspace);
    float* den = reinterpret_cast<float*>(static_cast<char*>(workspace) + df / 2);
    char* regA = static_cast<char*>(workspace) + df;
    char* regB = regA + align256(static_cast<size_t>(P) * std::max(z.rows, z.fhat));
    float2* rowsbuf = reinterpret_cast<float2*>(regA);
    float2* fhat = reinterpret_cast<float2*>(regA);
    float2* ghat = reinterpret_cast<float2*>(regB);
    float2* F = reinterpret_cast<float2*>(regB);
    tp::RawInput in{proj, proj_stride, dark, flat, frame_stride, n_dark, n_flat};
    bool first = true;
    auto mark = [&](int i) -> hipError_t {
        if (!first || !events || !events[i]) return hipSuccess;
        return hipEventRecord(static_cast<hipEvent_t>(events[i]), st);
    };
    hipError_t e = mark(0);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    e = tp::launch_darkflat(in, n_rows, plan->n, dmean, den, st);
    if (e != hipSuccess) return hip_fail(e, "darkflat launch");
    for (int r0 = 0; r0 < n_rows; r0 += static_cast<int>(2 * P)) {
        const int rows = std::min(static_cast<int>(2 * P), n_rows - r0);
        const int pp = (rows + 1) / 2;
        tp::RawInput ip = in;
        ip.proj = proj + static_cast<int64_t>(r0) * plan->n;
        const int64_t roff = static_cast<int64_t>(r0) * plan->n;
        if ((e = mark(1)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        e = tp::launch_lprec_rows(ip, rows, dmean + roff, den + roff, t, rowsbuf, st);
        if (e != hipSuccess) return hip_fail(e, "log-polar row-spline launch");
        if ((e = mark(2)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        e = tp::launch_lprec_logradial(t, rowsbuf, pp, ghat, st);
        if (e != hipSuccess) return hip_fail(e, "log-polar resampling launch");
        if ((e = mark(3)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        e = tp::launch_lprec_conv(t, ghat, pp, fhat, st);
        if (e != hipSuccess) return hip_fail(e, "log-polar convolution launch");
        if ((e = mark(4)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        e = tp::launch_lprec_sigma(t, fhat, pp, F, st);
        if (e != hipSuccess) return hip_fail(e, "log-polar sigma-transform launch");
        if ((e = mark(5)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        e = tp::launch_lprec_interp(t, F, pp, rows, vol + static_cast<int64_t>(r0) * plan->N * plan->N, st);
        if (e != hipSuccess) return hip_fail(e, "log-polar evaluation launch");
        if ((e = mark(6)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        first = false;
    }
    return TP_OK;
}

tp_status tp_peak_copy(const void* src, void* dst, int64_t bytes, void* stream) {
    if (!src || !dst) return fail(TP_EINVAL, "null buffer");
    if (bytes <= 0 || (bytes & 15)) return fail(TP_EINVAL, "bytes=%lld must be a positive multiple of 16",
                                                static_cast<long long>(bytes));
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15)
        return fail(TP_EINVAL, "buffers must be 16-byte aligned");
    const char* a = static_cast<const char*>(src);
    const char* b = static_cast<const char*>(dst);
    if (a < b + bytes && b < a + bytes) return fail(TP_EINVAL, "buffers overlap");
    const hipError_t e = tp::launch_peak_copy(src, dst, bytes, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "copy launch");
    return TP_OK;
}

tp_status tp_peak_valu(int32_t form, float* out, int32_t blocks, int32_t iters, int64_t* flop, void* stream) {
    if (!out || !flop) return fail(TP_EINVAL, "null argument");
    if (form < TP_VALU_FMA_F32 || form > TP_VALU_DOT2_F16) return fail(TP_EINVAL, "unknown VALU form %d", form);
    if (blocks <= 0 || blocks > (1 << 20) || iters <= 0 || iters > (1 << 24))
        return fail(TP_EINVAL, "blocks=%d iters=%d out of range", blocks, iters);
    *flop = tp::peak_valu_flop(form, blocks, iters);
    const hipError_t e = tp::launch_peak_valu(form, out, blocks, iters, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "VALU launch");
    return TP_OK;
}

tp_status tp_peak_fma(float* out, int32_t blocks, int32_t iters, int64_t* flop, void* stream) {
    return tp_peak_valu(TP_VALU_FMA_F32, out, blocks, iters, flop, stream);
}

tp_status tp_peak_lds(uint32_t* out, int32_t blocks, int32_t iters, int64_t* bytes, void* stream) {
    if (!out || !bytes) return fail(TP_EINVAL, "null argument");
    if (blocks <= 0 || blocks > (1 << 20) || iters <= 0 || iters > (1 << 24))
        return fail(TP_EINVAL, "blocks=%d iters=%d out of range", blocks, iters);
    *bytes = tp::peak_lds_bytes(blocks, iters);
    const hipError_t e = tp::launch_peak_lds(out, blocks, iters, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "LDS launch");
    return TP_OK;
}

}  // extern "C"
