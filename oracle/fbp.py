"""FP64 reference implementation of the FBP hot path (TEST INFRASTRUCTURE ONLY).

Only tests, the smoke check and the benchmark's CPU-baseline leg may use this
module.  It never imports the product package.

Notation (paper, Section 2.2): raw projections P[a][z][j] (angle a, detector
row z, detector column j), dark frames, flat frames, N_theta angles theta_a,
rotation axis ``center`` in detector pixels.  The readings taken where the
paper is silent are listed in each docstring.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

MIN_TRANSMISSION = 1e-6
"""Lower clamp of the transmission before the logarithm (the paper is silent
on photon-starved pixels; reading: clamp at 1e-6, so p <= -ln(1e-6))."""

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build_oracle
            build_oracle()
        lib = ctypes.CDLL(_LIB_PATH)
        d = ctypes.c_double
        i64 = ctypes.c_int64
        pd = ctypes.POINTER(ctypes.c_double)
        pi = ctypes.POINTER(ctypes.c_int64)
        i32 = ctypes.c_int
        lib.oracle_backproject.argtypes = [pd, i64, i64, i64, pd, d, i64, d, i32, pd]
        lib.oracle_backproject.restype = None
        lib.oracle_backproject_points.argtypes = [pd, i64, i64, pd, d, i64, d, i32, pi, pi, i64, pd]
        lib.oracle_backproject_points.restype = None
        lib.oracle_radon.argtypes = [pd, i64, i64, pd, d, i64, i64, pd]
        lib.oracle_radon.restype = None
        lib.oracle_fourier_backproject_points.argtypes = [pd, pd, i64, i64, pd, d, i64, d, pi, pi, i64, pd]
        lib.oracle_fourier_backproject_points.restype = None
        lib.oracle_lamino_backproject_points.argtypes = [pd, i64, i64, i64, pd, d, d, d, i64, i64, d, pi, pi, pi,
                                                          i64, pd]
        lib.oracle_lamino_backproject_points.restype = None
        lib.oracle_round_binary16.argtypes = [d]
        lib.oracle_round_binary16.restype = d
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_num_threads.restype = None
        _lib = lib
    return _lib


def _pd(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pi(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def num_threads() -> int:
    """Threads the C part of the oracle uses (OpenMP)."""
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))


# --------------------------------------------------------------------------
# Step 1: dark/flat correction and negative logarithm (Section 2.2).
# --------------------------------------------------------------------------
def dark_flat_mean(dark: np.ndarray, flat: np.ndarray):
    """Per-pixel arithmetic mean of the dark and flat frame stacks.

    dark: [n_dark][nz][n], flat: [n_flat][nz][n] (any integer type).
    Reading: the paper says only "dark-flat field correction"; the frames are
    averaged with the arithmetic mean.
    """
    d = np.asarray(dark, dtype=np.float64).mean(axis=0)
    f = np.asarray(flat, dtype=np.float64).mean(axis=0)
    return d, f


def normalize(proj: np.ndarray, dark: np.ndarray, flat: np.ndarray) -> np.ndarray:
    """p = -ln( max( (P - D) / max(F - D, 1), 1e-6 ) ), returned sinogram-major.

    proj: [n_angles][nz][n] raw counts (projection-major, as recorded).
    Returns p: [nz][n_angles][n] float64.
    Readings: natural logarithm; a dead pixel (F - D <= 0) uses a denominator
    of one count; photon starvation clamps the transmission at 1e-6.
    """
    d, f = dark_flat_mean(dark, flat)
    P = np.asarray(proj, dtype=np.float64)
    den = np.maximum(f - d, 1.0)
    t = (P - d[None, :, :]) / den[None, :, :]
    t = np.maximum(t, MIN_TRANSMISSION)
    p = -np.log(t)
    return np.ascontiguousarray(p.transpose(1, 0, 2))


# --------------------------------------------------------------------------
# Step 2: padded ramp filter along detector rows (Section 2.2).
# --------------------------------------------------------------------------
def pad_len(n: int) -> int:
    """Padded row length: the power of two at or above 2 n.

    Reading: the paper pads 16-bit data to powers of two; this build uses the
    same power-of-two length for every storage type.
    """
    return 1 << int(math.ceil(math.log2(2 * n)))


def ramp_kernel(L: int) -> np.ndarray:
    """Band-limited ramp h[m] = integral over |w| <= 1/2 of |w| exp(2 pi i w m) dw.

    Closed form: h[0] = 1/4, h[m] = -1/(pi^2 m^2) for odd m, 0 for even m != 0,
    for m in [-L/2, L/2).  Returned in FFT order (index m mod L).
    Reading: the paper names Shepp-Logan and Parzen windows but defines no
    filter; the plain band-limited ramp (cycles per pixel) is used.
    """
    m = np.arange(L, dtype=np.int64)
    m = np.where(m < L // 2, m, m - L)  # signed lag
    h = np.zeros(L, dtype=np.float64)
    h[m == 0] = 0.25
    odd = (m % 2) != 0
    h[odd] = -1.0 / (math.pi ** 2 * m[odd].astype(np.float64) ** 2)
    return h


def ramp_response(L: int) -> np.ndarray:
    """H[k] = sum_m h[m] exp(-2 pi i k m / L), real and even (FFT of ``ramp_kernel``)."""
    return np.fft.fft(ramp_kernel(L)).real


FILTERS = ("ramp", "shepp", "parzen")
"""Filter windows: the paper's tool offers Shepp-Logan and Parzen (its default,
used for every measurement in Section 3); plain ramp is the unwindowed case."""


def filter_window(x: float, kind: str) -> float:
    """Window W(x) on the ramp, x = |w| / (1/2) in [0, 1] (w in cycles per pixel).

    Reading: the paper names the windows but gives no formula; the textbook
    forms are taken.
      ramp:   W = 1.
      shepp:  W = sinc(x/2) = sin(pi x/2) / (pi x/2), so |w| W = |sin(pi w)| / pi,
              the response of the Shepp-Logan kernel.
      parzen: W = 1 - 6x^2 + 6|x|^3 for x <= 1/2, 2 (1 - x)^3 for 1/2 < x <= 1
              (the Parzen / de la Vallee Poussin window, zero at Nyquist).
    """
    x = abs(float(x))
    if kind == "ramp":
        return 1.0
    if kind == "shepp":
        return 1.0 if x == 0.0 else math.sin(0.5 * math.pi * x) / (0.5 * math.pi * x)
    if kind == "parzen":
        if x <= 0.5:
            return 1.0 - 6.0 * x * x + 6.0 * x ** 3
        return 2.0 * (1.0 - x) ** 3 if x <= 1.0 else 0.0
    raise ValueError(f"unknown filter {kind!r}")


_WINDOW_KNOTS = {"ramp": (), "shepp": (), "parzen": (0.5,)}
_kernel_cache: dict = {}


def filter_kernel(L: int, kind: str = "ramp") -> np.ndarray:
    """Windowed band-limited ramp h_W[m] = integral over |w| <= 1/2 of
    |w| W(2|w|) exp(2 pi i w m) dw, for m in [-L/2, L/2), FFT order.

    ramp: the closed form of ``ramp_kernel``.  Windowed kinds:
    h_W[m] = 2 * integral_0^{1/2} w W(2w) cos(2 pi m w) dw by QUADPACK's
    rule for cosine-weighted integrands (scipy.integrate.quad, weight='cos'),
    once per smooth piece of the window.
    """
    if kind == "ramp":
        return ramp_kernel(L)
    if kind not in FILTERS:
        raise ValueError(f"unknown filter {kind!r}")
    key = (int(L), kind)
    if key not in _kernel_cache:
        import warnings

        from scipy import integrate

        edges = [0.0] + [0.5 * k for k in _WINDOW_KNOTS[kind]] + [0.5]
        f = lambda w: w * filter_window(2.0 * w, kind)  # noqa: E731
        half = np.empty(L // 2 + 1, dtype=np.float64)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", integrate.IntegrationWarning)
            for m in range(L // 2 + 1):
                tot = 0.0
                for a, b in zip(edges[:-1], edges[1:]):
                    if m == 0:
                        v, _ = integrate.quad(f, a, b, epsabs=1e-17, epsrel=1e-13, limit=200)
                    else:
                        v, _ = integrate.quad(f, a, b, weight="cos", wvar=2.0 * math.pi * m, epsabs=1e-17,
                                              epsrel=1e-13, limit=200)
                    tot += v
                half[m] = 2.0 * tot
        m = np.arange(L, dtype=np.int64)
        m = np.where(m < L // 2, m, m - L)
        _kernel_cache[key] = half[np.abs(m)]
    return _kernel_cache[key].copy()


def filter_response(L: int, kind: str = "ramp") -> np.ndarray:
    """H_W[k] = sum_m h_W[m] exp(-2 pi i k m / L) (FFT of ``filter_kernel``), real."""
    return np.fft.fft(filter_kernel(L, kind)).real


def pad_rows(p: np.ndarray, L: int):
    """Edge-replicating pad of the last axis from n to L, data at offset floor((L-n)/2).

    Returns (u, off).  Reading: the paper pads before filtering to suppress
    artefacts from matter outside the field of view, which implies a
    non-zero (edge) pad rather than zeros.
    """
    n = p.shape[-1]
    off = (L - n) // 2
    u = np.empty(p.shape[:-1] + (L,), dtype=np.float64)
    u[..., off:off + n] = p
    u[..., :off] = p[..., :1]
    u[..., off + n:] = p[..., -1:]
    return u, off


def filter_rows(p: np.ndarray, L: int | None = None, kind: str = "ramp") -> np.ndarray:
    """q = crop( IFFT( H_W * FFT( pad(p) ) ) ) along the last axis, FP64."""
    n = p.shape[-1]
    L = pad_len(n) if L is None else L
    u, off = pad_rows(np.asarray(p, dtype=np.float64), L)
    H = filter_response(L, kind)
    y = np.fft.ifft(np.fft.fft(u, axis=-1) * H, axis=-1).real
    return np.ascontiguousarray(y[..., off:off + n])


def filter_rows_direct(p: np.ndarray, L: int | None = None, kind: str = "ramp") -> np.ndarray:
    """Same result as ``filter_rows`` by direct circular convolution with h.

    y[off + j] = sum_k u[k] h[(off + j - k) mod L]; O(n L) per row, for small
    sizes only.  Independent of the FFT route (used as its pin).
    """
    n = p.shape[-1]
    L = pad_len(n) if L is None else L
    u, off = pad_rows(np.asarray(p, dtype=np.float64), L)
    h = filter_kernel(L, kind)
    k = np.arange(L)
    out = np.empty(p.shape[:-1] + (n,), dtype=np.float64)
    for j in range(n):
        out[..., j] = u @ h[(off + j - k) % L]
    return out


# --------------------------------------------------------------------------
# Storage rounding (Section 2.1: 16-bit storage, 32-bit arithmetic).
# --------------------------------------------------------------------------
def round_f16(x: np.ndarray) -> np.ndarray:
    """Round to IEEE binary16 with round-to-nearest-even (numpy's conversion)."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float16).astype(np.float64)


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to bfloat16 with round-to-nearest-even (finite inputs).

    bfloat16 keeps the upper 16 bits of an IEEE binary32; rounding adds
    0x7FFF plus the lowest kept bit before truncation.
    """
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# Step 3: backprojection with linear interpolation (LineRec) and its transpose.
# --------------------------------------------------------------------------
def _w16(weights) -> int:
    if weights in (None, "f64"):
        return 0
    if weights == "f16":
        return 1
    raise ValueError(weights)


def round_binary16(x: float) -> float:
    """Nearest IEEE binary16 value of x (ties to even), as the C oracle rounds
    the interpolation weights of the 16-bit mode."""
    return float(_load().oracle_round_binary16(float(x)))


def backproject(q: np.ndarray, angles, center: float, N: int, scale: float | None = None,
                weights: str | None = None) -> np.ndarray:
    """f[z][iy][ix] = scale * sum_a ((1-w) Q(j0) + w Q(j0+1)), FP64 (C loop).

    q: [nz][n_angles][n]; voxel centres x = ix - N//2, y = iy - N//2 (ix fast);
    s = x cos + y sin + center; taps off the detector read zero.
    scale defaults to pi / n_angles (uniform 180-degree scan).
    ``weights='f16'``: the 16-bit mode (Section 2.1) -- (1-w) and w each
    rounded to the nearest binary16 value before the FP64 products.
    """
    q = np.ascontiguousarray(q, dtype=np.float64)
    if q.ndim == 2:
        q = q[None]
    nz, na, n = q.shape
    ang = np.ascontiguousarray(angles, dtype=np.float64)
    assert ang.shape == (na,)
    if scale is None:
        scale = math.pi / na
    f = np.empty((nz, N, N), dtype=np.float64)
    _load().oracle_backproject(_pd(q), nz, na, n, _pd(ang), float(center), N, float(scale), _w16(weights), _pd(f))
    return f


def backproject_points(q: np.ndarray, angles, center: float, N: int, ix, iy,
                       scale: float | None = None, weights: str | None = None) -> np.ndarray:
    """Backprojection of one slice q: [n_angles][n] at voxels (ix[k], iy[k]);
    ``weights`` as for ``backproject``."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    na, n = q.shape
    ang = np.ascontiguousarray(angles, dtype=np.float64)
    ix = np.ascontiguousarray(ix, dtype=np.int64)
    iy = np.ascontiguousarray(iy, dtype=np.int64)
    if scale is None:
        scale = math.pi / na
    out = np.empty(ix.shape[0], dtype=np.float64)
    _load().oracle_backproject_points(_pd(q), na, n, _pd(ang), float(center), N, float(scale), _w16(weights),
                                      _pi(ix), _pi(iy), ix.shape[0], _pd(out))
    return out


def radon(f: np.ndarray, angles, center: float, n: int) -> np.ndarray:
    """(R f)[z][a][j] = sum over voxels of f * ((1-w)[j0 = j] + w[j0 + 1 = j]).

    The transpose of ``backproject`` with scale 1 (voxel-driven scatter of the
    same hat weights).  f: [nz][N][N] -> [nz][n_angles][n].
    Reading: the paper defines no forward projector; the exact transpose of
    the linear-interpolation backprojector is used.
    """
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.ndim == 2:
        f = f[None]
    nz, N, N2 = f.shape
    assert N == N2
    ang = np.ascontiguousarray(angles, dtype=np.float64)
    na = ang.shape[0]
    out = np.empty((nz, na, n), dtype=np.float64)
    _load().oracle_radon(_pd(f), nz, N, _pd(ang), float(center), na, n, _pd(out))
    return out


# --------------------------------------------------------------------------
# The composition.
# --------------------------------------------------------------------------
def _storage_weights(storage):
    """Interpolation weights of each storage mode: binary16 in the 16-bit mode."""
    return "f16" if storage == "f16" else None


def _round_storage(x, storage):
    if storage in (None, "f32"):
        return x
    if storage == "f16":
        return round_f16(x)
    if storage == "bf16":
        return round_bf16(x)
    raise ValueError(storage)


def fbp(proj, dark, flat, angles, center: float, N: int | None = None, storage: str | None = None,
        kind: str = "ramp"):
    """FBP = backproject(filter(normalize(raw))), FP64, scale pi / n_angles.

    ``storage`` in {None/'f32', 'f16', 'bf16'} rounds the filtered rows to that
    type before backprojection (emulates reduced-precision storage with
    arithmetic kept in higher precision); 'f16' is the 16-bit mode and also
    holds the interpolation weights in binary16 (``backproject``).  'f32'
    applies no rounding: the FP32 GPU path is compared against the unrounded
    FP64 result.  ``kind`` picks the filter window (``FILTERS``).
    """
    p = normalize(proj, dark, flat)
    n = p.shape[-1]
    q = filter_rows(p, kind=kind)
    q = _round_storage(q, storage)
    return backproject(q, angles, center, n if N is None else N, weights=_storage_weights(storage))


def fbp_points(proj_slice, dark_slice, flat_slice, angles, center, N, ix, iy, storage=None, kind="ramp"):
    """FBP of one slice at listed voxels.

    proj_slice: [n_angles][n] raw counts of one detector row;
    dark_slice/flat_slice: [n_frames][n].
    """
    p = normalize(np.asarray(proj_slice)[:, None, :], np.asarray(dark_slice)[:, None, :],
                  np.asarray(flat_slice)[:, None, :])[0]
    q = _round_storage(filter_rows(p, kind=kind), storage)
    return backproject_points(q, angles, center, N, ix, iy, weights=_storage_weights(storage))


# --------------------------------------------------------------------------
# Fourier-domain backprojection (FourierRec).
# --------------------------------------------------------------------------
def filter_rows_padded(p: np.ndarray, L: int | None = None, kind: str = "ramp"):
    """Uncropped filtered rows y = IFFT(H_W * FFT(pad(p))), FP64: returns (y, off)."""
    n = p.shape[-1]
    L = pad_len(n) if L is None else L
    u, off = pad_rows(np.asarray(p, dtype=np.float64), L)
    y = np.fft.ifft(np.fft.fft(u, axis=-1) * filter_response(L, kind), axis=-1).real
    return y, off


def fourier_backproject_points(y: np.ndarray, angles, pos0: float, N: int, ix, iy,
                               scale: float | None = None) -> np.ndarray:
    """Backprojection of one slice's padded rows y: [n_angles][L] with the
    trigonometric interpolant of each row, at voxels (ix[k], iy[k]).

    f(x, y) = scale * sum_a y_a(x cos + y sin + pos0), where y_a(m) is the real
    trigonometric interpolant of row a (both Nyquist terms at half weight), so
    y_a(m) = y[a][m] at integer m.  pos0 is the padded-row position of the
    rotation axis (centre + pad offset).  Readings: the paper names the method
    (Fourier-based backprojection with exponential interpolation kernels in
    the frequency domain, Sections 2.2 and 3) without formulas; this is the
    sum such a method approximates, evaluated directly (FP64 C loop).
    """
    y = np.ascontiguousarray(y, dtype=np.float64)
    na, L = y.shape
    Y = np.fft.fft(y, axis=-1)
    yre = np.ascontiguousarray(Y.real)
    yim = np.ascontiguousarray(Y.imag)
    ang = np.ascontiguousarray(angles, dtype=np.float64)
    assert ang.shape == (na,)
    ix = np.ascontiguousarray(ix, dtype=np.int64)
    iy = np.ascontiguousarray(iy, dtype=np.int64)
    if scale is None:
        scale = math.pi / na
    out = np.empty(ix.shape[0], dtype=np.float64)
    _load().oracle_fourier_backproject_points(_pd(yre), _pd(yim), na, L, _pd(ang), float(pos0), N,
                                              float(scale), _pi(ix), _pi(iy), ix.shape[0], _pd(out))
    return out


def fourier_backproject(y: np.ndarray, angles, pos0: float, N: int, scale: float | None = None) -> np.ndarray:
    """``fourier_backproject_points`` at every voxel of each slice: y [nz][n_angles][L] -> [nz][N][N]."""
    y = np.asarray(y, dtype=np.float64)
    if y.ndim == 2:
        y = y[None]
    iy, ix = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ix = ix.ravel()
    iy = iy.ravel()
    return np.stack([fourier_backproject_points(y[z], angles, pos0, N, ix, iy, scale).reshape(N, N)
                     for z in range(y.shape[0])])


def fourier_fbp(proj, dark, flat, angles, center: float, N: int | None = None, kind: str = "ramp"):
    """FourierRec FBP: normalise, pad, filter, then ``fourier_backproject``
    with pos0 = center + pad offset; scale pi / n_angles."""
    p = normalize(proj, dark, flat)
    n = p.shape[-1]
    y, off = filter_rows_padded(p, kind=kind)
    return fourier_backproject(y, angles, center + off, n if N is None else N)


def fourier_fbp_points(proj_slice, dark_slice, flat_slice, angles, center, N, ix, iy, kind="ramp"):
    """FourierRec FBP of one slice at listed voxels (raw counts of one detector row)."""
    p = normalize(np.asarray(proj_slice)[:, None, :], np.asarray(dark_slice)[:, None, :],
                  np.asarray(flat_slice)[:, None, :])[0]
    y, off = filter_rows_padded(p, kind=kind)
    return fourier_backproject_points(y, angles, center + off, N, ix, iy)


# --------------------------------------------------------------------------
# Laminographic backprojection.
# --------------------------------------------------------------------------
def lamino_backproject_points(q: np.ndarray, angles, center_u: float, center_v: float, phi: float, N: int, Nz: int,
                              ix, iy, iz, scale: float | None = None) -> np.ndarray:
    """Laminographic backprojection of filtered projections q [n_angles][rows][n]
    at voxels (ix, iy, iz), FP64 (C loop).

    Reading of the geometry (the paper names laminography as a use of the
    direct backprojector without defining it): the rotation axis is tilted by
    phi from the beam (phi = pi/2 is tomography); voxel (x, y, z) is seen at
    column u = x cos + y sin + center_u and row
    v = (-x sin + y cos) cos(phi) + z sin(phi) + center_v, bilinear
    interpolation, zero off the detector; x = ix - N//2, y = iy - N//2,
    z = iz - Nz//2; scale defaults to pi / n_angles.
    """
    q = np.ascontiguousarray(q, dtype=np.float64)
    na, rows, n = q.shape
    ang = np.ascontiguousarray(angles, dtype=np.float64)
    assert ang.shape == (na,)
    ix = np.ascontiguousarray(ix, dtype=np.int64)
    iy = np.ascontiguousarray(iy, dtype=np.int64)
    iz = np.ascontiguousarray(iz, dtype=np.int64)
    if scale is None:
        scale = math.pi / na
    out = np.empty(ix.shape[0], dtype=np.float64)
    _load().oracle_lamino_backproject_points(_pd(q), na, rows, n, _pd(ang), float(center_u), float(center_v),
                                             float(phi), N, Nz, float(scale), _pi(ix), _pi(iy), _pi(iz),
                                             ix.shape[0], _pd(out))
    return out


def lamino_backproject(q: np.ndarray, angles, center_u: float, center_v: float, phi: float, N: int, Nz: int,
                       scale: float | None = None) -> np.ndarray:
    """``lamino_backproject_points`` at every voxel: -> [Nz][N][N]."""
    iz, iy, ix = np.meshgrid(np.arange(Nz), np.arange(N), np.arange(N), indexing="ij")
    v = lamino_backproject_points(q, angles, center_u, center_v, phi, N, Nz, ix.ravel(), iy.ravel(), iz.ravel(),
                                  scale)
    return v.reshape(Nz, N, N)


# --------------------------------------------------------------------------
# Least squares with the projector pair.
# --------------------------------------------------------------------------
def power_lambda_max(angles, center, N, n, iters: int = 30, seed: int = 0) -> float:
    """Largest eigenvalue of R^T R by power iteration from a seeded start (FP64)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((1, N, N))
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = backproject(radon(x, angles, center, n), angles, center, N, scale=1.0)
        lam = float(np.vdot(x, y))
        x = y / np.linalg.norm(y)
    return lam


def ls_gradient(x, y, angles, center):
    """Gradient of ||R x - y||^2: 2 R^T (R x - y)."""
    N = x.shape[-1]
    n = y.shape[-1]
    r = radon(x, angles, center, n) - y
    return 2.0 * backproject(r, angles, center, N, scale=1.0)


def ls_solve(y, angles, center, N, steps: int, eta: float, x0=None):
    """Gradient descent x_{k+1} = x_k - eta * 2 R^T (R x_k - y), x_0 = 0.

    Returns (x, losses) with losses[k] = ||R x_k - y||^2 before step k.
    Reading: the paper has no iterative solver; this plain gradient method
    with step eta = 1/(2 lambda_max(R^T R)) is the least-squares form used.
    """
    y = np.asarray(y, dtype=np.float64)
    if y.ndim == 2:
        y = y[None]
    x = np.zeros((y.shape[0], N, N)) if x0 is None else np.array(x0, dtype=np.float64)
    n = y.shape[-1]
    losses = []
    for _ in range(steps):
        r = radon(x, angles, center, n) - y
        losses.append(float(np.sum(r * r)))
        x = x - eta * 2.0 * backproject(r, angles, center, N, scale=1.0)
    return x, losses
