"""Pins of the oracle's Fourier-domain backprojection ("FourierRec", paper
Sections 2.2 and 3: backprojection evaluated with exponentials in the
frequency domain).

The oracle sums, for every voxel and angle, the real trigonometric interpolant
of the padded filtered row at the ray's position.  These tests pin it to
results fixed by other routes: exact interpolation at integer positions, FFT
upsampling at half-integer positions, band-limited rows whose interpolant is a
known cosine, circular-shift invariance, the linear-interpolation oracle where
both interpolants read exact samples, and the disc phantom's density.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2209_08450_amd import synth


def _grid(N):
    iy, ix = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    return ix.ravel(), iy.ravel()


def test_axis_voxel_reads_row_samples_at_any_angle():
    # The voxel on the rotation axis sits at the integer padded position pos0
    # for every angle, where the interpolant equals the stored sample.
    rng = np.random.default_rng(1)
    na, L, N = 7, 32, 16
    y = rng.standard_normal((na, L))
    ang = rng.uniform(0, 2 * math.pi, na)
    pos0 = 13.0
    v = oracle.fourier_backproject_points(y, ang, pos0, N, np.array([N // 2]), np.array([N // 2]), scale=0.75)
    assert abs(v[0] - 0.75 * y[:, 13].sum()) < 1e-12


@pytest.mark.parametrize("theta,axis", [(0.0, "x"), (math.pi / 2, "y")])
def test_single_axis_angle_reads_shifted_samples(theta, axis):
    rng = np.random.default_rng(2)
    L, N = 32, 12
    y = rng.standard_normal((1, L))
    pos0 = 10.0
    ix, iy = _grid(N)
    v = oracle.fourier_backproject_points(y, [theta], pos0, N, ix, iy, scale=1.0)
    c = (ix if axis == "x" else iy) - N // 2
    assert np.max(np.abs(v - y[0, (c + 10)])) < 1e-12


def test_half_integer_positions_match_fft_upsampling():
    # At m + 1/2 the trigonometric interpolant equals the odd samples of the
    # row upsampled by two through a zero-padded spectrum, with the Nyquist
    # coefficient split evenly between +L/2 and -L/2.
    rng = np.random.default_rng(3)
    L, N = 32, 16
    y = rng.standard_normal(L)
    Y = np.fft.fft(y)
    Y2 = np.zeros(2 * L, complex)
    Y2[:L // 2] = Y[:L // 2]
    Y2[2 * L - L // 2 + 1:] = Y[L // 2 + 1:]
    Y2[L // 2] = 0.5 * Y[L // 2]
    Y2[2 * L - L // 2] = 0.5 * Y[L // 2]
    y2 = np.fft.ifft(Y2).real * 2
    pos0 = 9.5
    ix, iy = _grid(N)
    v = oracle.fourier_backproject_points(y[None], [0.0], pos0, N, ix, iy, scale=1.0)
    m2 = (2 * (ix - N // 2 + pos0)).astype(int)  # 2 m, odd
    assert np.max(np.abs(v - y2[m2])) < 1e-12


@pytest.mark.parametrize("k0,phase", [(1, 0.3), (5, -1.1), (11, 2.0), (16, 0.0), (16, 0.9)])
def test_band_limited_rows_give_cosines(k0, phase):
    # A row sampled from cos(2 pi k0 m / L + phase), k0 < L/2, is its own
    # interpolant at every real m; at k0 = L/2 the samples are
    # cos(phase) (-1)^m and the half-weight Nyquist terms give
    # cos(phase) cos(pi m).
    rng = np.random.default_rng(4)
    L, N, na = 32, 14, 9
    ang = rng.uniform(0, math.pi, na)
    m = np.arange(L)
    y = np.stack([np.cos(2 * math.pi * k0 * m / L + phase + 0.2 * a) for a in range(na)])
    pos0 = 15.37
    ix, iy = _grid(N)
    v = oracle.fourier_backproject_points(y, ang, pos0, N, ix, iy, scale=0.5)
    x = ix - N // 2
    yy = iy - N // 2
    ref = np.zeros(ix.shape)
    for a in range(na):
        mm = x * math.cos(ang[a]) + yy * math.sin(ang[a]) + pos0
        ph = phase + 0.2 * a
        if 2 * k0 == L:
            ref += math.cos(ph) * np.cos(math.pi * mm)
        else:
            ref += np.cos(2 * math.pi * k0 * mm / L + ph)
    assert np.max(np.abs(v - 0.5 * ref)) < 1e-11


def test_circular_shift_of_rows_moves_the_axis():
    # Rolling every padded row by one sample and moving pos0 by one leaves the
    # interpolant along each ray unchanged.
    rng = np.random.default_rng(5)
    L, N, na = 32, 12, 5
    y = rng.standard_normal((na, L))
    ang = rng.uniform(0, math.pi, na)
    ix, iy = _grid(N)
    v0 = oracle.fourier_backproject_points(y, ang, 14.3, N, ix, iy)
    v1 = oracle.fourier_backproject_points(np.roll(y, 1, axis=1), ang, 15.3, N, ix, iy)
    assert np.max(np.abs(v0 - v1)) < 1e-12


def test_equals_linear_interpolation_where_both_read_samples():
    # One angle at 0 and an integer axis: every ray lands on a detector
    # sample, where linear and trigonometric interpolation agree; the
    # Fourier FBP then equals the linear-interpolation FBP of the same scan.
    n = 32
    rng = np.random.default_rng(6)
    proj = rng.integers(500, 4000, (1, 3, n)).astype(np.uint16)
    dark = np.full((1, 3, n), 100, np.uint16)
    flat = np.full((1, 3, n), 4100, np.uint16)
    ang = np.array([0.0])
    f_lin = oracle.fbp(proj, dark, flat, ang, n / 2)
    f_fr = oracle.fourier_fbp(proj, dark, flat, ang, n / 2)
    assert np.max(np.abs(f_lin - f_fr)) < 1e-12 * np.max(np.abs(f_lin))


def test_disc_fbp_centre_value():
    # Analytic projections of a uniform disc of density 1: the Fourier FBP is
    # the density inside (to discretisation error) and ~0 outside.
    n = N = 256
    half = n / 2
    ang = synth.uniform_angles(402)
    p = synth.chord_sinogram_np(np.array([[0.0, 0.0, 0.5, 0.5, 0.0, 1.0]]), ang, n, n / 2, half)
    y, off = oracle.filter_rows_padded(p)
    ix = np.concatenate([np.arange(N // 2 - 40, N // 2 + 40, 4), [N // 2 + 100]])
    iy = np.full(ix.shape, N // 2)
    v = oracle.fourier_backproject_points(y, ang, n / 2 + off, N, ix, iy) * half
    assert np.max(np.abs(v[:-1] - 1.0)) < 1e-2
    assert abs(v[-1]) < 1e-2


def test_ellipse_phantom_close_to_linear_interpolation_fbp():
    n = N = 256
    half = n / 2
    ell = synth.ellipses_2d(1)
    ang = synth.uniform_angles(402)
    p = synth.chord_sinogram_np(ell, ang, n, n / 2, half)
    rng = np.random.default_rng(7)
    ix = rng.integers(32, N - 32, 160)
    iy = rng.integers(32, N - 32, 160)
    y, off = oracle.filter_rows_padded(p)
    v = oracle.fourier_backproject_points(y, ang, n / 2 + off, N, ix, iy)
    lin = oracle.backproject_points(oracle.filter_rows(p), ang, n / 2, N, ix, iy)
    assert np.linalg.norm(v - lin) / np.linalg.norm(lin) < 0.05
    img = synth.rasterize_ellipses(ell, N, half)
    assert np.linalg.norm(v * half - img[iy, ix]) / np.linalg.norm(img[iy, ix]) < 0.15


def test_full_slice_helper_matches_points():
    rng = np.random.default_rng(8)
    y = rng.standard_normal((2, 4, 16))
    ang = rng.uniform(0, math.pi, 4)
    f = oracle.fourier_backproject(y, ang, 7.6, 8)
    ix, iy = _grid(8)
    for z in range(2):
        v = oracle.fourier_backproject_points(y[z], ang, 7.6, 8, ix, iy)
        assert np.array_equal(v.reshape(8, 8), f[z])
