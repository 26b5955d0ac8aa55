"""Pins of the oracle's padded ramp filter (paper, Section 2.2).

The paper defines no filter formula; the ramp is the band-limited |w| in
cycles per pixel.  The pins here do not reuse the oracle's formulas: the
kernel is checked by numerical quadrature, the FFT route by direct
convolution, the DC gain by an independent tail series (stored in
tests/golden), and the scale by the analytic result for a uniform disc.
"""
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from paper_2209_08450_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_pad_len_power_of_two_at_least_twice():
    for n, L in [(1, 2), (2, 4), (3, 8), (12, 32), (256, 512), (1000, 2048), (1024, 2048),
                 (2048, 4096), (4096, 8192)]:
        assert oracle.pad_len(n) == L


@pytest.mark.parametrize("m", [0, 1, 2, 3, 4, 7, 10, 31])
def test_ramp_kernel_matches_quadrature(m):
    L = 64
    h = oracle.ramp_kernel(L)
    v = quad(lambda w: abs(w) * math.cos(2 * math.pi * w * m), -0.5, 0.5, limit=400,
             points=[0.0])[0]
    assert abs(h[m] - v) < 1e-12
    assert abs(h[(-m) % L] - v) < 1e-12  # even


def test_ramp_response_real_even_and_dc_gain_golden():
    table = np.loadtxt(os.path.join(GOLDEN, "ramp_dc_gain.txt"), comments="#")
    for L, h0 in table:
        H = oracle.ramp_response(int(L))
        assert abs(H[0] - h0) < 1e-15 + 1e-11 * abs(h0)
        assert np.allclose(H[1:], H[:0:-1], atol=1e-15)  # even


def test_ramp_response_approaches_abs_frequency():
    # H[k] -> |k| / L for k away from 0 and from Nyquist (aliasing of the
    # band-limited ramp is O(1/L)).
    L = 1024
    H = oracle.ramp_response(L)
    k = np.arange(16, L // 2 - 16)
    assert np.max(np.abs(H[k] - k / L)) < 2.0 / L


@pytest.mark.parametrize("n", [5, 12, 33, 64])
def test_fft_route_equals_direct_convolution(n):
    rng = np.random.default_rng(n)
    p = rng.standard_normal((3, n))
    a = oracle.filter_rows(p)
    b = oracle.filter_rows_direct(p)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_constant_row_is_scaled_by_dc_gain():
    L = 4096
    h0 = dict(np.loadtxt(os.path.join(GOLDEN, "ramp_dc_gain.txt"), comments="#"))[float(L)]
    q = oracle.filter_rows(np.full((2, 2048), 3.5))
    assert np.max(np.abs(q - 3.5 * h0)) < 1e-12
    # about 2 / (pi^2 L): 4.947e-5 at L = 4096
    assert abs(h0 - 4.947e-5) < 1e-8


def test_disc_projection_filters_to_constant():
    # A uniform disc of radius R px and density mu per px projects to
    # 2 mu sqrt(R^2 - s^2); its ramp-filtered projection is mu / pi for |s| < R.
    n, R, mu = 512, 100.0, 1.0
    center = n / 2
    p = synth.chord_sinogram_np(np.array([[0, 0, R / (n / 2), R / (n / 2), 0.0, mu]]),
                                np.array([0.0]), n, center, n / 2) * (n / 2)
    q = oracle.filter_rows(p)[0]
    s = np.arange(n) - center
    # sampling the sqrt edge rings with an alternating error that decays
    # roughly like d^-1.8 with the distance d from the edge: 8e-4 at d = 32
    inside = np.abs(s) < R - 32
    assert np.max(np.abs(q[inside] - mu / math.pi)) < 1e-3
    # outside: (mu/pi)(1 - |s| / sqrt(s^2 - R^2)), away from the edge
    out = (np.abs(s) > R + 32) & (np.abs(s) < n / 2 - 8)
    want = (mu / math.pi) * (1 - np.abs(s[out]) / np.sqrt(s[out] ** 2 - R * R))
    assert np.max(np.abs(q[out] - want)) < 1e-3


def test_edge_padding_keeps_linear_ramp_interior():
    # The ramp filter annihilates linear functions in the continuum; with edge
    # padding only the boundary layer differs.  Check linearity instead:
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal((2, 4, 40))
    assert np.allclose(oracle.filter_rows(2 * a - 3 * b),
                       2 * oracle.filter_rows(a) - 3 * oracle.filter_rows(b), atol=1e-12)


def test_storage_rounding_matches_torch_conversions():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = rng.standard_normal(10000) * np.exp(rng.uniform(-8, 8, 10000))
    x = x.astype(np.float32).astype(np.float64)
    t = torch.from_numpy(x.astype(np.float32))
    assert np.array_equal(oracle.round_bf16(x), t.to(torch.bfloat16).to(torch.float64).numpy())
    assert np.array_equal(oracle.round_f16(x), t.to(torch.float16).to(torch.float64).numpy())
