"""Pins of the oracle's Shepp-Logan and Parzen windowed ramps.

The paper's tool offers the two windows (command-line interface, Section 2.4;
Parzen for every result of Section 3) without formulas.  The oracle takes
the textbook windows and computes each kernel tap by quadrature.  The pins
below come from elsewhere:

* Shepp-Logan: the classic closed-form kernel 2 / (pi^2 (1 - 4 m^2)) and,
  by telescoping its partial fractions, the exact DC gain of its truncation.
* Parzen: its centre tap integrated by hand (7/160), and the window as a
  scaled cubic B-spline evaluated by scipy's B-spline basis.
* All kinds: the DFT of the truncated kernel samples the continuous response
  up to the truncation tail, and the FFT route equals direct convolution.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import BSpline

import oracle

B3 = BSpline.basis_element([-2.0, -1.0, 0.0, 1.0, 2.0], extrapolate=False)


def _parzen_from_bspline(x):
    """Parzen window = cubic B-spline (4-fold box convolution) scaled to 1 at 0."""
    v = B3(2.0 * np.abs(np.asarray(x, dtype=np.float64)))
    return np.nan_to_num(v, nan=0.0) / B3(0.0)


def _signed_lags(L):
    m = np.arange(L)
    return np.where(m < L // 2, m, m - L)


@pytest.mark.parametrize("L", [16, 64, 512, 4096])
def test_shepp_kernel_is_the_shepp_logan_closed_form(L):
    h = oracle.filter_kernel(L, "shepp")
    m = _signed_lags(L).astype(np.float64)
    want = 2.0 / (math.pi ** 2 * (1.0 - 4.0 * m * m))
    assert np.max(np.abs(h - want)) < 1e-15


@pytest.mark.parametrize("L", [8, 32, 512, 2048])
def test_shepp_dc_gain_by_telescoping(L):
    # 2/(1-4m^2) = 1/(1-2m) + 1/(1+2m); the sum over |m| <= M telescopes to
    # 2/(2M+1).  With M = L/2 - 1 plus the unpaired lag -L/2:
    # H[0] = (2/pi^2) (1/(L-1) - 1/(L^2-1)) = 2L / (pi^2 (L^2 - 1)).
    H = oracle.filter_response(L, "shepp")
    want = 2.0 * L / (math.pi ** 2 * (L * L - 1.0))
    assert abs(H[0] - want) < 1e-15
    # a constant row stays constant under edge padding, so it is scaled by H[0]
    n = L // 2
    for route in (oracle.filter_rows, oracle.filter_rows_direct):
        q = route(np.full((2, n), 3.25), L, kind="shepp")
        assert np.max(np.abs(q - 3.25 * want)) < 1e-13


def test_parzen_center_tap_by_hand():
    # h[0] = 2 int_0^{1/2} w W(2w) dw = (1/2) int_0^1 x W(x) dx
    #      = (1/2) (1/8 - 6/64 + 6/160 + 2 (1/64 - 1/160)) = 7/160.
    for L in (8, 256):
        assert abs(oracle.filter_kernel(L, "parzen")[0] - 7.0 / 160.0) < 1e-16


def test_parzen_window_is_the_scaled_cubic_bspline():
    x = np.linspace(0.0, 1.0, 401)
    got = np.array([oracle.filter_window(v, "parzen") for v in x])
    assert np.max(np.abs(got - _parzen_from_bspline(x))) < 1e-14
    assert oracle.filter_window(1.0, "parzen") == 0.0


def test_shepp_window_at_nyquist():
    assert abs(oracle.filter_window(1.0, "shepp") - 2.0 / math.pi) < 1e-16
    assert oracle.filter_window(0.0, "shepp") == 1.0


def _continuous_response(kind, f):
    f = np.abs(f)
    if kind == "ramp":
        return f
    if kind == "shepp":
        return np.abs(np.sin(math.pi * f)) / math.pi
    return f * _parzen_from_bspline(2.0 * f)


@pytest.mark.parametrize("kind", ["ramp", "shepp", "parzen"])
def test_dft_of_truncated_kernel_samples_the_continuous_response(kind):
    # The infinite Fourier series of h_W is |w| W(2|w|) exactly; cutting it to
    # [-L/2, L/2) leaves an error bounded by the tail sum, <= 2/(pi^2 (L/2 - 1))
    # for kernels decaying like 1/(pi^2 m^2) or faster.
    L = 2048
    H = oracle.filter_response(L, kind)
    k = np.arange(L)
    f = np.where(k <= L // 2, k, k - L) / L
    tail = 2.0 / (math.pi ** 2 * (L / 2 - 1))
    err = np.abs(H - _continuous_response(kind, f))
    assert np.max(err) < tail
    assert np.allclose(H[1:], H[:0:-1], atol=1e-16)  # even
    # the windows change the response by far more than that bound
    if kind != "ramp":
        assert np.max(np.abs(H - oracle.ramp_response(L))) > 100 * tail


@pytest.mark.parametrize("kind", ["shepp", "parzen"])
@pytest.mark.parametrize("n", [5, 12, 33])
def test_windowed_fft_route_equals_direct_convolution(kind, n):
    rng = np.random.default_rng(100 + n)
    p = rng.standard_normal((3, n))
    a = oracle.filter_rows(p, kind=kind)
    b = oracle.filter_rows_direct(p, kind=kind)
    assert np.max(np.abs(a - b)) < 1e-13


def test_unknown_filter_is_rejected():
    with pytest.raises(ValueError):
        oracle.filter_kernel(64, "hann")
    with pytest.raises(ValueError):
        oracle.filter_window(0.3, "hann")
