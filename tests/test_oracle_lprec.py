"""Pins of the log-polar backprojection oracle (oracle/lprec.py): each step
against an independent computation, and the whole method against the direct
sum of trigonometric interpolants it approximates."""
import math

import numpy as np
import pytest

import oracle
from oracle import lprec as lp
from paper_2209_08450_amd import synth


def _bandlimited_rows(seed, na, L, kmax):
    """Random real rows whose spectra vanish beyond |k| = kmax."""
    rng = np.random.default_rng(seed)
    Y = np.zeros((na, L), dtype=complex)
    Y[:, 1:kmax] = rng.standard_normal((na, kmax - 1)) + 1j * rng.standard_normal((na, kmax - 1))
    Y[:, 0] = rng.standard_normal(na)
    Y[:, L - kmax + 1:] = np.conj(Y[:, 1:kmax][:, ::-1])
    return np.fft.ifft(Y, axis=-1).real * L


@pytest.mark.parametrize("na,N,spans,os,eps", [(64, 64, 3, 1.0, 0.5), (180, 256, 3, 1.2, 0.5),
                                                (100, 48, 2, 1.0, 0.3), (2048, 2048, 3, 1.2, 0.5),
                                                (37, 33, 5, 2.0, 1.0)])
def test_params_meet_their_constraints(na, N, spans, os, eps):
    pr = lp.lprec_params(na, N, spans, os, eps)
    for k in ("Ns", "NA", "M"):
        assert pr[k] & (pr[k] - 1) == 0, k
    assert lp.MIN_FFT <= pr["Ns"] and lp.MIN_FFT <= pr["NA"]
    # resolution: both grid steps at most 1 / (os * s_max) at the far edge
    assert pr["delta"] * pr["s_max"] * os <= 1.0 + 1e-12
    assert pr["dpsi"] * pr["s_max"] * os <= 1.0 + 1e-12
    # the data range [log s_min, log s_max] maps onto [margin, Ns - 1 - margin]
    j_min = (math.log(pr["s_min"]) - pr["sigma0"]) / pr["delta"]
    j_max = (math.log(pr["s_max"]) - pr["sigma0"]) / pr["delta"]
    assert abs(j_min - lp.SIGMA_MARGIN) < 1e-9 and abs(j_max - (pr["Ns"] - 1 - lp.SIGMA_MARGIN)) < 1e-6
    assert abs(pr["s_min"] - eps * pr["R"]) < 1e-9 * pr["R"]
    # linear convolution fits: NA >= rows + M (n_span - 1); the kernel stays below 90 degrees
    assert pr["NA"] >= pr["rows"] + pr["M"] * (pr["n_span"] - 1)
    assert abs(pr["d_lo"] * pr["dpsi"]) < math.pi / 2
    assert abs((pr["d_lo"] + pr["D"] - 1) * pr["dpsi"]) < math.pi / 2
    assert pr["n_span"] * spans >= na > (pr["n_span"] - 1) * spans


@pytest.mark.parametrize("spans,eps", [(3, 0.5), (2, 0.3), (4, 1.0)])
def test_every_ray_offset_is_at_least_eps_R(spans, eps):
    """Brute force over voxels and slot angles: the shifted ray offset of every
    voxel centre is >= s_min = eps R (so log s is defined on the image)."""
    na, N = 90, 40
    pr = lp.lprec_params(na, N, spans, 1.0, eps)
    iy, ix = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    x = ix.ravel() - N // 2
    y = iy.ravel() - N // 2
    for p in range(spans):
        beta, slots = lp.span_angles(pr, 0.0, p)
        xp = math.cos(beta) * x + math.sin(beta) * y + pr["a0"]
        yp = -math.sin(beta) * x + math.cos(beta) * y
        for k in range(pr["n_span"]):
            phi = (k - 0.5 * (pr["n_span"] - 1)) * pr["dtheta"]
            s = xp * math.cos(phi) + yp * math.sin(phi)
            assert s.min() >= pr["s_min"] - 1e-9
            # and equals the ray offset through the unshifted frame plus a0 cos(phi)
            th = beta + phi
            assert np.allclose(s - pr["a0"] * math.cos(phi), x * math.cos(th) + y * math.sin(th), atol=1e-9)


def test_bspline_weights_closed_forms():
    """Centred B-spline samples (quintic 66/26/1 over 120, cubic 4/1 over 6),
    partition of unity, reproduction of x, and the sampled transforms."""
    for deg, samples in [(5, {0: 66 / 120, 1: 26 / 120, 2: 1 / 120}), (3, {0: 4 / 6, 1: 1 / 6})]:
        offs, ws = lp.bspline_weights(np.array([0.0]), deg)
        for o, w in zip(offs, ws):
            assert abs(w[0] - samples.get(abs(o), 0.0)) < 1e-15
        t = np.linspace(0.0, 0.999, 37)
        offs, ws = lp.bspline_weights(t, deg)
        assert np.allclose(sum(ws), 1.0, atol=1e-14)
        # sum_i i beta(t - i) = t (B-splines reproduce linear functions)
        assert np.allclose(sum(o * w for o, w in zip(offs, ws)), t, atol=1e-14)
        n = 32
        k = np.arange(n)
        direct = sum(samples.get(abs(m), 0.0) * np.exp(-2j * np.pi * k * m / n) for m in range(-3, 4))
        assert np.allclose(lp.bspline_hat(k, n, deg), direct.real, atol=1e-15)
        assert np.allclose(direct.imag, 0.0, atol=1e-15)


def test_row_splines_reproduce_the_trigonometric_interpolant():
    """Step 1: the periodic spline at even half-sample positions is the row; at
    odd ones it is the trigonometric interpolant at m + 1/2, summed directly."""
    rng = np.random.default_rng(3)
    L = 64
    y = rng.standard_normal((3, L))
    c = lp.row_splines(y)
    m = np.arange(L)
    Y = np.fft.fft(y, axis=-1)
    k = np.arange(L)
    ks = np.where(k < L // 2, k, k - L)
    w = np.where(np.abs(ks) == L // 2, 0.5, 1.0)
    for a in range(3):
        even = lp.spline_eval_periodic(c[a], 2.0 * m)
        assert np.max(np.abs(even - y[a])) < 1e-12
        odd = lp.spline_eval_periodic(c[a], 2.0 * m + 1.0)
        # Nyquist term at half weight on both signs: w cos(pi (m + 1/2)) = 0 there
        direct = np.array([np.sum(w * (Y[a] * np.exp(2j * np.pi * ks * (mm + 0.5) / L)).real) / L for mm in m])
        assert np.max(np.abs(odd - direct)) < 1e-12


def test_convolution_step_equals_direct_sum_at_grid_nodes():
    """Steps 5-6: the spline of F_p evaluated at log-polar grid nodes equals
    dtheta sum_k G~_k(sigma_j + log cos(psi_m - phi_k)), with G~_k the
    trigonometric interpolant of the tapered samples, summed directly."""
    na, N = 40, 24
    pr = lp.lprec_params(na, N, 3, 1.0, 0.5)
    y = _bandlimited_rows(5, na, 64, 20)
    c_rows = lp.row_splines(y)
    beta, slots = lp.span_angles(pr, 0.1, 1)
    G = lp.log_radial_samples(c_rows, pr, slots, 30.0)
    C = lp.span_coefficients(G, pr)
    Ns = pr["Ns"]
    Gh = np.fft.fft(G, axis=-1)
    eta = np.fft.fftfreq(Ns) * Ns
    rng = np.random.default_rng(1)
    # nodes inside the image sector and the rho window
    rows = rng.integers(lp.ANGLE_MARGIN, pr["rows"] - lp.ANGLE_MARGIN, 6)
    cols = rng.integers(pr["j_lo"] + 8, pr["j_lo"] + pr["nj"] - 8, 6)
    offs, wz = lp.bspline_weights(np.zeros(1))
    for r, j in zip(rows, cols):
        m = r + pr["m_lo"]
        spline = sum(wa[0] * wb[0] * C[r + oa, j + ob] for oa, wa in zip(offs, wz) for ob, wb in zip(offs, wz))
        direct = 0.0
        for k in range(pr["n_span"]):
            t = j + np.log(np.cos((m - pr["M"] * k) * pr["dpsi"])) / pr["delta"]
            ph = np.exp(2j * np.pi * eta * t / Ns)
            v = Gh[k] * ph
            v[Ns // 2] = Gh[k, Ns // 2].real * np.cos(np.pi * t)
            direct += v.sum().real / Ns
        direct *= pr["dtheta"]
        assert abs(spline - direct) < 1e-10 * max(1.0, abs(direct)), (r, j, spline, direct)


def test_constant_rows_give_pi():
    """Rows identically 1: every voxel's backprojection over a half turn is pi."""
    f = lp.lprec_backproject(np.ones((64, 128)), 0.3, 64.0, 64, os=1.0, eps=0.5)[0]
    assert np.max(np.abs(f - math.pi)) < 2e-6


@pytest.mark.parametrize("spans", [2, 3, 5])
def test_bandlimited_rows_match_direct_sum(spans):
    """Rows band-limited to |k| <= L/8: the splines are then accurate and the
    method agrees with the direct sum of trigonometric interpolants to ~1e-6
    (angles from 0.3, off-centre axis, every voxel)."""
    na, N, L = 64, 64, 128
    y = _bandlimited_rows(7, na, L, L // 8)
    ang = 0.3 + np.arange(na) * math.pi / na
    iy, ix = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ref = oracle.fourier_backproject_points(y, ang, 60.5, N, ix.ravel(), iy.ravel())
    f = lp.lprec_backproject_points(y, 0.3, 60.5, N, ix.ravel(), iy.ravel(), spans=spans, os=1.0, eps=0.5)
    e = np.linalg.norm(f - ref) / np.linalg.norm(ref)
    assert e < 2e-6, e


def test_phantom_error_within_fp16_regime_bar_and_falls_with_oversampling():
    """Full-band filtered rows of a noisy phantom scan: within the 3e-3 bar at
    the default grid, and coarser grids are worse (the error is interpolation)."""
    N, na = 64, 64
    s = synth.phantom_2d_scan(seed=3, n_rows=1, n_angles=na, n_det=N)
    p = oracle.normalize(s.proj, s.dark, s.flat)[0]
    y, off = oracle.filter_rows_padded(p)
    iy, ix = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ref = oracle.fourier_backproject_points(y, s.angles, s.center + off, N, ix.ravel(), iy.ravel())
    errs = {}
    for os_ in (0.5, 1.2):
        f = lp.lprec_backproject_points(y, s.angles[0], s.center + off, N, ix.ravel(), iy.ravel(), os=os_, eps=0.5)
        errs[os_] = np.linalg.norm(f - ref) / np.linalg.norm(ref)
    assert errs[1.2] < 1e-3, errs
    assert errs[0.5] > 4 * errs[1.2], errs
