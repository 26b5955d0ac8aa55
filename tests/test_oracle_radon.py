"""Pins of the oracle's forward projector (transpose of the backprojector)."""
import math

import numpy as np

import oracle
from paper_2209_08450_amd import synth


def test_adjoint_identity():
    N, n, na = 48, 60, 29
    rng = np.random.default_rng(0)
    ang = synth.uniform_angles(na) + 0.01
    x = rng.standard_normal((2, N, N))
    y = rng.standard_normal((2, na, n))
    lhs = np.vdot(oracle.radon(x, ang, 31.7, n), y)
    rhs = np.vdot(x, oracle.backproject(y, ang, 31.7, N, scale=1.0))
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0) * 10


def test_mass_conservation():
    # the hat weights of every voxel sum to one on each angle
    N, n, na = 32, 64, 17
    rng = np.random.default_rng(1)
    f = rng.uniform(0, 1, (1, N, N))
    r = oracle.radon(f, synth.uniform_angles(na), n / 2, n)[0]
    assert np.allclose(r.sum(axis=1), f.sum(), rtol=1e-13)


def test_single_pixel_two_hat_weights():
    N, n = 16, 24
    f = np.zeros((1, N, N))
    ix, iy = 11, 5
    f[0, iy, ix] = 2.0
    ang = np.array([0.3, 1.1, 2.5])
    c = 12.2
    r = oracle.radon(f, ang, c, n)[0]
    for a, th in enumerate(ang):
        s = (ix - N // 2) * math.cos(th) + (iy - N // 2) * math.sin(th) + c
        j0 = math.floor(s)
        w = s - j0
        want = np.zeros(n)
        want[j0] = 2.0 * (1 - w)
        want[j0 + 1] = 2.0 * w
        assert np.allclose(r[a], want, atol=1e-14)


def test_rasterised_ellipse_matches_analytic_chords():
    # 4x4-supersampled rasterisation of ellipses projected by the oracle versus
    # the analytic chord lengths, N = 256.  The pixel-driven hat projector has
    # an O(1/N)-ish discretisation error (2.2e-2 here, 2.0e-2 at N = 512);
    # a half-pixel offset, a wrong orientation or a transposed image would
    # show as a larger error than neighbouring shifted geometries give.
    N = n = 256
    half = n / 2
    ell = synth.ellipses_2d(7, count=3)
    img = synth.rasterize_ellipses(ell, N, half, supersample=4)
    ang = synth.uniform_angles(24)
    r = oracle.radon(img[None], ang, n / 2, n)[0] / half  # pixel units -> normalised

    def err(center_shift=0.0, angles=ang):
        p = synth.chord_sinogram_np(ell, angles, n, n / 2 + center_shift, half)
        return np.linalg.norm(r - p) / np.linalg.norm(p)

    e0 = err()
    assert e0 < 3e-2
    assert err(0.25) > 1.2 * e0 and err(-0.25) > 1.2 * e0
    assert err(angles=ang + np.pi) > 10 * e0   # mirrored geometry
    assert err(angles=np.pi / 2 - ang) > 10 * e0  # x/y swapped
