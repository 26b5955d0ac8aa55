"""Pins of the oracle's laminographic backprojection (paper, Section 2.2: the
direct line-integral backprojector serves laminographic geometry, a rotation
axis tilted with respect to the beam).  Geometry reading: voxel (x, y, z) is
seen at column u = x cos + y sin + c_u and row
v = (-x sin + y cos) cos(phi) + z sin(phi) + c_v, bilinear interpolation,
zero off the detector."""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle


def test_tilt_of_ninety_degrees_is_tomography():
    # phi = pi/2: every slice reads one detector row (z + c_v) and the result
    # is the linear-interpolation backprojection of that row
    rng = np.random.default_rng(1)
    na, rows, n, N, Nz = 9, 12, 20, 14, 5
    q = rng.standard_normal((na, rows, n))
    ang = rng.uniform(0, math.pi, na)
    cu, cv = 9.3, 6.0
    f = oracle.lamino_backproject(q, ang, cu, cv, math.pi / 2, N, Nz)
    for iz in range(Nz):
        r = iz - Nz // 2 + int(cv)
        want = oracle.backproject(q[:, r, :][None], ang, cu, N)[0]
        assert np.max(np.abs(f[iz] - want)) < 1e-12


@pytest.mark.parametrize("phi", [0.35, 1.0, 2.2])
def test_matches_library_bilinear_interpolation(phi):
    # scipy's order-1 map_coordinates with grid-constant zero padding is an
    # independent evaluation of the same bilinear sum, including voxels whose
    # taps fall off every edge of the detector
    rng = np.random.default_rng(2)
    na, rows, n, N, Nz = 7, 11, 13, 12, 6
    q = rng.standard_normal((na, rows, n))
    ang = rng.uniform(-math.pi, 2 * math.pi, na)
    cu, cv = 6.4, 5.2
    f = oracle.lamino_backproject(q, ang, cu, cv, phi, N, Nz, scale=1.0)
    iz, iy, ix = np.meshgrid(np.arange(Nz), np.arange(N), np.arange(N), indexing="ij")
    x, y, z = ix - N // 2, iy - N // 2, iz - Nz // 2
    want = np.zeros(f.shape)
    off_detector = 0
    for a in range(na):
        c, s = math.cos(ang[a]), math.sin(ang[a])
        u = x * c + y * s + cu
        v = (-x * s + y * c) * math.cos(phi) + z * math.sin(phi) + cv
        off_detector += int(np.sum((u < 0) | (u > n - 1) | (v < 0) | (v > rows - 1)))
        want += ndimage.map_coordinates(q[a], [v.ravel(), u.ravel()], order=1, mode="grid-constant",
                                        cval=0.0).reshape(f.shape)
    assert np.max(np.abs(f - want)) < 1e-12
    assert off_detector > 0  # taps past the detector edges were part of the comparison


def test_constant_projections_give_pi():
    # q = 1 on a detector that holds every tap: each angle adds 1, scale pi/na
    na, N, Nz = 16, 10, 4
    q = np.ones((na, 40, 40))
    ang = np.arange(na) * 2 * math.pi / na
    f = oracle.lamino_backproject(q, ang, 19.5, 19.5, 0.7, N, Nz)
    assert np.max(np.abs(f - math.pi)) < 1e-12


def test_points_match_full_volume():
    rng = np.random.default_rng(3)
    q = rng.standard_normal((5, 9, 10))
    ang = rng.uniform(0, math.pi, 5)
    f = oracle.lamino_backproject(q, ang, 4.7, 4.1, 0.9, 8, 5)
    ix, iy, iz = rng.integers(0, 8, 30), rng.integers(0, 8, 30), rng.integers(0, 5, 30)
    v = oracle.lamino_backproject_points(q, ang, 4.7, 4.1, 0.9, 8, 5, ix, iy, iz)
    assert np.array_equal(v, f[iz, iy, ix])
