"""Pins of the oracle's sampled-voxel helpers against its pinned full-slice
compositions.

``fbp_points`` and ``fourier_fbp_points`` evaluate one detector row's FBP
(paper, Section 2.2: correction, -log, padded filtering, backprojection) at
listed voxels.  They are the checkers of every paper-scale GPU test, so each
is held equal to the full-slice composition (``fbp`` / ``fourier_fbp``, pinned
by closed forms in the other oracle tests) read at the same voxels, on scans
chosen so that a slicing, row-selection, N-versus-n, centre or storage
mistake changes the values: several frames of darks and flats with different
values per row, a voxel grid larger and smaller than the detector, a
non-integer, off-centre axis, every filter window and storage rounding.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2209_08450_amd import synth

CASES = [
    # (n_angles, n_rows, n_det, center, N)
    (13, 3, 20, 9.37, 24),     # N > n, axis left of the middle, fractional
    (9, 4, 31, 17.5, 22),      # odd detector, N < n, half-integer axis
    (16, 2, 16, 8.0, 16),      # N = n, integer axis on the middle
]


def _scan(n_angles, n_rows, n_det, center, seed):
    s = synth.ellipsoid_scan_np(seed, n_angles, n_rows, n_det, center=center, n_ellipsoids=12,
                                n_dark=3, n_flat=4)
    return s


def _voxels(N, seed):
    rng = np.random.default_rng(seed)
    ix = rng.integers(0, N, 40)
    iy = rng.integers(0, N, 40)
    # the four corners and the centre too
    ix = np.concatenate([ix, [0, N - 1, 0, N - 1, N // 2]])
    iy = np.concatenate([iy, [0, 0, N - 1, N - 1, N // 2]])
    return ix, iy


@pytest.mark.parametrize("kind", oracle.FILTERS)
@pytest.mark.parametrize("storage", [None, "f16", "bf16"])
@pytest.mark.parametrize("case", CASES)
def test_fbp_points_equal_full_slice(case, storage, kind):
    na, nz, n, c, N = case
    s = _scan(na, nz, n, c, seed=5)
    full = oracle.fbp(s.proj, s.dark, s.flat, s.angles, c, N, storage=storage, kind=kind)
    assert full.shape == (nz, N, N)
    ix, iy = _voxels(N, seed=na + nz)
    for z in range(nz):
        pts = oracle.fbp_points(s.proj[:, z, :], s.dark[:, z, :], s.flat[:, z, :], s.angles, c, N, ix, iy,
                                storage=storage, kind=kind)
        want = full[z][iy, ix]
        assert np.max(np.abs(pts - want)) <= 1e-12 * max(1.0, np.max(np.abs(full[z])))


def test_fbp_points_see_their_own_row():
    # rows differ, so reading the wrong row (or mixing frames of another row)
    # would change the value: every row's points differ from every other row's
    na, nz, n, c, N = 11, 3, 18, 8.6, 18
    s = _scan(na, nz, n, c, seed=9)
    ix, iy = _voxels(N, seed=3)
    vals = [oracle.fbp_points(s.proj[:, z, :], s.dark[:, z, :], s.flat[:, z, :], s.angles, c, N, ix, iy)
            for z in range(nz)]
    for a in range(nz):
        for b in range(a + 1, nz):
            assert np.max(np.abs(vals[a] - vals[b])) > 1e-6


@pytest.mark.parametrize("kind", oracle.FILTERS)
@pytest.mark.parametrize("case", CASES)
def test_fourier_fbp_points_equal_full_slice(case, kind):
    na, nz, n, c, N = case
    s = _scan(na, nz, n, c, seed=6)
    full = oracle.fourier_fbp(s.proj, s.dark, s.flat, s.angles, c, N, kind=kind)
    assert full.shape == (nz, N, N)
    ix, iy = _voxels(N, seed=na * 7 + nz)
    for z in range(nz):
        pts = oracle.fourier_fbp_points(s.proj[:, z, :], s.dark[:, z, :], s.flat[:, z, :], s.angles, c, N,
                                        ix, iy, kind=kind)
        want = full[z][iy, ix]
        assert np.max(np.abs(pts - want)) <= 1e-12 * max(1.0, np.max(np.abs(full[z])))


def test_points_helpers_use_the_pad_offset_and_centre():
    # With one angle at 0 and an integer axis, both helpers read filtered
    # samples at j = ix - N//2 + c, so a pad-offset or centre slip would show
    # as a shift of the row: compare with the filtered row itself.
    n, c, N = 20, 11, 16
    rng = np.random.default_rng(4)
    proj = rng.integers(500, 4000, size=(1, 1, n)).astype(np.uint16)
    dark = np.full((2, 1, n), 100, dtype=np.uint16)
    flat = np.full((2, 1, n), 4100, dtype=np.uint16)
    ang = np.array([0.0])
    q = oracle.filter_rows(oracle.normalize(proj, dark, flat))[0, 0]
    ix = np.arange(N)
    iy = np.full(N, 3)
    want = math.pi * q[ix - N // 2 + c]
    got = oracle.fbp_points(proj[:, 0, :], dark[:, 0, :], flat[:, 0, :], ang, c, N, ix, iy)
    assert np.max(np.abs(got - want)) < 1e-12
    gotf = oracle.fourier_fbp_points(proj[:, 0, :], dark[:, 0, :], flat[:, 0, :], ang, c, N, ix, iy)
    assert np.max(np.abs(gotf - want)) < 1e-10
