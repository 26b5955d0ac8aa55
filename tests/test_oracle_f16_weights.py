"""Pins of the oracle's 16-bit mode of the backprojection (paper, Section 2.1:
16-bit arithmetic, with higher precision where accuracy needs it): the two
interpolation weights (1 - w) and w are held as binary16 numbers, the products
and their sum are exact (FP64 here)."""
import math

import numpy as np

import oracle
from paper_2209_08450_amd import synth


def test_round_binary16_matches_numpy_half_conversion():
    # numpy converts double -> half with round-to-nearest-even, independently
    # of the oracle's C helper
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.uniform(0.0, 1.0, 4000), rng.uniform(0.0, 1e-3, 500), 10.0 ** rng.uniform(-9, 0, 500)])
    for x in xs:
        assert oracle.round_binary16(x) == float(np.float16(x)), x


def test_round_binary16_ties_and_subnormals():
    # 0.5 + 2^-12 lies halfway between 0.5 and 0.5 + 2^-11: ties go to the even
    # significand (0.5); 0.5 + 3 * 2^-12 goes up to 0.5 + 2^-10
    assert oracle.round_binary16(0.5 + 2.0 ** -12) == 0.5
    assert oracle.round_binary16(0.5 + 3 * 2.0 ** -12) == 0.5 + 2.0 ** -10
    # binary16 spacing is 2^-24 below 2^-14: 2^-25 ties to 0, 3 * 2^-25 to 2^-23
    assert oracle.round_binary16(2.0 ** -25) == 0.0
    assert oracle.round_binary16(3 * 2.0 ** -25) == 2.0 ** -23
    assert oracle.round_binary16(1.0 - 2.0 ** -13) == 1.0
    for k in range(2049):  # multiples of 2^-11 in [0, 1] are binary16 numbers
        assert oracle.round_binary16(k / 2048.0) == k / 2048.0


def test_single_voxel_weights_by_hand():
    # one angle, one voxel: f = scale * (h(1 - w) Q[j0] + h(w) Q[j0 + 1]) with
    # h the numpy half conversion, evaluated here independently of the C loop
    N, n = 16, 24
    rng = np.random.default_rng(4)
    q = rng.standard_normal((1, 3, n))
    ang = np.array([0.31, 1.7, 2.9])
    c = 11.37
    f = oracle.backproject(q, ang, c, N, scale=0.75, weights="f16")[0]
    for iy, ix in [(0, 0), (3, 11), (8, 8), (15, 2)]:
        x, y = ix - N // 2, iy - N // 2
        want = 0.0
        for a, t in enumerate(ang):
            s = x * math.cos(t) + y * math.sin(t) + c
            j0 = math.floor(s)
            w = s - j0
            q0 = q[0, a, j0] if 0 <= j0 < n else 0.0
            q1 = q[0, a, j0 + 1] if 0 <= j0 + 1 < n else 0.0
            want += float(np.float16(1.0 - w)) * q0 + float(np.float16(w)) * q1
        assert abs(f[iy, ix] - 0.75 * want) < 1e-13


def test_f16_weights_stay_within_half_a_unit_of_the_exact_ones():
    # each weight moves by at most half a binary16 spacing (2^-12 in [0.5, 1],
    # less below), so per tap pair |delta| <= 2^-12 (|Q0| + |Q1|)
    N = n = 48
    na = 29
    c = 23.4
    rng = np.random.default_rng(5)
    q = rng.standard_normal((1, na, n))
    ang = synth.uniform_angles(na) + 0.2
    exact = oracle.backproject(q, ang, c, N, scale=1.0)[0]
    half = oracle.backproject(q, ang, c, N, scale=1.0, weights="f16")[0]
    yy, xx = np.mgrid[0:N, 0:N]
    bound = np.zeros((N, N))
    qp = np.concatenate([np.zeros((na, 1)), q[0], np.zeros((na, 2))], axis=1)  # taps off the detector read 0
    for a, t in enumerate(ang):
        s = (xx - N // 2) * math.cos(t) + (yy - N // 2) * math.sin(t) + c
        j0 = np.floor(s).astype(int)
        i0 = np.clip(j0 + 1, 0, n + 1)
        i1 = np.clip(j0 + 2, 0, n + 1)
        bound += 2.0 ** -12 * (np.abs(qp[a, i0]) + np.abs(qp[a, i1]))
    assert np.all(np.abs(half - exact) <= bound + 1e-12)
    assert np.max(np.abs(half - exact)) > 0  # the mode is not a no-op


def test_constant_rows_in_f16_mode_stay_near_pi():
    # (1 - w) and w rounded separately: the pair sums to 1 within 2^-11, so a
    # constant sinogram backprojects to pi within pi * 2^-11
    N = n = 64
    na = 45
    ang = synth.uniform_angles(na)
    f = oracle.backproject(np.ones((1, na, n)), ang, n / 2 + 0.3, N, weights="f16")[0]
    yy, xx = np.mgrid[0:N, 0:N]
    inner = np.hypot(xx - N // 2, yy - N // 2) < n / 2 - 3
    assert np.max(np.abs(f[inner] - math.pi)) <= math.pi * 2.0 ** -11
    assert np.max(np.abs(f[inner] - math.pi)) > 0


def test_points_follow_the_full_backprojection_in_f16_mode():
    N, n, na = 40, 52, 31
    rng = np.random.default_rng(6)
    q = rng.standard_normal((na, n))
    ang = synth.uniform_angles(na) - 0.4
    full = oracle.backproject(q[None], ang, 25.8, N, weights="f16")[0]
    ix = rng.integers(0, N, 60)
    iy = rng.integers(0, N, 60)
    pts = oracle.backproject_points(q, ang, 25.8, N, ix, iy, weights="f16")
    assert np.max(np.abs(pts - full[iy, ix])) < 1e-12


def test_fbp_f16_storage_uses_f16_weights():
    s = synth.phantom_2d_scan(seed=7, n_rows=2, n_angles=36, n_det=40, center=19.6)
    rows = oracle.round_f16(oracle.filter_rows(oracle.normalize(s.proj, s.dark, s.flat)))
    want = oracle.backproject(rows, s.angles, s.center, 40, weights="f16")
    got = oracle.fbp(s.proj, s.dark, s.flat, s.angles, s.center, storage="f16")
    assert np.max(np.abs(got - want)) < 1e-12
    # bf16 storage keeps exact weights
    rows_b = oracle.round_bf16(oracle.filter_rows(oracle.normalize(s.proj, s.dark, s.flat)))
    want_b = oracle.backproject(rows_b, s.angles, s.center, 40)
    assert np.max(np.abs(oracle.fbp(s.proj, s.dark, s.flat, s.angles, s.center, storage="bf16") - want_b)) < 1e-12
