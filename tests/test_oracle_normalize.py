"""Pins of the oracle's dark/flat correction and -log (paper, Section 2.2)."""
import math

import numpy as np

import oracle


def _stack(value, frames, nz=2, n=3):
    return np.full((frames, nz, n), value, dtype=np.uint16)


def test_half_transmission_gives_ln2():
    # dark 100, flat 4100, raw 2100 -> transmission exactly 1/2 -> p = ln 2
    proj = _stack(2100, 4)
    p = oracle.normalize(proj, _stack(100, 1), _stack(4100, 1))
    assert p.shape == (2, 4, 3)
    assert np.all(p == -math.log(0.5))


def test_photon_starvation_clamps():
    # raw equal to dark -> transmission 0 -> clamped at 1e-6
    p = oracle.normalize(_stack(100, 2), _stack(100, 1), _stack(4100, 1))
    assert np.allclose(p, -math.log(1e-6), rtol=0, atol=1e-15)
    assert abs(p.max() - 13.815510557964274) < 1e-12
    # raw below dark is clamped the same way
    p = oracle.normalize(_stack(50, 2), _stack(100, 1), _stack(4100, 1))
    assert np.allclose(p, -math.log(1e-6))


def test_dead_pixel_uses_unit_denominator():
    # flat == dark -> denominator one count -> t = P - D
    p = oracle.normalize(_stack(101, 1), _stack(100, 1), _stack(100, 1))
    assert np.allclose(p, 0.0, atol=1e-15)
    p = oracle.normalize(_stack(100 + 1, 1), _stack(100, 1), _stack(99, 1))
    assert np.allclose(p, 0.0, atol=1e-15)


def test_frames_are_averaged():
    dark = np.stack([_stack(90, 1)[0], _stack(110, 1)[0]])     # mean 100
    flat = np.stack([_stack(4000, 1)[0], _stack(4200, 1)[0]])  # mean 4100
    p = oracle.normalize(_stack(2100, 3), dark, flat)
    assert np.allclose(p, math.log(2.0), rtol=0, atol=1e-15)


def test_layout_projection_major_to_sinogram_major():
    rng = np.random.default_rng(0)
    na, nz, n = 5, 3, 7
    proj = rng.integers(200, 4000, (na, nz, n)).astype(np.uint16)
    dark = rng.integers(90, 110, (2, nz, n)).astype(np.uint16)
    flat = rng.integers(4000, 4100, (3, nz, n)).astype(np.uint16)
    p = oracle.normalize(proj, dark, flat)
    a, z, j = 4, 1, 6
    d = dark[:, z, j].astype(float).mean()
    f = flat[:, z, j].astype(float).mean()
    want = -math.log((float(proj[a, z, j]) - d) / (f - d))
    assert p.shape == (nz, na, n)
    assert abs(p[z, a, j] - want) < 1e-14
