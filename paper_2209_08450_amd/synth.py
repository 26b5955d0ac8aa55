"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds the measurement model only -- random-ellipse phantoms, their
analytic parallel-beam line integrals, Beer-Lambert attenuation and Poisson
counting noise -- and none of the reconstruction's arithmetic (no dark/flat
correction, no filtering, no backprojection).  Both the HIP path and the CPU
oracle receive inputs produced here.

Geometry conventions (match the reconstruction's): image half-width ``half``
pixels spans normalised coordinate 1; detector column j sits at
s = (j - center) / half; the ray at angle theta and offset s is the line
x cos(theta) + y sin(theta) = s.  Densities are per normalised unit length, so
line integrals are dimensionless and a reconstruction in pixel units times
``half`` approximates the density.

The paper's workloads (Section 3) are synthetic N^3 data sets and a 12-bit
glass-bead scan with 2048 projections over 180 degrees; none is available, so
phantoms of random ellipses (2-D) and ellipsoids (3-D) stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


# --------------------------------------------------------------------------
# Phantom parameters.
# --------------------------------------------------------------------------
def ellipses_2d(seed: int, count: int = 10, radius: float = 0.7,
                axes=(0.05, 0.35), density=(0.1, 1.0)) -> np.ndarray:
    """Random ellipses [count, 6] = (x0, y0, a, b, phi, mu).

    Centres uniform in a disc of ``radius``; semi-axes U[axes]; orientation
    U[0, pi); additive density U[density].
    """
    rng = np.random.default_rng(seed)
    r = radius * np.sqrt(rng.uniform(0.0, 1.0, count))
    t = rng.uniform(0.0, 2.0 * math.pi, count)
    a = rng.uniform(axes[0], axes[1], count)
    b = rng.uniform(axes[0], axes[1], count)
    phi = rng.uniform(0.0, math.pi, count)
    mu = rng.uniform(density[0], density[1], count)
    return np.stack([r * np.cos(t), r * np.sin(t), a, b, phi, mu], axis=1)


def ellipsoids_3d(seed: int, count: int = 200, radius: float = 0.7,
                  axes=(0.03, 0.25), density=(0.1, 1.0)) -> np.ndarray:
    """Random ellipsoids [count, 8] = (x0, y0, z0, a, b, c, phi, mu).

    Centres uniform in a ball of ``radius``; semi-axes U[axes]; rotation phi
    about the z (rotation) axis U[0, pi); additive density U[density].
    """
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((count, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = radius * np.cbrt(rng.uniform(0.0, 1.0, count))
    c = v * r[:, None]
    ax = rng.uniform(axes[0], axes[1], (count, 3))
    phi = rng.uniform(0.0, math.pi, count)
    mu = rng.uniform(density[0], density[1], count)
    return np.concatenate([c, ax, phi[:, None], mu[:, None]], axis=1)


def slice_ellipses(ell3: np.ndarray, zn: float) -> np.ndarray:
    """Cross-section of ellipsoids at normalised height zn -> ellipses [m, 6].

    An ellipsoid cut at height zn (|zn - z0| < c) is an ellipse with the same
    centre and orientation and semi-axes scaled by sqrt(1 - ((zn - z0)/c)^2).
    """
    d = (zn - ell3[:, 2]) / ell3[:, 5]
    keep = np.abs(d) < 1.0
    e = ell3[keep]
    k = np.sqrt(1.0 - d[keep] ** 2)
    return np.stack([e[:, 0], e[:, 1], e[:, 3] * k, e[:, 4] * k, e[:, 6], e[:, 7]], axis=1)


def uniform_angles(n_angles: int) -> np.ndarray:
    """theta_a = a pi / n_angles, a = 0..n_angles-1 (a 180-degree scan)."""
    return np.arange(n_angles, dtype=np.float64) * (math.pi / n_angles)


def row_height(z: int, n_rows: int, half: float) -> float:
    """Normalised height of detector row z (rows share the pixel pitch)."""
    return (z - n_rows // 2) / half


# --------------------------------------------------------------------------
# Analytic line integrals.
# --------------------------------------------------------------------------
def chord_sinogram_np(ell2: np.ndarray, angles: np.ndarray, n_det: int, center: float,
                      half: float) -> np.ndarray:
    """Exact line integrals of additive ellipses, float64 numpy [n_angles][n_det].

    For an ellipse with semi-axes (A, B), orientation phi, centre (x0, y0) and
    density mu, the chord at (theta, s) is
        2 mu A B sqrt(alpha^2 - s'^2) / alpha^2,   |s'| < alpha,
    with alpha^2 = A^2 cos^2(theta-phi) + B^2 sin^2(theta-phi) and
    s' = s - (x0 cos theta + y0 sin theta).
    """
    th = np.asarray(angles, dtype=np.float64)[:, None]
    s = (np.arange(n_det, dtype=np.float64) - center)[None, :] / half
    out = np.zeros((th.shape[0], n_det), dtype=np.float64)
    for x0, y0, A, B, phi, mu in np.asarray(ell2, dtype=np.float64):
        al2 = (A * np.cos(th - phi)) ** 2 + (B * np.sin(th - phi)) ** 2
        sp = s - (x0 * np.cos(th) + y0 * np.sin(th))
        r = al2 - sp * sp
        out += np.where(r > 0, 2.0 * mu * A * B * np.sqrt(np.maximum(r, 0.0)) / al2, 0.0)
    return out


def chord_sinogram_volume(ell3: np.ndarray, rows, n_rows: int, angles: np.ndarray, n_det: int,
                          center: float, half: float, device="cpu", dtype=None):
    """Analytic line integrals of an ellipsoid phantom for detector ``rows``.

    Returns a torch tensor [len(rows)][n_angles][n_det] on ``device``.  Works
    row-batched: each ellipsoid contributes only to the rows it intersects.
    """
    import torch

    dtype = dtype or (torch.float64 if str(device) == "cpu" else torch.float32)
    rows = list(rows)
    nr = len(rows)
    th = torch.as_tensor(np.asarray(angles, dtype=np.float64), device=device).to(dtype)
    ct, st = torch.cos(th), torch.sin(th)
    s = ((torch.arange(n_det, device=device, dtype=dtype) - center) / half)
    out = torch.zeros((nr, th.shape[0], n_det), device=device, dtype=dtype)
    zn = np.array([row_height(z, n_rows, half) for z in rows])
    for x0, y0, z0, A, B, C, phi, mu in np.asarray(ell3, dtype=np.float64):
        d = (zn - z0) / C
        hit = np.nonzero(np.abs(d) < 1.0)[0]
        if hit.size == 0:
            continue
        k2 = torch.as_tensor(1.0 - d[hit] ** 2, device=device, dtype=dtype)  # [h]
        al2 = (A * torch.cos(th - phi)) ** 2 + (B * torch.sin(th - phi)) ** 2  # [na]
        sp = s[None, :] - (x0 * ct + y0 * st)[:, None]  # [na, n]
        r = k2[:, None, None] * al2[None, :, None] - (sp * sp)[None]  # [h, na, n]
        val = torch.sqrt(torch.clamp_min(r, 0.0)) * (2.0 * mu * A * B) / al2[None, :, None]
        idx = torch.as_tensor(hit, device=device)
        out.index_add_(0, idx, val)
    return out


def rasterize_ellipses(ell2: np.ndarray, N: int, half: float, supersample: int = 4) -> np.ndarray:
    """Density image [N][N] of additive ellipses, averaged over sub-pixel samples.

    Pixel (iy, ix) is centred at ((ix - N//2)/half, (iy - N//2)/half).
    """
    ss = supersample
    off = (np.arange(ss) + 0.5) / ss - 0.5
    c = (np.arange(N) - N // 2)[:, None] + off[None, :]  # [N, ss]
    c = c.reshape(-1) / half
    X, Y = np.meshgrid(c, c)  # Y varies along axis 0 (rows = iy)
    img = np.zeros_like(X)
    for x0, y0, A, B, phi, mu in np.asarray(ell2, dtype=np.float64):
        dx, dy = X - x0, Y - y0
        u = dx * math.cos(phi) + dy * math.sin(phi)
        v = -dx * math.sin(phi) + dy * math.cos(phi)
        img += np.where((u / A) ** 2 + (v / B) ** 2 <= 1.0, mu, 0.0)
    return img.reshape(N, ss, N, ss).mean(axis=(1, 3))


# --------------------------------------------------------------------------
# Counting model.
# --------------------------------------------------------------------------
def counts_np(p: np.ndarray, flat_level: float, dark_level: float, rng: np.random.Generator,
              max_count: int = 65535, dark_poisson: bool = False) -> np.ndarray:
    """Raw detector counts: Poisson(flat e^{-p}) + dark, clipped, uint16."""
    lam = flat_level * np.exp(-np.asarray(p, dtype=np.float64))
    v = rng.poisson(lam).astype(np.float64)
    v += rng.poisson(dark_level, size=v.shape) if dark_poisson else dark_level
    return np.clip(v, 0, max_count).astype(np.uint16)


@dataclass
class ScanData:
    """Raw scan in the recorded layout.

    proj: uint16 [n_angles][n_rows][n_det]; dark/flat: uint16 [frames][n_rows][n_det];
    angles: float64 [n_angles] (host); center: rotation axis in detector pixels.
    Arrays are numpy (host) or torch tensors (device) depending on the maker.
    """
    proj: object
    dark: object
    flat: object
    angles: np.ndarray
    center: float
    n_vox: int


def phantom_2d_scan(seed: int = 1, n_rows: int = 16, n_angles: int = 180, n_det: int = 256,
                    center: float | None = None, n_ellipses: int = 10, flat_level: float = 4000.0,
                    dark_level: float = 100.0) -> ScanData:
    """Small scan: one 2-D random-ellipse phantom repeated on every row.

    Phantom seed ``seed``; counting noise seeded per row by SeedSequence([seed, z]).
    One dark frame identically ``dark_level``; one flat frame
    Poisson(flat_level) + dark_level; raw = Poisson(flat e^{-p}) + dark.
    """
    center = n_det / 2 if center is None else center
    half = n_det / 2
    ell = ellipses_2d(seed, n_ellipses)
    ang = uniform_angles(n_angles)
    p = chord_sinogram_np(ell, ang, n_det, center, half)  # [na][n]
    proj = np.empty((n_angles, n_rows, n_det), dtype=np.uint16)
    flat = np.empty((1, n_rows, n_det), dtype=np.uint16)
    dark = np.full((1, n_rows, n_det), int(dark_level), dtype=np.uint16)
    for z in range(n_rows):
        rng = np.random.default_rng(np.random.SeedSequence([seed, z]))
        proj[:, z, :] = counts_np(p, flat_level, dark_level, rng)
        flat[0, z, :] = counts_np(np.zeros(n_det), flat_level, dark_level, rng)
    return ScanData(proj, dark, flat, ang, float(center), n_det)


def ellipsoid_scan_np(seed: int, n_angles: int, n_rows: int, n_det: int, center=None,
                      n_ellipsoids: int = 200, flat_level: float = 3600.0, dark_level: float = 100.0,
                      n_dark: int = 20, n_flat: int = 20, max_count: int = 4095,
                      rows=None) -> ScanData:
    """12-bit scan of a 3-D ellipsoid phantom, host numpy (small sizes).

    raw = clip(Poisson(flat e^{-p}) + Poisson(dark), 0, 4095); darks Poisson(dark);
    flats Poisson(flat) + Poisson(dark).  ``rows`` selects a subset of detector
    rows of an ``n_rows``-row detector (noise seeded per row by
    SeedSequence([seed, z])).
    """
    center = n_det / 2 if center is None else center
    half = n_det / 2
    rows = list(range(n_rows)) if rows is None else list(rows)
    ell = ellipsoids_3d(seed, n_ellipsoids)
    ang = uniform_angles(n_angles)
    proj = np.empty((n_angles, len(rows), n_det), dtype=np.uint16)
    dark = np.empty((n_dark, len(rows), n_det), dtype=np.uint16)
    flat = np.empty((n_flat, len(rows), n_det), dtype=np.uint16)
    for i, z in enumerate(rows):
        e2 = slice_ellipses(ell, row_height(z, n_rows, half))
        p = chord_sinogram_np(e2, ang, n_det, center, half)
        rng = np.random.default_rng(np.random.SeedSequence([seed, z]))
        proj[:, i, :] = counts_np(p, flat_level, dark_level, rng, max_count, dark_poisson=True)
        dark[:, i, :] = np.clip(rng.poisson(dark_level, (n_dark, n_det)), 0, max_count)
        flat[:, i, :] = counts_np(np.zeros((n_flat, n_det)), flat_level, dark_level, rng, max_count,
                                  dark_poisson=True)
    return ScanData(proj, dark, flat, ang, float(center), n_det)


def ellipsoid_scan_torch(seed: int, n_angles: int, n_rows: int, n_det: int, device, center=None,
                         n_ellipsoids: int = 200, flat_level: float = 3600.0, dark_level: float = 100.0,
                         n_dark: int = 20, n_flat: int = 20, max_count: int = 4095,
                         rows_per_batch: int = 16, out=None, progress=None) -> ScanData:
    """Same measurement model as ``ellipsoid_scan_np`` generated with torch on ``device``.

    For paper-scale scans (e.g. 2048 angles x 2048 rows x 2048 columns).  The
    noise comes from torch's generator seeded with (seed, batch); it is not the
    numpy stream, so checks against the oracle copy the needed raw rows back to
    the host.  Device containers are int16 tensors holding the uint16 bit
    patterns (view them as uint16 on the host).  ``out`` may supply a
    preallocated int16 [n_angles][n_rows][n_det].
    """
    import torch

    center = n_det / 2 if center is None else center
    half = n_det / 2
    ell = ellipsoids_3d(seed, n_ellipsoids)
    ang = uniform_angles(n_angles)
    proj = out if out is not None else torch.empty((n_angles, n_rows, n_det), dtype=torch.int16,
                                                   device=device)
    gen = torch.Generator(device=device)
    for b, z0 in enumerate(range(0, n_rows, rows_per_batch)):
        z1 = min(n_rows, z0 + rows_per_batch)
        gen.manual_seed(int(np.random.SeedSequence([seed, 1, b]).generate_state(1)[0]))
        p = chord_sinogram_volume(ell, range(z0, z1), n_rows, ang, n_det, center, half, device=device)
        lam = flat_level * torch.exp(-p)
        v = torch.poisson(lam, generator=gen)
        v += torch.poisson(torch.full_like(v, dark_level), generator=gen)
        v = torch.clamp(v, 0, max_count).to(torch.int32).to(torch.int16)
        proj[:, z0:z1, :] = v.permute(1, 0, 2)
        del p, lam, v
        if progress is not None:
            progress(z1, n_rows)
    gen.manual_seed(int(np.random.SeedSequence([seed, 2]).generate_state(1)[0]))
    dk = torch.poisson(torch.full((n_dark, n_rows, n_det), dark_level, device=device), generator=gen)
    dark = torch.clamp(dk, 0, max_count).to(torch.int32).to(torch.int16)
    fl = torch.poisson(torch.full((n_flat, n_rows, n_det), flat_level, device=device), generator=gen)
    fl += torch.poisson(torch.full_like(fl, dark_level), generator=gen)
    flat = torch.clamp(fl, 0, max_count).to(torch.int32).to(torch.int16)
    return ScanData(proj, dark, flat, ang, float(center), n_det)


def noisy_line_integrals(p: np.ndarray, flat_level: float, rng: np.random.Generator) -> np.ndarray:
    """Line integrals with counting noise in its Gaussian limit.

    y = p + sqrt(e^{p} / flat_level) * N(0, 1): the variance of -ln of a
    Poisson count with mean flat_level e^{-p}, to first order.
    """
    p = np.asarray(p, dtype=np.float64)
    return p + np.sqrt(np.exp(p) / flat_level) * rng.standard_normal(p.shape)


def noisy_line_integrals_torch(p, flat_level: float, generator):
    """Torch version of ``noisy_line_integrals`` on p's device."""
    import torch
    e = torch.randn(p.shape, generator=generator, device=p.device, dtype=p.dtype)
    return p + torch.sqrt(torch.exp(p) / flat_level) * e


def ls_problem_torch(seed: int, n_slices: int, n_vox: int, n_angles: int, device, flat_level: float = 4000.0,
                     n_ellipsoids: int = 200):
    """Noisy line integrals y [n_slices][n_angles][n_vox] of the central slices of
    an ellipsoid phantom on an n_vox^3 grid, in pixel units (the FP32 least-squares
    data of the differentiation workload).  Returns (y, angles, center)."""
    import torch
    half = n_vox / 2
    center = n_vox / 2
    ell = ellipsoids_3d(seed, n_ellipsoids)
    ang = uniform_angles(n_angles)
    z0 = n_vox // 2 - n_slices // 2
    p = chord_sinogram_volume(ell, range(z0, z0 + n_slices), n_vox, ang, n_vox, center, half, device=device,
                              dtype=torch.float32)
    g = torch.Generator(device=device)
    g.manual_seed(int(np.random.SeedSequence([seed, 3]).generate_state(1)[0]))
    y = noisy_line_integrals_torch(p, flat_level, g) * half  # pixel units: line integral of a per-pixel density
    return y.contiguous(), ang, center
