"""Pins of the oracle's least-squares pieces (gradient, step size, descent)."""
import numpy as np

import oracle
from paper_2209_08450_amd import synth


def _setup(N=12, n=16, na=9):
    return synth.uniform_angles(na) + 0.05, n / 2 - 0.3, N, n


def test_gradient_matches_central_differences():
    ang, c, N, n = _setup()
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, N, N))
    y = rng.standard_normal((1, len(ang), n))
    g = oracle.ls_gradient(x, y, ang, c)

    def loss(v):
        r = oracle.radon(v, ang, c, n) - y
        return float(np.sum(r * r))

    for _ in range(5):
        d = rng.standard_normal(x.shape)
        eps = 1e-3
        fd = (loss(x + eps * d) - loss(x - eps * d)) / (2 * eps)  # exact for a quadratic
        assert abs(fd - np.vdot(g, d)) <= 1e-8 * max(1.0, abs(fd))


def test_power_iteration_matches_dense_eigenvalue():
    ang, c, N, n = _setup(N=8, n=12, na=8)
    lam = oracle.power_lambda_max(ang, c, N, n, iters=300)
    # dense R from unit vectors, largest eigenvalue of R^T R by LAPACK
    R = np.stack([oracle.radon(e.reshape(1, N, N), ang, c, n).reshape(-1)
                  for e in np.eye(N * N)], axis=1)
    want = np.linalg.eigvalsh(R.T @ R)[-1]
    assert abs(lam - want) <= 1e-6 * want


def test_descent_is_monotone_and_converges_on_consistent_data():
    ang, c, N, n = _setup(N=16, n=24, na=24)
    ell = synth.ellipses_2d(3, count=4)
    img = synth.rasterize_ellipses(ell, N, N / 2)[None]
    y = oracle.radon(img, ang, c, n)
    lam = oracle.power_lambda_max(ang, c, N, n, iters=60)
    x, losses = oracle.ls_solve(y, ang, c, N, steps=200, eta=1.0 / (2 * lam))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(losses, losses[1:]))
    assert losses[-1] < 1e-2 * losses[0]
