"""GPU tests of the differentiable projector pair and the least-squares form."""
import numpy as np
import pytest

import oracle
from paper_2209_08450_amd import synth
from tests._util import note, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_08450_amd import autograd, tp
    return tp, autograd


def _loss_fp64(tp, plan, x, y):
    r = to_host(tp.radon(plan, x)).astype(np.float64) - to_host(y).astype(np.float64)
    return float(np.sum(r * r))


def test_gradient_matches_central_differences(mods):
    import torch
    tp, ag = mods
    na, n = 64, 64
    ang = synth.uniform_angles(na) + 0.03
    plan = tp.Plan(ang, n, n / 2 - 0.4)
    rng = np.random.default_rng(0)
    x = to_dev(rng.standard_normal((2, n, n)).astype(np.float32)).requires_grad_(True)
    y = to_dev(rng.standard_normal((2, na, n)).astype(np.float32))
    note("autograd FD 64x64")
    loss = torch.sum((ag.radon(x, plan) - y).double() ** 2)
    loss.backward()
    g = to_host(x.grad).astype(np.float64)
    x0 = x.detach()
    for i in range(4):
        d = rng.standard_normal(x0.shape).astype(np.float32)
        eps = 1e-2
        dd = to_dev(d)
        fd = (_loss_fp64(tp, plan, x0 + eps * dd, y) - _loss_fp64(tp, plan, x0 - eps * dd, y)) / (2 * eps)
        an = float(np.sum(g * d))
        # quadratic loss: central differences are exact up to FP32 rounding of R x
        assert abs(fd - an) <= 1e-3 * abs(an), (i, fd, an)


def test_backproject_fn_gradient(mods):
    import torch
    tp, ag = mods
    na, n = 48, 64
    plan = tp.Plan(synth.uniform_angles(na), n, n / 2)
    rng = np.random.default_rng(1)
    q = to_dev(rng.standard_normal((1, na, n)).astype(np.float32)).requires_grad_(True)
    w = to_dev(rng.standard_normal((1, n, n)).astype(np.float32))
    note("autograd backproject grad")
    s = torch.sum(ag.backproject(q, plan, scale=0.5).double() * w.double())
    s.backward()
    d = rng.standard_normal(q.shape).astype(np.float32)
    dd = to_dev(d)
    f = lambda v: float(torch.sum(tp.backproject(plan, v, scale=0.5).double() * w.double()))  # noqa: E731
    eps = 1e-2
    fd = (f(q.detach() + eps * dd) - f(q.detach() - eps * dd)) / (2 * eps)
    an = float(np.sum(to_host(q.grad).astype(np.float64) * d))
    assert abs(fd - an) <= 1e-4 * abs(an)


def test_ls_trajectory_matches_oracle(mods):
    import torch
    tp, ag = mods
    N, na = 96, 60
    ang = synth.uniform_angles(na)
    c = N / 2
    ell = synth.ellipses_2d(5, count=6)
    img = synth.rasterize_ellipses(ell, N, N / 2)
    y64 = oracle.radon(np.stack([img, img[::-1]]), ang, c, N)
    rng = np.random.default_rng(2)
    y64 = y64 + 0.01 * rng.standard_normal(y64.shape)
    y32 = y64.astype(np.float32)
    lam = oracle.power_lambda_max(ang, c, N, N, iters=60)
    eta = 1.0 / (2.0 * lam)
    plan = tp.Plan(ang, N, c)
    note("LS trajectory 2x96^2, 15 steps")
    x_gpu, l_gpu = ag.ls_solve(plan, to_dev(y32), steps=15, eta=eta)
    x_ref, l_ref = oracle.ls_solve(y32.astype(np.float64), ang, c, N, steps=15, eta=eta)
    assert rel_l2(to_host(x_gpu), x_ref) < 1e-4
    assert np.max(np.abs(np.array(l_gpu) - np.array(l_ref)) / np.array(l_ref)) < 1e-4
    # the device power iteration agrees with the oracle's
    lam_gpu = ag.power_lambda_max(plan, iters=60)
    assert abs(lam_gpu - lam) < 1e-3 * lam


def test_ls_128_slices_1024_900_angles(mods):
    """The differentiation workload: 30 gradient steps on 128 slices of 1024^2
    from 900 angles of noisy data; the loss must not increase and must drop."""
    import torch
    tp, ag = mods
    y, ang, c = synth.ls_problem_torch(seed=4, n_slices=128, n_vox=1024, n_angles=900, device="cuda")
    plan = tp.Plan(ang, 1024, c)
    note("LS 128x1024^2x900, 30 steps")
    eta = ag.step_size(plan)
    x, losses = ag.ls_solve(plan, y, steps=30, eta=eta)
    torch.cuda.synchronize()
    note(f"losses {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert all(b <= a * (1 + 1e-6) for a, b in zip(losses, losses[1:]))
    assert losses[-1] < 0.5 * losses[0]
    assert torch.isfinite(x).all()
