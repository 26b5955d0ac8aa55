"""GPU parity of the laminographic backprojection (tp_lamino_backproject:
tilted rotation axis, bilinear interpolation of filtered projections) against
the FP64 oracle."""
import math

import numpy as np
import pytest

import oracle
from tests._util import assert_parity, note, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_08450_amd import tp as mod
    return mod


def _case(seed, na, rows, n):
    rng = np.random.default_rng(seed)
    q = rng.standard_normal((na, rows, n)).astype(np.float32)
    ang = np.arange(na) * 2 * math.pi / na + 0.1
    return q, ang


@pytest.mark.parametrize("tilt", [0.05, 0.45, 1.1, 2.4])
def test_lamino_matches_oracle(tp, tilt):
    # 40 angles over a full turn, 30 detector rows x 50 columns, a 45^2 x 13
    # volume (tiles of 32 past the edge, slice blocks of 8 with a ragged end);
    # tilt 0.05 needs windows of 50 rows (more than 64 KiB of LDS)
    q, ang = _case(1, 40, 30, 50)
    N, Nz, cu, cv = 45, 13, 24.3, 14.6
    plan = tp.Plan(ang, 50, cu, N)
    note(f"lamino tilt {tilt}")
    got = to_host(tp.lamino_backproject(plan, to_dev(q), tilt, cv, Nz)).astype(np.float64)
    want = oracle.lamino_backproject(q.astype(np.float64), ang, cu, cv, tilt, N, Nz)
    e = rel_l2(got, want)
    note(f"rel-L2 {e}")
    assert e < 1e-5
    assert np.max(np.abs(got - want)) < 1e-5 * np.max(np.abs(want))


@pytest.mark.parametrize("na", [1, 3, 5, 37])
def test_lamino_ragged_angle_blocks(tp, na):
    # angles are taken 4 at a time, the next block staged while the current
    # one is summed: a single partial block, one full block plus a partial
    # one, and a long run ending in a partial block
    q, ang = _case(8, na, 18, 40)
    ang = ang * 0.9 + 0.05 * np.arange(na) ** 1.5  # uneven spacing
    N, Nz, cu, cv = 40, 9, 19.2, 8.6
    plan = tp.Plan(ang, 40, cu, N)
    got = to_host(tp.lamino_backproject(plan, to_dev(q), 0.9, cv, Nz)).astype(np.float64)
    want = oracle.lamino_backproject(q.astype(np.float64), ang, cu, cv, 0.9, N, Nz)
    assert rel_l2(got, want) < 1e-5
    assert np.max(np.abs(got - want)) < 1e-5 * np.max(np.abs(want))


@pytest.mark.parametrize("tilt", [0.05, 0.8, 2.4])
@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_lamino_reduced_precision_inputs(tp, storage, tilt):
    # FP16 projections are staged as raw FP16 pairs, BF16 as FP32 pairs; tilt
    # 0.05 needs windows of more than 32 rows (the rows past the ones loaded a
    # block ahead are staged after the barrier)
    import torch
    q, ang = _case(2, 24, 20, 40)
    N, Nz, cu, cv = 36, 8, 19.5, 9.5
    plan = tp.Plan(ang, 40, cu, N)
    dt = torch.float16 if storage == "f16" else torch.bfloat16
    qd = to_dev(q).to(dt)
    qr = to_host(qd).astype(np.float64)  # the rounded values the kernel reads
    got = to_host(tp.lamino_backproject(plan, qd, tilt, cv, Nz)).astype(np.float64)
    want = oracle.lamino_backproject(qr, ang, cu, cv, tilt, N, Nz)
    assert rel_l2(got, want) < 1e-5
    assert np.max(np.abs(got - want)) < 1e-5 * np.max(np.abs(want))


def test_lamino_tomography_tilt_matches_linear_backprojection(tp):
    # tilt pi/2 and an integer row centre: slice iz reads detector row
    # iz - Nz/2 + center_v, and the result is the tomographic backprojection
    q, ang = _case(3, 36, 12, 48)
    N, Nz, cu, cv = 48, 8, 23.7, 6.0
    plan = tp.Plan(ang, 48, cu, N)
    got = to_host(tp.lamino_backproject(plan, to_dev(q), math.pi / 2, cv, Nz)).astype(np.float64)
    rows = [iz - Nz // 2 + int(cv) for iz in range(Nz)]
    slab = np.ascontiguousarray(np.transpose(q[:, rows, :], (1, 0, 2)))  # [slices][angles][n]
    lin = to_host(tp.backproject(plan, to_dev(slab))).astype(np.float64)
    assert rel_l2(got, lin) < 1e-6


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_lamino_slice_ranges_bitwise(tp, storage):
    import torch
    q, ang = _case(4, 20, 16, 32)
    N, Nz, cu, cv = 32, 11, 15.5, 7.3
    plan = tp.Plan(ang, 32, cu, N)
    qd = to_dev(q) if storage == "f32" else to_dev(q).to(torch.float16)
    full = to_host(tp.lamino_backproject(plan, qd, 0.7, cv, Nz))
    for z0, nz in [(0, 3), (3, 5), (8, 3)]:
        part = to_host(tp.lamino_backproject(plan, qd, 0.7, cv, Nz, z0=z0, nz=nz))
        assert np.array_equal(part, full[z0:z0 + nz])


def test_lamino_large_detector_sampled(tp):
    # 1024 columns and rows, 64 angles, a 1024^2 x 8 slab: sampled voxels
    import torch
    q, ang = _case(5, 64, 256, 1024)
    N, Nz, cu, cv = 1024, 8, 511.5, 127.25
    plan = tp.Plan(ang, 1024, cu, N)
    note("lamino 64 x 256 x 1024 -> 8 x 1024^2")
    got = to_host(tp.lamino_backproject(plan, to_dev(q), 1.2, cv, Nz))
    rng = np.random.default_rng(6)
    ix, iy, iz = rng.integers(0, N, 200), rng.integers(0, N, 200), rng.integers(0, Nz, 200)
    want = oracle.lamino_backproject_points(q.astype(np.float64), ang, cu, cv, 1.2, N, Nz, ix, iy, iz)
    assert_parity(got[iz, iy, ix], want, "f32", label="lamino 1024 columns sampled")
    torch.cuda.empty_cache()


def test_lamino_argument_errors(tp):
    q, ang = _case(7, 8, 6, 16)
    plan = tp.Plan(ang, 16, 7.5, 16)
    qd = to_dev(q)
    for kw in (dict(tilt=0.0), dict(tilt=math.pi), dict(z0=4, nz=5)):
        args = dict(tilt=0.5, center_v=2.0, n_slices=8, z0=0, nz=None)
        args.update(kw)
        with pytest.raises(tp.TpError) as ei:
            tp.lamino_backproject(plan, qd, args["tilt"], args["center_v"], args["n_slices"], z0=args["z0"],
                                  nz=args["nz"])
        assert ei.value.status == tp.TP_EINVAL
