"""GPU parity of tp_backproject and tp_radon against the FP64 oracle, the exact
transposition of the pair, and the bitwise invariance under tuning."""
import math

import numpy as np
import pytest

import oracle
from paper_2209_08450_amd import synth
from tests._util import F16_MODE_MAX_REL, F16_MODE_REL_L2, assert_parity, note, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_08450_amd import tp as mod
    return mod


GEOMS = [
    # (n_angles, n_det, n_vox, center, rows)
    (180, 256, 256, 128.0, 5),     # several tiles, ragged slice group
    (37, 100, 90, 47.3, 3),        # odd angles, ragged tiles, N != n
    (16, 64, 64, 29.75, 9),
    (1, 40, 33, 19.0, 1),
    (64, 128, 160, 64.0, 2),       # image larger than the detector: off-detector taps
    (24, 70, 70, 200.0, 2),        # axis far off the detector
]


@pytest.mark.parametrize("g", GEOMS)
def test_backproject_matches_oracle(tp, g):
    na, n, N, c, rows = g
    rng = np.random.default_rng(na * 7 + n)
    ang = synth.uniform_angles(na) + 0.013
    q = rng.standard_normal((rows, na, n))
    plan = tp.Plan(ang, n, c, N)
    note(f"backproject f32 {g}")
    got = to_host(tp.backproject(plan, to_dev(q.astype(np.float32))))
    want = oracle.backproject(q.astype(np.float32).astype(np.float64), ang, c, N)
    assert got.shape == want.shape
    if np.linalg.norm(want) == 0:  # every ray misses the detector
        assert np.all(got == 0)
    else:
        assert_parity(got, want, "f32", label=f"backproject {g}")


@pytest.mark.parametrize("g", GEOMS)
def test_backproject_f16_rows_match_oracle_16bit_mode(tp, g):
    """FP16 rows (the v_dot2 kernel, pair staging with its detector-edge path)
    against the oracle's 16-bit mode on the same stored rows."""
    na, n, N, c, rows = g
    rng = np.random.default_rng(na * 5 + n)
    ang = synth.uniform_angles(na) + 0.021
    q = to_dev(rng.standard_normal((rows, na, n)).astype(np.float32)).half()
    stored = to_host(q).astype(np.float64)
    plan = tp.Plan(ang, n, c, N)
    note(f"backproject f16 {g}")
    got = to_host(tp.backproject(plan, q))
    want = oracle.backproject(stored, ang, c, N, weights="f16")
    # one angle: a voxel is a single term, so a weight that rounds to the
    # neighbouring FP16 value moves it by up to 2^-11 of a tap (no averaging)
    mx = F16_MODE_MAX_REL if na > 1 else 2.0 ** -9
    if np.linalg.norm(want) == 0:  # every ray misses the detector
        assert np.all(got == 0)
    else:
        assert_parity(got, want, "f32", rel=F16_MODE_REL_L2, mx=mx, label=f"backproject f16 {g}")


def test_backproject_constant_rows_give_pi(tp):
    na, n = 90, 128
    ang = synth.uniform_angles(na)
    plan = tp.Plan(ang, n, n / 2)
    note("backproject q=1")
    f = to_host(tp.backproject(plan, to_dev(np.ones((2, na, n), np.float32))))
    yy, xx = np.mgrid[0:n, 0:n]
    inner = np.hypot(xx - n // 2, yy - n // 2) < n / 2 - 2
    assert np.max(np.abs(f[:, inner] - math.pi)) < 2e-6


@pytest.mark.parametrize("dt", ["f16", "bf16"])
def test_backproject_half_storage(tp, dt):
    import torch
    na, n, N, c = 45, 96, 96, 47.5
    rng = np.random.default_rng(5)
    ang = synth.uniform_angles(na)
    q = rng.standard_normal((3, na, n)).astype(np.float32)
    t = to_dev(q).to(tp.torch_dtype(tp.dtype_code(dt)))
    stored = to_host(t).astype(np.float64)
    plan = tp.Plan(ang, n, c, N)
    note(f"backproject {dt}")
    got = to_host(tp.backproject(plan, t))
    if dt == "f16":
        # FP16 rows run the 16-bit mode: interpolation weights held in binary16
        want = oracle.backproject(stored, ang, c, N, weights="f16")
        assert_parity(got, want, "f32", rel=F16_MODE_REL_L2, mx=F16_MODE_MAX_REL, label="backproject f16 rows")
    else:
        assert_parity(got, oracle.backproject(stored, ang, c, N), "f32", label=f"backproject {dt} rows")
    torch.cuda.synchronize()


def test_backproject_accumulate_and_scale(tp):
    import torch
    na, n = 20, 64
    rng = np.random.default_rng(6)
    ang = synth.uniform_angles(na)
    q = rng.standard_normal((2, na, n)).astype(np.float32)
    plan = tp.Plan(ang, n, 31.5)
    note("backproject accumulate")
    out = torch.full((2, n, n), 3.0, device="cuda")
    tp.backproject(plan, to_dev(q), scale=0.5, out=out, accumulate=True)
    want = 3.0 + oracle.backproject(q.astype(np.float64), ang, 31.5, n, scale=0.5)
    assert rel_l2(to_host(out), want) < 1e-6


def test_tuning_variants_are_bitwise_identical(tp):
    import torch

    from paper_2209_08450_amd import tune
    na, n, N, c, rows = 70, 120, 110, 61.2, 11
    rng = np.random.default_rng(8)
    ang = synth.uniform_angles(na) + 0.2
    q32 = to_dev(rng.standard_normal((rows, na, n)).astype(np.float32))
    plan = tp.Plan(ang, n, c, N)
    for st, q in (("f32", q32), ("f16", q32.half()), ("bf16", q32.bfloat16())):
        ref = None
        for k in (1, 2, 4, 8, 16):
            for a in (8, 16, 32, 64):
                try:
                    plan.set_tuning(st, k, a)
                except tp.TpError:
                    # rejected only when the staged block exceeds the LDS
                    assert not tune.legal(st, k, a)
                    continue
                assert plan.get_tuning(st) == (k, a)
                note(f"backproject {st} tuning K={k} A={a}")
                f = tp.backproject(plan, q)
                torch.cuda.synchronize()
                if ref is None:
                    ref = f.clone()
                else:
                    assert torch.equal(f, ref), (st, k, a)


@pytest.mark.parametrize("g", GEOMS)
def test_radon_matches_oracle(tp, g):
    na, n, N, c, rows = g
    rng = np.random.default_rng(na + 3 * n)
    ang = synth.uniform_angles(na) + 0.013
    x = rng.standard_normal((rows, N, N)).astype(np.float32)
    plan = tp.Plan(ang, n, c, N)
    note(f"radon {g}")
    got = to_host(tp.radon(plan, to_dev(x)))
    want = oracle.radon(x.astype(np.float64), ang, c, n)
    if np.linalg.norm(want) == 0:
        assert np.all(got == 0)
    else:
        assert_parity(got, want, "f32", label=f"radon {g}")


@pytest.mark.parametrize("g", GEOMS[:3])
def test_adjoint_dot_product(tp, g):
    na, n, N, c, rows = g
    rng = np.random.default_rng(17)
    ang = synth.uniform_angles(na) + 0.013
    x = rng.standard_normal((rows, N, N)).astype(np.float32)
    y = rng.standard_normal((rows, na, n)).astype(np.float32)
    plan = tp.Plan(ang, n, c, N)
    note(f"adjoint {g}")
    Rx = to_host(tp.radon(plan, to_dev(x))).astype(np.float64)
    Rty = to_host(tp.backproject(plan, to_dev(y), scale=1.0)).astype(np.float64)
    lhs = np.vdot(Rx, y.astype(np.float64))
    rhs = np.vdot(x.astype(np.float64), Rty)
    assert abs(lhs - rhs) / max(abs(lhs), abs(rhs)) < 1e-5


def test_radon_is_exact_transpose_of_backproject(tp):
    # Build both system matrices from unit vectors: with one nonzero input the
    # FP32 sums are exact, so the matrices must agree bitwise.
    N, n, na, c = 12, 18, 5, 8.6
    ang = synth.uniform_angles(na) + 0.1
    plan = tp.Plan(ang, n, c, N)
    units_img = np.eye(N * N, dtype=np.float32).reshape(N * N, N, N)
    units_sino = np.eye(na * n, dtype=np.float32).reshape(na * n, na, n)
    note("transpose check")
    A_radon = to_host(tp.radon(plan, to_dev(units_img))).reshape(N * N, na * n)      # rows: voxels
    A_bp = to_host(tp.backproject(plan, to_dev(units_sino), scale=1.0)).reshape(na * n, N * N)
    assert np.array_equal(A_radon, A_bp.T)
    # and both equal the FP64 hat weights up to FP32 rounding of (1-w, w)
    A64 = oracle.radon(np.eye(N * N).reshape(N * N, N, N), ang, c, n).reshape(N * N, na * n)
    assert np.max(np.abs(A_radon - A64)) < 1e-5


def test_radon_mass_conservation(tp):
    N, n, na = 64, 128, 33
    rng = np.random.default_rng(19)
    f = rng.uniform(0, 1, (2, N, N)).astype(np.float32)
    plan = tp.Plan(synth.uniform_angles(na), n, n / 2, N)
    note("radon mass")
    r = to_host(tp.radon(plan, to_dev(f))).astype(np.float64)
    assert np.allclose(r.sum(axis=2), f.astype(np.float64).sum(axis=(1, 2))[:, None], rtol=2e-6)


def test_radon_sparse_angles_use_global_fallback(tp):
    # 8 angles over 180 degrees on a 512^2 image: the strip a work-group's
    # angles cross is far wider than the LDS buffer, so candidates are read
    # from global memory; results must match the oracle all the same
    N = n = 512
    ang = synth.uniform_angles(8) + 0.05
    rng = np.random.default_rng(23)
    x = rng.standard_normal((2, N, N)).astype(np.float32)
    plan = tp.Plan(ang, n, n / 2 + 0.3, N)
    note("radon sparse angles (global fallback)")
    got = to_host(tp.radon(plan, to_dev(x)))
    assert_parity(got, oracle.radon(x.astype(np.float64), ang, n / 2 + 0.3, n), "f32", label="radon sparse")


def test_radon_mixed_narrow_and_wide_strips(tp):
    # 40 angles within 0.1 rad (narrow strips, summed through LDS) and 8
    # spread over 2 rad (strips wider than the LDS buffer, summed from global
    # memory) in one plan, ragged bins (330 = 5 x 64 + 10): both kernels of one
    # call write their own work-groups.  20 slices use groups of 8 angles, 3
    # slices groups of 4; the slices both calls share are bitwise equal.
    N, n = 300, 330
    rng = np.random.default_rng(37)
    ang = np.concatenate([0.2 + 0.1 * rng.random(40), np.linspace(0.9, 2.9, 8)])
    c = 161.3
    plan = tp.Plan(ang, n, c, N)
    x = rng.standard_normal((20, N, N)).astype(np.float32)
    note("radon mixed narrow/wide strips, 20 slices")
    got = to_host(tp.radon(plan, to_dev(x)))
    assert_parity(got, oracle.radon(x.astype(np.float64), ang, c, n), "f32", label="radon mixed strips")
    note("radon mixed narrow/wide strips, 3 slices")
    got3 = to_host(tp.radon(plan, to_dev(x[:3])))
    assert np.array_equal(got3, got[:3])


def test_radon_widest_slices_group_four_angles(tp):
    # 32000-voxel slices: with 32-slice groups the tile tables of 8 angles
    # would take a work-group past the 160 KB of LDS, so the projector groups
    # 4 angles there.  17 slices of a sparse volume (70 GB; every angle sweeps
    # rows, so no transposed copy); 4 angles within 1.5 mrad (one group whose
    # strips fit LDS) and 2 angles 0.05 rad apart (one group of wide strips,
    # read from global memory).  Each voxel's weights are the FP64 oracle's
    # system-matrix entries: its backprojection of a one-hot sinogram at that
    # voxel (scale 1, the exact transpose).
    import torch
    N, n = 32000, 8192  # the detector is limited by the filter's pad length
    rows = 17
    ang = np.array([0.1, 0.1005, 0.101, 0.1015, 0.5, 0.55])
    c = n / 2 + 0.25
    plan = tp.Plan(ang, n, c, N)
    assert plan.radon_workspace_bytes(rows) == 0
    pts = [(0, 16000, 16000, 1.0), (3, 13300, 18700, 2.5), (16, 18500, 14100, -1.5), (9, 17000, 15500, 0.75)]
    note("radon 17 x 32000^2 sparse, 6 angles x 8192 bins")
    torch.cuda.empty_cache()
    x = torch.zeros((rows, N, N), dtype=torch.float32, device="cuda")
    for z, iy, ix, v in pts:
        x[z, iy, ix] = v
    got = tp.radon(plan, x).cpu().numpy().astype(np.float64)
    del x
    torch.cuda.empty_cache()
    want = np.zeros((rows, len(ang), n))
    for z, iy, ix, v in pts:
        for a, t in enumerate(ang):
            s = (ix - N // 2) * math.cos(t) + (iy - N // 2) * math.sin(t) + c
            for j in range(math.floor(s) - 1, math.floor(s) + 3):
                if 0 <= j < n:
                    q = np.zeros((len(ang), n))
                    q[a, j] = 1.0
                    want[z, a, j] += v * oracle.backproject_points(q, ang, c, N, [ix], [iy], scale=1.0)[0]
    assert np.count_nonzero(want) >= 2 * len(ang) * len(pts) - 4
    # FP32 weights from the split coordinate: a few ulp of the weights
    assert np.max(np.abs(got - want)) < 1e-5 * 2.5


def test_unsorted_nonuniform_angles(tp):
    # arbitrary order, full circle, repeated angle: the plan's grouping of
    # angles by sweep axis must not change either projector's results
    N, n = 96, 110
    rng = np.random.default_rng(29)
    ang = rng.uniform(0, 2 * math.pi, 41)
    ang[7] = ang[3]
    c = 54.6
    plan = tp.Plan(ang, n, c, N)
    x = rng.standard_normal((3, N, N)).astype(np.float32)
    q = rng.standard_normal((3, 41, n)).astype(np.float32)
    note("unsorted angles")
    assert_parity(to_host(tp.radon(plan, to_dev(x))), oracle.radon(x.astype(np.float64), ang, c, n), "f32",
                  label="radon unsorted angles")
    assert_parity(to_host(tp.backproject(plan, to_dev(q), scale=1.0)),
                  oracle.backproject(q.astype(np.float64), ang, c, N, scale=1.0), "f32",
                  label="backproject unsorted angles")


def test_backproject_more_than_4gb_of_rows(tp):
    # 16 slices of 17477 angles x 8192 columns in f16: one slice group spans
    # 4.6 GB of filtered rows, past 32-bit byte offsets.  Checked against the
    # oracle at sampled voxels of the first and the last slice.
    import torch
    na, n, rows = 17477, 8192, 16
    ang = synth.uniform_angles(na)
    plan = tp.Plan(ang, n, n / 2.0)
    assert plan.get_tuning("f16")[0] == 16
    g = torch.Generator(device="cuda").manual_seed(31)
    q = torch.randn((rows, na, n), generator=g, device="cuda").half()
    note("backproject 16 x 17477 x 8192 f16")
    vol = tp.backproject(plan, q)
    rng = np.random.default_rng(31)
    ix = rng.integers(0, n, 48)
    iy = rng.integers(0, n, 48)
    for z in (0, rows - 1):
        qz = q[z].cpu().numpy().astype(np.float64)
        want = oracle.backproject_points(qz, ang, n / 2.0, n, ix, iy, weights="f16")
        got = vol[z].cpu().numpy()[iy, ix].astype(np.float64)
        # FP32 sums of 17477 random terms with binary16 weights rounded from
        # the kernel's FP32 coordinate (F16_MODE_*); an addressing mistake
        # would be O(1)
        assert_parity(got, want, "f32", rel=F16_MODE_REL_L2, mx=F16_MODE_MAX_REL,
                      label=f"backproject >4 GB rows, slice {z}")
    del q, vol
    torch.cuda.empty_cache()


def test_radon_workspace_contract(tp):
    import torch
    na, n, rows = 30, 64, 3
    rng = np.random.default_rng(41)
    ang = synth.uniform_angles(na)
    plan = tp.Plan(ang, n, 31.5)
    x = to_dev(rng.standard_normal((rows, n, n)).astype(np.float32))
    need = plan.radon_workspace_bytes(rows)
    assert need == rows * n * n * 4  # a transposed copy: some angles sweep columns
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    note("radon explicit workspace")
    ref = tp.radon(plan, x)
    assert torch.equal(tp.radon(plan, x, workspace=ws), ref)
    with pytest.raises(tp.TpError, match="workspace"):
        tp.radon(plan, x, workspace=ws[: need // 2])
    with pytest.raises(tp.TpError, match="overlaps"):
        tp.radon(plan, x, workspace=x.view(torch.uint8).reshape(-1))
    # every angle within 45 degrees of the x axis: no transpose, no workspace
    ang2 = np.linspace(-0.7, 0.7, 25)
    plan2 = tp.Plan(ang2, n, 31.5)
    assert plan2.radon_workspace_bytes(rows) == 0
    note("radon without workspace")
    got = to_host(tp.radon(plan2, x)).astype(np.float64)
    want = oracle.radon(to_host(x).astype(np.float64), ang2, 31.5, n)
    assert_parity(got, want, "f32", label="radon without workspace")
    torch.cuda.synchronize()


def test_radon_32_slice_groups(tp):
    # more than 16 rows take 32 slices per work-group: one full group and a
    # partial one (40 = 32 + 8), angles sweeping both rows and columns
    na, n, rows = 50, 96, 40
    rng = np.random.default_rng(43)
    ang = synth.uniform_angles(na) + 0.05
    plan = tp.Plan(ang, n, 47.3)
    x = rng.standard_normal((rows, n, n)).astype(np.float32)
    note("radon 40 rows (32-slice groups)")
    got = to_host(tp.radon(plan, to_dev(x))).astype(np.float64)
    want = oracle.radon(x.astype(np.float64), ang, 47.3, n)
    assert_parity(got, want, "f32", label="radon 40 rows")
    for z in (0, 31, 32, 39):
        assert rel_l2(got[z], want[z]) < 1e-5, z
    # each slice alone gives the same bits as inside the group
    one = to_host(tp.radon(plan, to_dev(np.ascontiguousarray(x[33:34])))).astype(np.float64)
    assert np.array_equal(one[0], got[33])


def test_projector_pair_differentiation_shape(tp):
    # the least-squares workload's calls: 128 slices of 1024^2 from 900 angles
    # (four 32-slice groups per launch), random volume; two whole slices of
    # R f (the first and the last of the call) against the oracle, and the
    # adjoint on the same shape by the dot-product identity
    import torch
    na, n, rows = 900, 1024, 128
    ang = synth.uniform_angles(na)
    plan = tp.Plan(ang, n, 511.5)
    gen = torch.Generator(device="cuda").manual_seed(44)
    x = torch.randn((rows, n, n), generator=gen, device="cuda")
    note("radon 128 x 1024^2 x 900")
    r = tp.radon(plan, x)
    zs = [0, rows - 1]
    xs = x[zs].cpu().numpy().astype(np.float64)
    got = r[zs].cpu().numpy().astype(np.float64)
    want = oracle.radon(xs, ang, 511.5, n)
    errs = [rel_l2(got[i], want[i]) for i in range(len(zs))]
    note(f"radon rel-L2 {errs}")
    assert max(errs) < 1e-5
    assert_parity(got, want, "f32", label="radon 128 x 1024^2 x 900, first and last slices")
    # <R x, y> = <x, R^T y> over the whole call with y = R x (both sides are
    # |R x|^2, far from zero, so FP32 rounding stays a small relative error);
    # sums in FP64
    bt = tp.backproject(plan, r, scale=1.0)
    lhs = float(torch.sum(r.double() * r.double()))
    rhs = float(torch.sum(x.double() * bt.double()))
    note(f"dot products {lhs} {rhs}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    del x, r, bt
    torch.cuda.empty_cache()
