"""GPU parity of the log-polar FBP (tp_lprec_fbp_chunk: normalise -> pad ->
filter -> half-sample row splines -> log-radial resampling -> convolution over
(angle, log-radius) by FFTs -> spline evaluation at the voxels) against the
FP64 oracle of the same method (oracle/lprec.py), and against the direct sum
of trigonometric interpolants it approximates."""
import math

import numpy as np
import pytest

import oracle
from oracle import lprec as olp
from paper_2209_08450_amd import synth
from tests._util import assert_parity, note, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_08450_amd import tp as mod
    return mod


@pytest.fixture(scope="module")
def scan96():
    # 5 rows: the last pair holds one slice
    return synth.phantom_2d_scan(seed=3, n_rows=5, n_angles=120, n_det=96, center=46.7)


def _angles(na, theta0):
    return theta0 + np.arange(na) * math.pi / na


def _run(tp, s, angles, n_vox=0, kind="ramp", spans=0, os=0.0, eps=0.0, workspace_bytes=None, plan=None):
    import torch
    plan = plan or tp.Plan(angles, s.proj.shape[2], s.center, n_vox)
    ws = None
    if workspace_bytes is not None:
        ws = torch.empty(workspace_bytes, dtype=torch.uint8, device="cuda")
    out = tp.lprec_fbp_chunk(plan, to_dev(s.proj), to_dev(s.dark), to_dev(s.flat), workspace=ws, kind=kind,
                             spans=spans, os=os, eps=eps)
    torch.cuda.synchronize()
    return to_host(out).astype(np.float64)


def _oracle(s, rows, theta0, N=None, kind="ramp", spans=3, os=1.0, eps=1.0):
    return olp.lprec_fbp(s.proj[:, rows], s.dark[:, rows], s.flat[:, rows], theta0, s.center, N, kind=kind,
                         spans=spans, os=os, eps=eps)


def test_grid_query_matches_oracle_sizing(tp):
    for args in [(2048, 2048, 3, 1.2, 0.5), (120, 96, 3, 1.2, 0.5), (120, 96, 2, 1.0, 0.3), (64, 80, 4, 2.0, 1.0)]:
        g = tp.lprec_grid(*args)
        o = olp.lprec_params(*args)
        for k, v in g.items():
            if k in o:
                assert v == o[k], (args, k, v, o[k])


@pytest.mark.parametrize("spans,os,eps", [(3, 1.0, 1.0), (3, 1.2, 0.5), (2, 1.0, 0.3), (4, 2.0, 1.0)])
def test_lprec_matches_oracle_full_slices(tp, scan96, spans, os, eps):
    ang = _angles(120, 0.3)
    note(f"lprec 120x5x96 centre 46.7, spans {spans} os {os} eps {eps}")
    got = _run(tp, scan96, ang, spans=spans, os=os, eps=eps)
    want = _oracle(scan96, slice(0, 5), 0.3, spans=spans, os=os, eps=eps)
    assert_parity(got, want, "f32", label=f"lprec spans {spans}")


@pytest.mark.parametrize("kind", ["shepp", "parzen"])
def test_lprec_windows(tp, scan96, kind):
    ang = _angles(120, 0.0)
    note(f"lprec {kind} 120x5x96")
    got = _run(tp, scan96, ang, kind=kind)
    want = _oracle(scan96, slice(0, 5), 0.0, kind=kind)
    assert_parity(got, want, "f32", label=f"lprec {kind}")


@pytest.mark.parametrize("n_vox", [64, 130])
def test_lprec_voxel_grid_sizes(tp, scan96, n_vox):
    ang = _angles(120, -0.7)
    note(f"lprec N={n_vox} from 96 columns")
    got = _run(tp, scan96, ang, n_vox=n_vox)
    want = _oracle(scan96, slice(0, 5), -0.7, N=n_vox)
    assert_parity(got, want, "f32", label=f"lprec N={n_vox}")


def test_lprec_uneven_span_slots(tp):
    """100 angles over 3 spans: the last span has an empty slot."""
    s = synth.phantom_2d_scan(seed=5, n_rows=2, n_angles=100, n_det=64, center=32.0)
    ang = _angles(100, 1.1)
    note("lprec 100x2x64, spans 3 (34 + 34 + 32 slots used)")
    got = _run(tp, s, ang)
    want = _oracle(s, slice(0, 2), 1.1)
    assert_parity(got, want, "f32", label="lprec uneven spans")


def test_lprec_multi_pass_equals_one_pass(tp, scan96):
    """A workspace for one pair runs the rows in three passes; every pass
    computes each pair alone, so the slices are bitwise those of one pass."""
    ang = _angles(120, 0.3)
    plan = tp.Plan(ang, 96, scan96.center)
    one = _run(tp, scan96, ang, plan=plan)
    small = plan.lprec_workspace_bytes(2)
    note(f"lprec multi-pass, workspace {small} bytes")
    multi = _run(tp, scan96, ang, plan=plan, workspace_bytes=small + 4096)
    assert np.array_equal(one, multi)


def test_lprec_near_direct_sum(tp):
    """Against the sum it approximates (every ray read by the trigonometric
    interpolant of its row): within the FP16-regime bar at the default grid,
    256 columns x 180 angles (the 16-slice workload's geometry)."""
    s = synth.phantom_2d_scan(seed=1, n_rows=3, n_angles=180, n_det=256)
    ang = _angles(180, 0.0)
    note("lprec 180x3x256 vs direct sum")
    got = _run(tp, s, ang)
    want = oracle.fourier_fbp(s.proj, s.dark, s.flat, ang, s.center)
    errs = [rel_l2(got[z], want[z]) for z in range(3)]
    note(f"rel-L2 vs direct sum per slice {errs}")
    assert max(errs) < 3e-3


def test_lprec_paper_scale_sampled(tp):
    """2048 angles x 2048 columns (the 2048^3 workload's geometry), 4 rows of
    the 12-bit ellipsoid scan: sampled voxels against the direct sum, within
    half the FP16-regime bar (the default grid measures about 9e-4)."""
    import torch
    n, na = 2048, 2048
    rows = [1021, 1022, 1023, 1024]
    s = synth.ellipsoid_scan_np(seed=2, n_angles=na, n_rows=n, n_det=n, rows=rows)
    plan = tp.Plan(s.angles, n, s.center)
    note("lprec 2048 x 4 rows x 2048 (default grid)")
    out = tp.lprec_fbp_chunk(plan, to_dev(s.proj), to_dev(s.dark), to_dev(s.flat))
    torch.cuda.synchronize()
    got = to_host(out).astype(np.float64)
    rng = np.random.default_rng(9)
    e_all = []
    for z in (0, 3):
        ix = rng.integers(0, n, 160)
        iy = rng.integers(0, n, 160)
        want = oracle.fourier_fbp_points(s.proj[:, z], s.dark[:, z], s.flat[:, z], s.angles, s.center, n, ix, iy)
        e = rel_l2(got[z, iy, ix], want)
        note(f"row {rows[z]}: rel-L2 vs direct sum at 160 voxels {e:.3e}")
        e_all.append(e)
    assert max(e_all) < 1.5e-3


def test_lprec_host_errors(tp, scan96):
    import torch
    ang = _angles(120, 0.3)
    plan = tp.Plan(ang, 96, scan96.center)
    p, d, f = to_dev(scan96.proj), to_dev(scan96.dark), to_dev(scan96.flat)
    with pytest.raises(tp.TpError, match="spans"):
        tp.lprec_fbp_chunk(plan, p, d, f, spans=5)
    with pytest.raises(tp.TpError, match="oversampling"):
        tp.lprec_fbp_chunk(plan, p, d, f, os=20.0)
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(tp.TpError, match="workspace"):
        tp.lprec_fbp_chunk(plan, p, d, f, workspace=ws)
    bad = ang.copy()
    bad[7] += 1e-3
    plan2 = tp.Plan(bad, 96, scan96.center)
    with pytest.raises(tp.TpError, match="equally spaced"):
        tp.lprec_fbp_chunk(plan2, p, d, f)
    torch.cuda.synchronize()
