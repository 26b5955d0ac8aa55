"""GPU parity of the Fourier-domain FBP (tp_fourier_fbp_chunk: normalise ->
pad -> filter -> polar spectra -> Gaussian gather onto a Cartesian frequency
grid -> 2-D inverse FFT -> deconvolution) against the FP64 oracle's direct
sum of trigonometric interpolants."""
import math

import numpy as np
import pytest

import oracle
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
def scan64():
    return synth.phantom_2d_scan(seed=3, n_rows=7, n_angles=90, n_det=64, center=31.3)


def _run(tp, s, angles=None, n_vox=0, kind="ramp", half_width=0, workspace_bytes=None, plan=None):
    import torch
    ang = s.angles if angles is None else angles
    plan = plan or tp.Plan(ang, s.proj.shape[2], s.center, n_vox)
    rows = s.proj.shape[1]
    ws = None
    if workspace_bytes is not None:
        ws = torch.empty(workspace_bytes, dtype=torch.uint8, device="cuda")
    out = tp.fourier_fbp_chunk(plan, to_dev(s.proj), to_dev(s.dark), to_dev(s.flat), workspace=ws, kind=kind,
                               half_width=half_width)
    torch.cuda.synchronize()
    return to_host(out).astype(np.float64)


def _oracle(s, rows, angles=None, N=None, kind="ramp"):
    ang = s.angles if angles is None else angles
    return oracle.fourier_fbp(s.proj[:, rows], s.dark[:, rows], s.flat[:, rows], ang, s.center, N, kind=kind)


def test_fourier_matches_oracle_full_slices(tp, scan64):
    note("fourier ramp 90x7x64, centre 31.3")
    got = _run(tp, scan64)
    want = _oracle(scan64, slice(0, 7))
    errs = [rel_l2(got[z], want[z]) for z in range(7)]  # odd count: the last slice has a zero partner
    note(f"rel-L2 per slice {errs}")
    assert max(errs) < 1e-5
    assert_parity(got, want, "f32", label="fourier 90x7x64")


@pytest.mark.parametrize("kind", ["shepp", "parzen"])
def test_fourier_windows(tp, scan64, kind):
    note(f"fourier {kind} 90x7x64")
    got = _run(tp, scan64, kind=kind)
    want = _oracle(scan64, slice(0, 7), kind=kind)
    assert_parity(got, want, "f32", label=f"fourier {kind}")


def test_fourier_angles_over_full_circle_and_negative(tp, scan64):
    # Angles in [-pi, 2 pi), unsorted and uneven: the plan reduces them modulo
    # pi, reverses the rows of those reduced by an odd multiple of pi, and
    # sorts them for the gather.
    rng = np.random.default_rng(11)
    ang = rng.uniform(-math.pi, 2 * math.pi, 90)
    note("fourier 90 random angles in [-pi, 2pi)")
    got = _run(tp, scan64, angles=ang)
    want = _oracle(scan64, slice(0, 7), angles=ang)
    assert_parity(got, want, "f32", label="fourier random angles")


@pytest.mark.parametrize("n_vox", [48, 100])
def test_fourier_voxel_grid_sizes(tp, scan64, n_vox):
    # 48: grid side = pad length (one grid point per frequency sample);
    # 100: grid side 256 = 2 x pad length (two grid points per sample)
    note(f"fourier n_vox {n_vox}")
    got = _run(tp, scan64, n_vox=n_vox)
    want = _oracle(scan64, slice(0, 7), N=n_vox)
    assert got.shape == (7, n_vox, n_vox)
    assert_parity(got, want, "f32", label=f"fourier n_vox {n_vox}")


@pytest.mark.parametrize("n,rows,center", [(63, 3, 30.0), (100, 1, 61.7), (64, 2, 20.25)])
def test_fourier_detector_widths_and_axes(tp, n, rows, center):
    # odd width (pad offset (L - n) / 2 rounds down), a width that is not a
    # power of two with a single row (its partner is zero), an axis far from
    # the detector centre
    s = synth.phantom_2d_scan(seed=9, n_rows=rows, n_angles=72, n_det=n, center=center)
    note(f"fourier n={n} rows={rows} centre={center}")
    got = _run(tp, s)
    want = _oracle(s, slice(0, rows))
    assert_parity(got, want, "f32", label=f"fourier n={n} rows={rows}")


def test_fourier_passes_bitwise(tp, scan64):
    plan = tp.Plan(scan64.angles, 64, scan64.center)
    one = _run(tp, scan64, plan=plan)
    # room for one pair of rows per pass (plus the dark/flat tables of all 7 rows)
    need = plan.fourier_workspace_bytes(2) - tp._normalize_ws(2, 64) + tp._normalize_ws(7, 64)
    note("fourier multi-pass workspace")
    several = _run(tp, scan64, plan=plan, workspace_bytes=need + 4096)
    assert np.array_equal(one, several)


def test_fourier_deterministic(tp, scan64):
    plan = tp.Plan(scan64.angles, 64, scan64.center)
    a = _run(tp, scan64, plan=plan)
    b = _run(tp, scan64, plan=plan)
    assert np.array_equal(a, b)


def test_fourier_half_width_accuracy(tp, scan64):
    want = _oracle(scan64, slice(0, 7))
    errs = {}
    for hw in (3, 4, 5, 6, 8):
        note(f"fourier half width {hw}")
        errs[hw] = rel_l2(_run(tp, scan64, half_width=hw), want)
    note(f"rel-L2 by half width {errs}")
    assert errs[3] > errs[4] > errs[5]
    assert errs[3] > 10 * errs[6]
    assert errs[6] < 1e-5 and errs[8] < 1e-5


def test_fourier_paper_geometry_sampled(tp):
    # 2048 angles x 2048 columns (grid side 4096, pad length 4096), three rows
    # of the 12-bit ellipsoid scan: an odd count, so the last row is unpaired.
    import torch
    rows = [700, 701, 1400]
    s = synth.ellipsoid_scan_np(2, 2048, 2048, 2048, rows=rows)
    note("fourier 2048 angles x 3 rows x 2048")
    got = _run(tp, s)
    rng = np.random.default_rng(12)
    ix = rng.integers(0, 2048, 40)
    iy = rng.integers(0, 2048, 40)
    errs = []
    for i in range(3):
        want = oracle.fourier_fbp_points(s.proj[:, i], s.dark[:, i], s.flat[:, i], s.angles, s.center, 2048,
                                         ix, iy)
        errs.append(rel_l2(got[i, iy, ix], want))
        assert_parity(got[i, iy, ix], want, "f32", label=f"fourier paper geometry row {rows[i]}")
    note(f"rel-L2 at sampled voxels {errs}")
    assert max(errs) < 1e-5, errs
    torch.cuda.empty_cache()


def test_fourier_bench_launch_shape_sampled(tp):
    """The launch the benchmark times: one 256-row chunk of 2048 angles x 2048
    columns (128 slice pairs in one pass, grid side 4096) of a 12-bit
    ellipsoid scan generated on the GPU; three rows spread over the chunk
    checked at 40 sampled voxels each against the oracle's direct sum."""
    import torch
    s = synth.ellipsoid_scan_torch(seed=6, n_angles=2048, n_rows=256, n_det=2048, device="cuda", center=1024.0)
    rows = [0, 129, 255]
    host = {name: getattr(s, name)[:, rows].cpu().numpy().view(np.uint16) for name in ("proj", "dark", "flat")}
    plan = tp.Plan(s.angles, 2048, s.center)
    note("fourier 2048 x 256 x 2048")
    vol = tp.fourier_fbp_chunk(plan, s.proj, s.dark, s.flat)
    got = vol[rows].cpu().numpy().astype(np.float64)
    del vol
    torch.cuda.empty_cache()
    rng = np.random.default_rng(13)
    errs = []
    for i in range(len(rows)):
        ix, iy = rng.integers(0, 2048, 40), rng.integers(0, 2048, 40)
        want = oracle.fourier_fbp_points(host["proj"][:, i], host["dark"][:, i], host["flat"][:, i], s.angles,
                                         s.center, 2048, ix, iy)
        errs.append(rel_l2(got[i, iy, ix], want))
        assert_parity(got[i, iy, ix], want, "f32", label=f"fourier bench chunk row {rows[i]}")
    note(f"rel-L2 at sampled voxels {errs}")
    assert max(errs) < 1e-5, errs
    plan.close()


@pytest.mark.parametrize("n", [512, 4096])
def test_fourier_register_transform_sizes(tp, n):
    # pad length and grid side 1024 (n = 512) and 8192 (n = 4096): the
    # register-resident transforms at their smallest and largest lengths
    import torch
    s = synth.phantom_2d_scan(seed=5, n_rows=2, n_angles=96, n_det=n, center=n / 2 - 0.25)
    note(f"fourier 96 angles x 2 rows x {n}")
    got = _run(tp, s)
    rng = np.random.default_rng(13)
    ix = rng.integers(0, n, 48)
    iy = rng.integers(0, n, 48)
    errs = []
    for i in range(2):
        want = oracle.fourier_fbp_points(s.proj[:, i], s.dark[:, i], s.flat[:, i], s.angles, s.center, n, ix, iy)
        errs.append(rel_l2(got[i, iy, ix], want))
        assert_parity(got[i, iy, ix], want, "f32", label=f"fourier n={n} row {i}")
    note(f"rel-L2 at sampled voxels {errs}")
    assert max(errs) < 1e-5, errs
    torch.cuda.empty_cache()


def test_fourier_widest_detector(tp):
    # 8192 columns: pad length and grid side 16384, the largest supported
    # (LDS transforms with 1024 threads and 128 KB of LDS), one row
    import torch
    s = synth.phantom_2d_scan(seed=6, n_rows=1, n_angles=24, n_det=8192, center=4095.5)
    note("fourier 24 angles x 1 row x 8192")
    got = _run(tp, s)
    rng = np.random.default_rng(14)
    ix = rng.integers(0, 8192, 48)
    iy = rng.integers(0, 8192, 48)
    want = oracle.fourier_fbp_points(s.proj[:, 0], s.dark[:, 0], s.flat[:, 0], s.angles, s.center, 8192, ix, iy)
    assert_parity(got[0, iy, ix], want, "f32", label="fourier widest detector")
    torch.cuda.empty_cache()


def test_fourier_close_to_linear_interpolation_fbp(tp, scan64):
    # sanity: the two interpolations differ by the linear interpolation's
    # smoothing only
    plan = tp.Plan(scan64.angles, 64, scan64.center)
    fr = _run(tp, scan64, plan=plan)
    lin = to_host(tp.fbp_chunk(plan, to_dev(scan64.proj), to_dev(scan64.dark), to_dev(scan64.flat), "f32"))
    assert rel_l2(lin, fr) < 0.15


def test_fourier_argument_errors(tp, scan64):
    import ctypes
    import torch
    plan = tp.Plan(scan64.angles, 64, scan64.center)
    proj, dark, flat = to_dev(scan64.proj), to_dev(scan64.dark), to_dev(scan64.flat)
    with pytest.raises(tp.TpError) as ei:
        tp.fourier_fbp_chunk(plan, proj, dark, flat, half_width=9)
    assert ei.value.status == tp.TP_EINVAL
    tiny = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(tp.TpError) as ei:
        tp.fourier_fbp_chunk(plan, proj, dark, flat, workspace=tiny)
    assert ei.value.status == tp.TP_EINVAL and "workspace" in str(ei.value)
    big = tp.Plan(scan64.angles, 64, scan64.center, 9000)  # grid side 32768
    assert tp._fourier_prepare(big.handle, tp.TP_RAMP, 0) == tp.TP_EUNSUPPORTED
    p = ctypes.c_void_p(proj.data_ptr())
    ws = torch.empty(plan.fourier_workspace_bytes(7), dtype=torch.uint8, device="cuda")
    st = tp._fourier_chunk(plan.handle, p, 0, ctypes.c_void_p(dark.data_ptr()), 1, ctypes.c_void_p(flat.data_ptr()),
                           1, 0, 0, tp.TP_RAMP, 0, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                           ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p())
    assert st == tp.TP_EINVAL  # zero rows, rejected before any launch
