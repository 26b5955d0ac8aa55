"""GPU parity of the fused tp_fbp_chunk (normalise -> filter -> backproject)
against the FP64 oracle, at the 16-slice ellipse scan and at paper scale."""
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
def scan16():
    return synth.phantom_2d_scan(seed=1, n_rows=16, n_angles=180, n_det=256)


@pytest.fixture(scope="module")
def ref16(scan16):
    s = scan16
    return {st: oracle.fbp(s.proj, s.dark, s.flat, s.angles, s.center, storage=st)
            for st in (None, "f16", "bf16")}


def _run(tp, s, storage, plan=None):
    plan = plan or tp.Plan(s.angles, s.proj.shape[2], s.center, s.n_vox)
    out = tp.fbp_chunk(plan, to_dev(s.proj), to_dev(s.dark), to_dev(s.flat), storage)
    return to_host(out).astype(np.float64)


def test_fbp_f32_16_slices(tp, scan16, ref16):
    note("fbp f32 180x16x256")
    got = _run(tp, scan16, "f32")
    want = ref16[None]
    assert_parity(got, want, "f32", label="fbp 16 slices")
    for z in range(16):
        assert rel_l2(got[z], want[z]) < 1e-5


def test_fbp_f16_storage(tp, scan16, ref16):
    note("fbp f16 180x16x256")
    got = _run(tp, scan16, "f16")
    e, _ = assert_parity(got, ref16[None], "f16", label="fbp 16 slices")
    # against the oracle with the same storage rounding: FP32-level agreement
    # except where an FP32/FP64 difference flips an FP16 rounding
    assert rel_l2(got, ref16["f16"]) < 0.25 * e + 1e-5


def test_fbp_bf16_storage(tp, scan16, ref16):
    note("fbp bf16 180x16x256")
    got = _run(tp, scan16, "bf16")
    e, _ = assert_parity(got, ref16[None], "bf16", label="fbp 16 slices")
    assert rel_l2(got, ref16["bf16"]) < 0.25 * e + 1e-5


def test_fbp_ragged_geometry(tp):
    # odd angle count (an unpaired last row), odd detector width, N != n,
    # several frames, centre off the middle
    s = synth.ellipsoid_scan_np(seed=4, n_angles=45, n_rows=5, n_det=97, center=50.3, n_dark=3, n_flat=4)
    plan = tp.Plan(s.angles, 97, s.center, 80)
    note("fbp ragged 45x5x97 -> 80")
    out = tp.fbp_chunk(plan, to_dev(s.proj), to_dev(s.dark), to_dev(s.flat), "f32")
    got = to_host(out).astype(np.float64)
    want = oracle.fbp(s.proj, s.dark, s.flat, s.angles, s.center, N=80)
    assert_parity(got, want, "f32", label="fbp ragged")


def test_fbp_equals_separate_calls(tp, scan16):
    import torch
    s = scan16
    plan = tp.Plan(s.angles, 256, s.center)
    P, D, F = to_dev(s.proj), to_dev(s.dark), to_dev(s.flat)
    note("fbp fused vs separate")
    fused = tp.fbp_chunk(plan, P, D, F, "f32")
    sino = tp.normalize(P, D, F, "f32")
    filt = tp.filter(sino)
    sep = tp.backproject(plan, filt)
    torch.cuda.synchronize()
    # the fused kernel normalises in registers; same FP32 expressions -> equal
    assert rel_l2(to_host(fused), to_host(sep)) < 1e-6


def test_fbp_paper_scale_sampled(tp):
    """2048 angles x 2048 columns (the 2048^3 workload's per-slice shape), two
    rows of the 200-ellipsoid 12-bit scan, default tuning; the oracle evaluates
    1024 sampled voxels per slice."""
    rows = [700, 1300]
    s = synth.ellipsoid_scan_np(seed=2, n_angles=2048, n_rows=2048, n_det=2048, center=1024.0, rows=rows)
    plan = tp.Plan(s.angles, 2048, s.center)
    note("fbp 2048x2x2048 f32/f16")
    got32 = to_host(tp.fbp_chunk(plan, to_dev(s.proj), to_dev(s.dark), to_dev(s.flat), "f32"))
    got16 = to_host(tp.fbp_chunk(plan, to_dev(s.proj), to_dev(s.dark), to_dev(s.flat), "f16"))
    rng = np.random.default_rng(0)
    e32, e16 = [], []
    for i in range(len(rows)):
        ix = rng.integers(0, 2048, 1024)
        iy = rng.integers(0, 2048, 1024)
        want = oracle.fbp_points(s.proj[:, i], s.dark[:, i], s.flat[:, i], s.angles, s.center, 2048, ix, iy)
        e32.append(rel_l2(got32[i][iy, ix], want))
        e16.append(rel_l2(got16[i][iy, ix], want))
        assert_parity(got32[i][iy, ix], want, "f32", label=f"paper-scale row {rows[i]}")
        assert_parity(got16[i][iy, ix], want, "f16", label=f"paper-scale row {rows[i]}")
    note(f"paper-scale rel-L2 f32 {e32} f16 {e16}")
    assert max(e32) < 1e-5
    assert max(e16) < 3e-3


def test_fbp_bench_launch_shape_sampled(tp):
    """The launch the 2048^3 benchmark times: one 256-row chunk of 2048 angles
    x 2048 columns (default tuning, all three storage types) of a 12-bit
    ellipsoid scan generated on the GPU; three rows spread over the chunk (its
    first and last slice blocks included) checked at 512 sampled voxels each,
    and the chunk's first and last slices checked whole (2048^2 voxels each)
    against the oracle's full-slice FBP."""
    import torch
    s = synth.ellipsoid_scan_torch(seed=5, n_angles=2048, n_rows=256, n_det=2048, device="cuda", center=1024.0)
    rows = [0, 129, 255]
    host = {name: getattr(s, name)[:, rows].cpu().numpy().view(np.uint16) for name in ("proj", "dark", "flat")}
    plan = tp.Plan(s.angles, 2048, s.center)
    rng = np.random.default_rng(3)
    pts = [(rng.integers(0, 2048, 512), rng.integers(0, 2048, 512)) for _ in rows]
    want = [oracle.fbp_points(host["proj"][:, i], host["dark"][:, i], host["flat"][:, i], s.angles, s.center, 2048,
                              ix, iy) for i, (ix, iy) in enumerate(pts)]
    whole = [0, 2]  # positions in `rows` of the chunk's first and last slices
    want_full = oracle.fbp(host["proj"][:, whole], host["dark"][:, whole], host["flat"][:, whole], s.angles,
                           s.center)
    for storage, tol in (("f32", 1e-5), ("f16", 3e-3), ("bf16", 3e-3)):
        note(f"fbp 2048 x 256 x 2048 {storage}")
        vol = tp.fbp_chunk(plan, s.proj, s.dark, s.flat, storage)
        got = vol[rows].cpu().numpy().astype(np.float64)
        del vol
        torch.cuda.empty_cache()
        errs = [rel_l2(got[i][iy, ix], want[i]) for i, (ix, iy) in enumerate(pts)]
        note(f"{storage} rel-L2 {errs}")
        assert max(errs) < tol
        for i, (ix, iy) in enumerate(pts):
            assert_parity(got[i][iy, ix], want[i], storage, rel=tol, label=f"bench chunk row {rows[i]} sampled")
        assert_parity(got[whole], want_full, storage, rel=tol, label="bench chunk first and last slices whole")
    plan.close()


@pytest.mark.parametrize("kind", ["shepp", "parzen"])
def test_fbp_windowed_filters(tp, scan16, kind):
    # the paper's filter choices; Parzen is its default
    s = scan16
    note(f"fbp {kind} 180x16x256")
    want = oracle.fbp(s.proj, s.dark, s.flat, s.angles, s.center, kind=kind)
    want16 = oracle.fbp(s.proj, s.dark, s.flat, s.angles, s.center, storage="f16", kind=kind)
    plan = tp.Plan(s.angles, 256, s.center)
    run = lambda st: to_host(tp.fbp_chunk(plan, to_dev(s.proj), to_dev(s.dark), to_dev(s.flat), st,  # noqa: E731
                                          kind=kind)).astype(np.float64)
    assert_parity(run("f32"), want, "f32", label=f"fbp {kind}")
    e, _ = assert_parity(run("f16"), want, "f16", label=f"fbp {kind}")
    assert rel_l2(run("f16"), want16) < 0.25 * e + 1e-5
    assert_parity(run("bf16"), want, "bf16", label=f"fbp {kind}")
    # the window changes the reconstruction
    assert rel_l2(want, oracle.fbp(s.proj, s.dark, s.flat, s.angles, s.center)) > 1e-2


def test_fbp_windowed_graph_capture_needs_prepared_tables(tp):
    import torch
    s = synth.ellipsoid_scan_np(seed=9, n_angles=24, n_rows=3, n_det=40, center=19.5, n_dark=1, n_flat=1)
    plan = tp.Plan(s.angles, 40, s.center)
    P, D, F = to_dev(s.proj), to_dev(s.dark), to_dev(s.flat)
    out = torch.empty((3, 40, 40), device="cuda")
    ws = torch.empty(plan.fbp_workspace_bytes(3, "f32"), dtype=torch.uint8, device="cuda")
    st = torch.cuda.Stream()
    note("fbp shepp capture without prepared tables")
    g = torch.cuda.CUDAGraph()
    with pytest.raises(tp.TpError, match="tp_filter_prepare"):
        with torch.cuda.graph(g, stream=st, capture_error_mode="thread_local"):
            tp.fbp_chunk(plan, P, D, F, "f32", out=out, workspace=ws, kind="shepp")
    torch.cuda.synchronize()
    note("fbp shepp capture with prepared tables, replays")
    tp.filter_prepare(tp.pad_len(40), "shepp")
    want = oracle.fbp(s.proj, s.dark, s.flat, s.angles, s.center, kind="shepp")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st, capture_error_mode="thread_local"):
        tp.fbp_chunk(plan, P, D, F, "f32", out=out, workspace=ws, kind="shepp")
    for rep in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert rel_l2(to_host(out).astype(np.float64), want) < 1e-5, rep


def test_zero_rows_rejected_before_launch(tp):
    import ctypes

    import torch
    s = synth.ellipsoid_scan_np(seed=3, n_angles=8, n_rows=2, n_det=32, center=15.5, n_dark=1, n_flat=1)
    plan = tp.Plan(s.angles, 32, s.center)
    buf = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    nul = ctypes.c_void_p()
    note("zero-row calls")
    assert tp._backproject(plan.handle, p, tp.TP_F32, 0, 1.0, p, 0, nul) == tp.TP_EINVAL
    assert "n_rows" in tp.last_error()
    assert tp._radon(plan.handle, p, 0, p, p, 1 << 20, nul) == tp.TP_EINVAL
    assert tp._fbp_chunk(plan.handle, p, 0, p, 1, p, 1, 0, 0, tp.TP_RAMP, tp.TP_F32, p, 1 << 20, p,
                         nul) == tp.TP_EINVAL
    assert tp._normalize(p, 0, p, 1, p, 1, 0, 8, 0, 32, tp.TP_F32, p, p, 1 << 20, nul) == tp.TP_EINVAL
    torch.cuda.synchronize()


def test_fbp_widest_detector(tp):
    # n_det = 8192, the widest a plan takes: pad length 16384 (the LDS FFT path
    # of the fused kernel), 8192^2 slices; sampled voxels against the oracle
    s = synth.ellipsoid_scan_np(seed=6, n_angles=24, n_rows=2, n_det=8192, center=4095.5, n_dark=2, n_flat=2)
    plan = tp.Plan(s.angles, 8192, s.center)
    note("fbp 24 x 2 x 8192 f32")
    out = tp.fbp_chunk(plan, to_dev(s.proj), to_dev(s.dark), to_dev(s.flat), "f32")
    rng = np.random.default_rng(7)
    ix, iy = rng.integers(0, 8192, 256), rng.integers(0, 8192, 256)
    for z in range(2):
        want = oracle.fbp_points(s.proj[:, z], s.dark[:, z], s.flat[:, z], s.angles, s.center, 8192, ix, iy)
        got = to_host(out[z])[iy, ix].astype(np.float64)
        assert_parity(got, want, "f32", label=f"widest detector row {z}")


def test_wrong_output_tensors_refused(tp, scan16):
    # a caller's output tensor that does not match what the kernels write is
    # refused before any launch (the C ABI sees only its pointer)
    import torch
    s = scan16
    plan = tp.Plan(s.angles, 256, s.center)
    proj, dark, flat = to_dev(s.proj), to_dev(s.dark), to_dev(s.flat)
    bad = [torch.empty((16, 256, 255), device="cuda"),                      # too small
           torch.empty((16, 256, 256), dtype=torch.float16, device="cuda"),  # wrong type
           torch.empty((256, 256, 16), device="cuda").permute(2, 0, 1)]     # not contiguous
    for out in bad:
        with pytest.raises(ValueError):
            tp.fbp_chunk(plan, proj, dark, flat, "f32", out=out)
        with pytest.raises(ValueError):
            tp.fourier_fbp_chunk(plan, proj, dark, flat, out=out)
    with pytest.raises(ValueError):
        tp.normalize(proj, dark, flat, out=torch.empty((16, 180, 255), device="cuda"))
    with pytest.raises(ValueError):
        tp.radon(plan, torch.zeros((2, 256, 256), device="cuda"), out=torch.empty((2, 180, 200), device="cuda"))
    with pytest.raises(ValueError):
        tp.lamino_backproject(plan, torch.zeros((180, 8, 256), device="cuda"), 1.0, 4.0, 4,
                              out=torch.empty((3, 256, 256), device="cuda"))
    plan.close()
