"""GPU tests of the three-stream chunk pipeline and the autotuner."""
import numpy as np
import pytest

import oracle
from paper_2209_08450_amd import synth
from tests._util import assert_parity, note, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_08450_amd import pipeline, tp, tune
    s = synth.ellipsoid_scan_np(seed=7, n_angles=90, n_rows=100, n_det=128, center=63.5, n_dark=3, n_flat=4)
    return tp, pipeline, tune, s


def _monolithic(tp, plan, s, storage):
    out = tp.fbp_chunk(plan, to_dev(s.proj), to_dev(s.dark), to_dev(s.flat), storage)
    return to_host(out)


def _source(s):
    proj = s.proj.view(np.int16)
    dark = s.dark.view(np.int16)
    flat = s.flat.view(np.int16)

    def fill(z0, z1, p, d, f):
        np.copyto(p.numpy(), proj[:, z0:z1, :])
        np.copyto(d.numpy(), dark[:, z0:z1, :])
        np.copyto(f.numpy(), flat[:, z0:z1, :])
    return fill


def _sink(result):
    def put(z0, z1, vol):
        result[z0:z1] = vol.numpy()
    return put


@pytest.mark.parametrize("graphs,poison,storage,buffers", [(True, False, "f16", 2), (False, True, "f16", 2),
                                                           (True, True, "f32", 2), (True, False, "bf16", 2),
                                                           (True, True, "f16", 3), (False, True, "f32", 4)])
def test_pipeline_bitwise_equals_monolithic(env, graphs, poison, storage, buffers):
    # poisoned buffers (NaN before each use) expose a missing dependency; with
    # more buffers the hazards move to chunk k - buffers
    tp, pipeline, _, s = env
    plan = tp.Plan(s.angles, 128, s.center)
    want = _monolithic(tp, plan, s, storage)
    chunks = pipeline.uneven_chunks(100, (7, 13, 32))
    pl = pipeline.ChunkPipeline(plan, max_rows=32, n_dark=3, n_flat=4, storage=storage, use_graphs=graphs,
                                poison=poison, buffers=buffers)
    got = np.full((100, 128, 128), np.nan, np.float32)
    note(f"pipeline graphs={graphs} poison={poison} {storage} buffers={buffers}")
    st = pl.run(chunks, _source(s), _sink(got))
    assert st.chunks == len(chunks) and st.rows == 100
    if graphs:
        assert st.graph_replays == len(chunks)
        assert st.graphs_captured == len({(k % buffers, z1 - z0) for k, (z0, z1) in enumerate(chunks)})
    assert np.array_equal(got, want)


def test_pipeline_fp16_slices(env, tmp_path):
    # the 16-bit mode end to end: FP16 rows and FP16 slices out of the
    # pipeline (graphs, uneven chunks) equal the monolithic call's FP16 slices
    # bitwise, those are its FP32 slices rounded once, and the file sink
    # writes 2-byte voxels
    import torch
    tp, pipeline, _, s = env
    plan = tp.Plan(s.angles, 128, s.center)
    P, D, F = to_dev(s.proj), to_dev(s.dark), to_dev(s.flat)
    want32 = tp.fbp_chunk(plan, P, D, F, "f16")
    want16 = tp.fbp_chunk(plan, P, D, F, "f16", out_dtype="f16")
    assert want16.dtype == torch.float16
    assert torch.equal(want16, want32.half())
    chunks = pipeline.uneven_chunks(100, (7, 13, 32))
    pl = pipeline.ChunkPipeline(plan, max_rows=32, n_dark=3, n_flat=4, storage="f16", use_graphs=True,
                                out_dtype="f16")
    got = np.full((100, 128, 128), np.nan, np.float16)
    note("pipeline FP16 slices")
    pl.run(chunks, _source(s), _sink(got))
    assert np.array_equal(got, to_host(want16).astype(np.float16))
    path = tmp_path / "vol16.raw"
    sink = pipeline.FileSink(path, 100, 128, threads=4, elem_bytes=2)
    pl.run(chunks, _source(s), sink)
    sink.flush()
    on_disk = np.fromfile(path, dtype=np.float16).reshape(100, 128, 128)
    assert np.array_equal(on_disk, got)
    want = oracle.fbp(s.proj, s.dark, s.flat, s.angles, s.center)
    assert_parity(got.astype(np.float64), want, "f16", label="pipeline FP16 slices")
    with pytest.raises(ValueError):
        pipeline.ChunkPipeline(plan, max_rows=32, n_dark=3, n_flat=4, storage="f32", out_dtype="f16")
    with pytest.raises(tp.TpError):
        tp.fbp_chunk(plan, P, D, F, "f32", out_dtype="f16")  # FP16 slices need FP16 rows
    with pytest.raises(tp.TpError):
        tp.fbp_chunk(plan, P, D, F, "f16", out_dtype="bf16")  # no BF16 slices


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_pipeline_matches_oracle(env, storage):
    # the pipelined volume, uneven chunks 7/13/32 through three streams with
    # graphs, against the FP64 oracle's FBP of the same scan: every slice,
    # chunk-boundary slices included, element by element
    tp, pipeline, _, s = env
    plan = tp.Plan(s.angles, 128, s.center)
    chunks = pipeline.uneven_chunks(100, (7, 13, 32))
    pl = pipeline.ChunkPipeline(plan, max_rows=32, n_dark=3, n_flat=4, storage=storage, use_graphs=True)
    got = np.full((100, 128, 128), np.nan, np.float32)
    note(f"pipeline vs oracle {storage}")
    pl.run(chunks, _source(s), _sink(got))
    want = oracle.fbp(s.proj, s.dark, s.flat, s.angles, s.center)
    assert_parity(got, want, storage, label="pipeline 90 x 100 x 128, chunks 7/13/32")
    edges = sorted({z for z0, z1 in chunks for z in (z0, z1 - 1)})
    assert_parity(got[edges], want[edges], storage, label="pipeline chunk-boundary slices")


def test_pipeline_fourier_matches_oracle_at_chunk_boundaries(env):
    # the Fourier-domain path through the pipeline: the first and last slice of
    # every chunk at sampled voxels against the oracle's direct sum
    tp, pipeline, _, s = env
    plan = tp.Plan(s.angles, 128, s.center)
    chunks = pipeline.uneven_chunks(100, (32, 16))
    pl = pipeline.ChunkPipeline(plan, max_rows=32, n_dark=3, n_flat=4, method="fourier")
    got = np.full((100, 128, 128), np.nan, np.float32)
    note("pipeline fourier vs oracle")
    pl.run(chunks, _source(s), _sink(got))
    rng = np.random.default_rng(21)
    ix, iy = rng.integers(0, 128, 96), rng.integers(0, 128, 96)
    for z in sorted({z for z0, z1 in chunks for z in (z0, z1 - 1)}):
        want = oracle.fourier_fbp_points(s.proj[:, z], s.dark[:, z], s.flat[:, z], s.angles, s.center, 128, ix, iy)
        assert_parity(got[z][iy, ix], want, "f32", label=f"pipeline fourier slice {z}")


def test_pipeline_parzen_bitwise_equals_monolithic(env):
    tp, pipeline, _, s = env
    plan = tp.Plan(s.angles, 128, s.center)
    want = to_host(tp.fbp_chunk(plan, to_dev(s.proj), to_dev(s.dark), to_dev(s.flat), "f16", kind="parzen"))
    pl = pipeline.ChunkPipeline(plan, max_rows=32, n_dark=3, n_flat=4, storage="f16", kind="parzen")
    got = np.full((100, 128, 128), np.nan, np.float32)
    note("pipeline parzen f16 graphs")
    pl.run(pipeline.uneven_chunks(100, (32, 9)), _source(s), _sink(got))
    assert np.array_equal(got, want)


def test_pipeline_fourier_bitwise_equals_monolithic(env):
    # even chunk sizes keep the slice pairs of one monolithic call, so every
    # pair goes through the same arithmetic
    tp, pipeline, _, s = env
    plan = tp.Plan(s.angles, 128, s.center)
    want = to_host(tp.fourier_fbp_chunk(plan, to_dev(s.proj), to_dev(s.dark), to_dev(s.flat), kind="parzen"))
    pl = pipeline.ChunkPipeline(plan, max_rows=32, n_dark=3, n_flat=4, kind="parzen", method="fourier")
    got = np.full((100, 128, 128), np.nan, np.float32)
    note("pipeline fourier parzen graphs")
    pl.run(pipeline.uneven_chunks(100, (32, 16)), _source(s), _sink(got))
    assert np.array_equal(got, want)
    assert pl.stats.graphs_captured > 0


@pytest.mark.parametrize("graphs,buffers", [(True, 3), (False, 2)])
def test_pipeline_lprec_bitwise_equals_monolithic(env, graphs, buffers):
    # the log-polar backprojector behind the same streams: even chunk sizes
    # keep the slice pairs of one monolithic call (one pass per chunk there,
    # one pass over all rows here); poisoned buffers expose a missing dependency
    tp, pipeline, _, s = env
    plan = tp.Plan(s.angles, 128, s.center)
    want = to_host(tp.lprec_fbp_chunk(plan, to_dev(s.proj), to_dev(s.dark), to_dev(s.flat), kind="shepp"))
    pl = pipeline.ChunkPipeline(plan, max_rows=32, n_dark=3, n_flat=4, kind="shepp", method="lprec",
                                use_graphs=graphs, poison=True, buffers=buffers)
    got = np.full((100, 128, 128), np.nan, np.float32)
    note(f"pipeline lprec graphs={graphs} buffers={buffers}")
    st = pl.run(pipeline.uneven_chunks(100, (32, 16)), _source(s), _sink(got))
    assert st.rows == 100
    assert np.array_equal(got, want)


def test_pipeline_lprec_needs_equal_angles(env):
    tp, pipeline, _, s = env
    ang = s.angles.copy()
    ang[3] += 1e-3  # no longer theta_0 + a pi / n_angles
    plan = tp.Plan(ang, 128, s.center)
    with pytest.raises((ValueError, RuntimeError)):
        pipeline.ChunkPipeline(plan, max_rows=32, n_dark=3, n_flat=4, method="lprec")

def test_fourier_fp16_slices_and_pipeline(env):
    # 16-bit volumes from the Fourier-domain path: each voxel's FP32 value
    # rounded once (bitwise the FP32 slices rounded), and the same slices out
    # of the pipeline with poisoned buffers; the log-polar path refuses them
    import torch
    tp, pipeline, _, s = env
    plan = tp.Plan(s.angles, 128, s.center)
    P, D, F = to_dev(s.proj), to_dev(s.dark), to_dev(s.flat)
    want32 = tp.fourier_fbp_chunk(plan, P, D, F, kind="parzen")
    want16 = tp.fourier_fbp_chunk(plan, P, D, F, kind="parzen", out_dtype="f16")
    assert want16.dtype == torch.float16
    assert torch.equal(want16, want32.half())
    pl = pipeline.ChunkPipeline(plan, max_rows=32, n_dark=3, n_flat=4, kind="parzen", method="fourier",
                                out_dtype="f16", poison=True)
    got = np.full((100, 128, 128), np.nan, np.float16)
    note("pipeline fourier f16 slices")
    pl.run(pipeline.uneven_chunks(100, (32, 16)), _source(s), _sink(got))
    assert np.array_equal(got, want16.cpu().numpy())
    with pytest.raises(ValueError):
        tp.fourier_fbp_chunk(plan, P, D, F, out_dtype="bf16")
    with pytest.raises(ValueError):
        pipeline.ChunkPipeline(plan, max_rows=32, n_dark=3, n_flat=4, method="lprec", out_dtype="f16")

def test_pipeline_files_to_file_bitwise_equals_monolithic(env, tmp_path):
    # storage on both ends: the source reads row chunks from raw projection-major
    # files, the sink writes slices into one volume file (native reader and
    # writer threads)
    tp, pipeline, _, s = env
    plan = tp.Plan(s.angles, 128, s.center)
    want = _monolithic(tp, plan, s, "f16")
    na, rows, n = s.proj.shape
    for name, arr in (("proj", s.proj), ("dark", s.dark), ("flat", s.flat)):
        np.ascontiguousarray(arr).tofile(tmp_path / f"{name}.raw")
    src = pipeline.FileSource(tmp_path / "proj.raw", tmp_path / "dark.raw", tmp_path / "flat.raw", na, rows, n,
                              s.dark.shape[0], s.flat.shape[0], threads=4)
    sink = pipeline.FileSink(tmp_path / "vol.raw", rows, 128, threads=4)
    pl = pipeline.ChunkPipeline(plan, max_rows=32, n_dark=s.dark.shape[0], n_flat=s.flat.shape[0], storage="f16")
    note("pipeline files to file f16")
    pl.run(pipeline.uneven_chunks(rows, (32, 9)), src, sink)
    got = np.fromfile(tmp_path / "vol.raw", np.float32).reshape(rows, 128, 128)
    assert np.array_equal(got, want)


def test_graph_replays_repeat_with_eager_work_between(env):
    import torch
    tp, pipeline, _, s = env
    plan = tp.Plan(s.angles, 128, s.center)
    want = _monolithic(tp, plan, s, "f16")
    chunks = pipeline.uneven_chunks(100, (32, 64))
    pl = pipeline.ChunkPipeline(plan, max_rows=64, n_dark=3, n_flat=4, storage="f16", use_graphs=True)
    for rep in range(3):
        note(f"pipeline replay round {rep}")
        got = np.zeros((100, 128, 128), np.float32)
        pl.run(chunks, _source(s), _sink(got))
        assert np.array_equal(got, want), rep
        # eager work and synchronisation of the program between replays
        _monolithic(tp, plan, s, "f32")
        torch.cuda.synchronize()
    assert pl.stats.graphs_captured == len({(k % pl.nbuf, z1 - z0) for k, (z0, z1) in enumerate(chunks)})


def test_source_failure_names_chunk_and_pipeline_recovers(env):
    tp, pipeline, _, s = env
    plan = tp.Plan(s.angles, 128, s.center)
    chunks = pipeline.uneven_chunks(100, (32,))
    pl = pipeline.ChunkPipeline(plan, max_rows=32, n_dark=3, n_flat=4, storage="f16")
    good = _source(s)

    def bad(z0, z1, p, d, f):
        if z0 >= 64:
            raise OSError("read failed")
        good(z0, z1, p, d, f)

    note("pipeline source failure")
    with pytest.raises(RuntimeError, match=r"chunk 2 \(rows \[64, 96\)\)"):
        pl.run(chunks, bad, lambda *a: None)
    got = np.zeros((100, 128, 128), np.float32)
    pl.run(chunks, good, _sink(got))
    assert np.array_equal(got, _monolithic(tp, plan, s, "f16"))


def test_sink_failure_is_reported(env):
    tp, pipeline, _, s = env
    plan = tp.Plan(s.angles, 128, s.center)
    pl = pipeline.ChunkPipeline(plan, max_rows=50, n_dark=3, n_flat=4, storage="f16")

    def sink(z0, z1, vol):
        if z0 == 50:
            raise ValueError("disk full")

    note("pipeline sink failure")
    with pytest.raises(RuntimeError, match=r"rows \[50, 100\)"):
        pl.run([(0, 50), (50, 100)], _source(s), sink)


def test_autotuner_on_device(env, tmp_path):
    import torch
    tp, _, tune, s = env
    plan = tp.Plan(s.angles, 128, s.center)
    q = to_dev(np.random.default_rng(0).standard_normal((9, 90, 128)).astype(np.float32)).half()
    ref = tp.backproject(plan, q)
    note("autotuner f16")
    k, a = tune.tune_backproject(plan, "f16", rows=8, reps=2, path=str(tmp_path / "t.json"))
    assert (k, a) in tune.candidates("f16") and plan.get_tuning("f16") == (k, a)
    assert torch.equal(tp.backproject(plan, q), ref)
