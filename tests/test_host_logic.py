"""Host-side logic that needs no GPU: chunk partitions and the tuner's
selection and cache (with an injected timing function)."""
import json
import os

import pytest

from paper_2209_08450_amd import tune


def test_uneven_chunks_cover_rows_once():
    pipeline = pytest.importorskip("paper_2209_08450_amd.pipeline")
    for n_rows, pattern, start in [(2048, (32, 64, 128), 0), (100, (7, 13, 32), 0), (5, (8,), 0),
                                   (97, (32, 64, 128), 10), (1, (3,), 0)]:
        ch = pipeline.uneven_chunks(n_rows, pattern, start)
        rows = [z for z0, z1 in ch for z in range(z0, z1)]
        assert rows == list(range(start, n_rows))
        assert all(0 < z1 - z0 <= max(pattern) for z0, z1 in ch)
        sizes = [z1 - z0 for z0, z1 in ch]
        assert sizes[:-1] == [pattern[i % len(pattern)] for i in range(len(sizes) - 1)]
    with pytest.raises(ValueError):
        pipeline.uneven_chunks(10, (0,))


def test_pipeline_needs_two_buffers():
    # fewer than two buffers per direction cannot overlap anything: refused
    # before any plan or device memory is touched
    pipeline = pytest.importorskip("paper_2209_08450_amd.pipeline")
    for bad in (0, 1):
        with pytest.raises(ValueError, match="buffers"):
            pipeline.ChunkPipeline(None, max_rows=8, n_dark=1, n_flat=1, buffers=bad)


def test_tuner_legal_candidates():
    c16 = tune.candidates("f16")
    c32 = tune.candidates("f32")
    assert (8, 64) in c16 and (8, 64) in c32  # f32: 32 B x 48 bins x 64 + 1 KiB = 97 KiB fits 160 KiB
    # groups of 64 bytes or more get one 16-byte bank group of padding
    assert tune.bin_pitch(16) == 16 and tune.bin_pitch(32) == 32 and tune.bin_pitch(64) == 80
    assert all(tune.legal("f32", k, a) for k, a in c32)
    # f16 stages pairs (Q[j], Q[j+1]): 4 bytes per slice and bin, as f32
    assert c16 == c32 and (16, 64) not in c16
    assert (16, 32) in c32  # 80 B x 48 x 32 + 512 = 120.5 KiB


class FakePlan:
    n_angles, n_det, n_vox = 90, 128, 128

    def __init__(self):
        self.tuning = {}

    def set_tuning(self, storage, k, a):
        self.tuning[storage] = (k, a)


def test_tuner_picks_fastest_and_caches(tmp_path):
    path = str(tmp_path / "tune.json")
    calls = []

    def measure(k, a):
        calls.append((k, a))
        return abs(k - 4) + abs(a - 16) / 8 + 1.0  # minimum at (4, 16)

    plan = FakePlan()
    choice = tune.tune_backproject(plan, "f32", rows=8, path=path, measure=measure, device_name="fake")
    assert choice == (4, 16) and plan.tuning["f32"] == (4, 16)
    assert len(calls) == len(tune.candidates("f32"))
    d = json.load(open(path))
    key = tune.cache_key("fake", "f32", 90, 128, 128, 8)
    assert d[key]["choice"] == [4, 16]
    # second call is served from the cache: no measurements
    calls.clear()
    plan2 = FakePlan()
    assert tune.tune_backproject(plan2, "f32", rows=8, path=path, measure=measure, device_name="fake") == (4, 16)
    assert calls == [] and plan2.tuning["f32"] == (4, 16)
    # a different shape is tuned anew and both entries are kept
    plan3 = FakePlan()
    plan3.n_angles = 180
    tune.tune_backproject(plan3, "f32", rows=8, path=path, measure=measure, device_name="fake")
    assert len(json.load(open(path))) == 2


def test_tuner_cache_tolerates_corruption(tmp_path):
    path = str(tmp_path / "tune.json")
    with open(path, "w") as f:
        f.write("{not json")
    assert tune.load_cache(path) == {}
    plan = FakePlan()
    assert tune.tune_backproject(plan, "f16", path=path, measure=lambda k, a: k + a, device_name="x") == (1, 8)
    assert os.path.exists(path)
