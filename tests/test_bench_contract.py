"""Host-side parts of bench.py's contract: the one-GPU guard, the committed
traffic records (used only while they match the kernel sources), and the
algorithmic work counts the roofline fields are computed from."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_traffic_records_are_ignored_for_other_sources(bench, tmp_path, monkeypatch):
    # a record taken on other kernel source (another hash) must not be reported
    for name in ("traffic_backproject.json", "traffic_lamino.json"):
        d = json.load(open(os.path.join(ROOT, "profiles", name)))
        d["kernel_sha"] = "0000000000000000"
        os.makedirs(tmp_path / "profiles", exist_ok=True)
        json.dump(d, open(tmp_path / "profiles" / name, "w"))
    os.makedirs(tmp_path / "paper_2209_08450_amd" / "csrc", exist_ok=True)
    for src in ("k_backproject.hip", "k_lamino.hip"):
        with open(tmp_path / "paper_2209_08450_amd" / "csrc" / src, "wb") as f:
            f.write(open(os.path.join(ROOT, "paper_2209_08450_amd", "csrc", src), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.load_traffic("f16", 256, 2048, 2048) is None
    assert bench.load_lamino_traffic() is None


def test_traffic_records_describe_their_launch(bench):
    # where a record matches its kernel, it is for the launch shape the bench times
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic_lamino.json")))
    e = d["f16"]
    c = bench.LAMINO
    assert (e["n"], e["angles"], e["slices"], e["tilt"]) == (c["n"], c["angles"], c["slices"], c["tilt"])
    assert e["algorithmic_bytes_per_launch"] == c["angles"] * c["rows"] * c["n"] * 2 + c["slices"] * c["n"] ** 2 * 4
    # the written bytes are the slab, once
    assert e["write_kib"] * 1024 == c["slices"] * c["n"] ** 2 * 4


def test_fourier_work_count(bench):
    # (L + 1) samples per angle and slice pair, each meeting (2h)^2 grid points at 6 flop
    assert bench.fourier_flop_per_pair(2048, 4096, 6) == 2048 * 4097 * 144 * 6


def test_filter_roofline_bytes(bench):
    # 2048^3 scan, FP16 storage: 2 B raw in + 2 B filtered out per sample
    e = bench.filter_roofline("f16", 50.0, 2048, 2048, 2048)
    assert e["bytes_per_volume"] == 2048 ** 3 * 4
    assert abs(e["achieved"] - 2048 ** 3 * 4 / 0.05 / 1e9) < 0.1
    assert e["frac"] == round(e["achieved"] / 8000.0, 4)
    assert bench.filter_roofline("f32", 50.0, 2, 3, 4)["bytes_per_volume"] == 2 * 3 * 4 * 6
