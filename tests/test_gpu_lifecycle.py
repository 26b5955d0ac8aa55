"""GPU tests of the lifecycle calls: tp_prepare (tables and kernel attributes
built before graph capture), the tuning table applied at plan creation, and
tp_shutdown (run in a fresh process, where no other test's plans are alive)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2209_08450_amd import synth
from tests._util import assert_parity, note, to_dev, to_host

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_08450_amd import tp as mod
    return mod


def test_prepare_then_capture_without_an_eager_run(tp):
    # A tiling whose staged block needs more than 64 KiB of LDS (F16, 16
    # slices x 32 angles: 120.5 KiB) and a windowed filter: after tp_prepare the
    # very first call may be a graph capture.  Replays, with eager work and
    # synchronisation between them, equal an eager call bitwise and the oracle
    # within the FP16 bounds.
    import torch
    s = synth.ellipsoid_scan_np(seed=12, n_angles=64, n_rows=20, n_det=96, center=47.6, n_dark=2, n_flat=2)
    plan = tp.Plan(s.angles, 96, s.center)
    plan.set_tuning("f16", 16, 32)
    plan.prepare("parzen", "f16")
    P, D, F = to_dev(s.proj), to_dev(s.dark), to_dev(s.flat)
    out = torch.empty((20, 96, 96), device="cuda")
    ws = torch.empty(plan.fbp_workspace_bytes(20, "f16"), dtype=torch.uint8, device="cuda")
    st = torch.cuda.Stream()
    note("capture fbp parzen f16 (K=16, A=32) without an eager run")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st, capture_error_mode="thread_local"):
        tp.fbp_chunk(plan, P, D, F, "f16", out=out, workspace=ws, kind="parzen")
    eager = tp.fbp_chunk(plan, P, D, F, "f16", kind="parzen")
    torch.cuda.synchronize()
    want = oracle.fbp(s.proj, s.dark, s.flat, s.angles, s.center, kind="parzen")
    for rep in range(3):
        out.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        tp.fbp_chunk(plan, P, D, F, "f32", kind="parzen")  # eager work between replays
        torch.cuda.synchronize()
    assert_parity(to_host(out), want, "f16", label="prepared capture parzen")
    plan.close()


def test_tuning_table_sets_new_plans(tp, tmp_path):
    import torch

    from paper_2209_08450_amd import tune
    dev = torch.cuda.get_device_name()
    ang = synth.uniform_angles(40)
    path = str(tmp_path / "tune.json")
    tune.save_cache({tune.cache_key(dev, "f16", 40, 64, 64, 16): {"choice": [4, 32]},
                     tune.cache_key(dev, "f32", 40, 64, 64, 16): {"choice": [2, 64]}}, path)
    note("tuning table applied at plan creation")
    tp.tune_load(path)
    try:
        plan = tp.Plan(ang, 64, 31.5)
        assert plan.get_tuning("f16") == (4, 32)
        assert plan.get_tuning("f32") == (2, 64)
        assert plan.get_tuning("bf16") == (16, 8)  # no entry: the default
        other = tp.Plan(ang, 64, 31.5, 48)  # another shape: defaults
        assert other.get_tuning("f16") == (16, 8)
        q = to_dev(np.random.default_rng(2).standard_normal((5, 40, 64)).astype(np.float32)).half()
        got = tp.backproject(plan, q)
        plan.set_tuning("f16", 16, 16)
        assert torch.equal(tp.backproject(plan, q), got)  # tilings never change results
        plan.close()
        other.close()
    finally:
        tp.tune_load(None)


_SHUTDOWN_SCRIPT = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
from paper_2209_08450_amd import synth, tp
from tests._util import to_dev

s = synth.ellipsoid_scan_np(seed=13, n_angles=32, n_rows=4, n_det=64, center=31.2, n_dark=1, n_flat=1)
P, D, F = to_dev(s.proj), to_dev(s.dark), to_dev(s.flat)
plan = tp.Plan(s.angles, 64, s.center)
plan.prepare("shepp", "f32")
first = tp.fbp_chunk(plan, P, D, F, "f32", kind="shepp").cpu()
try:
    tp.shutdown()
    raise SystemExit("shutdown accepted while a plan is alive")
except tp.TpError as e:
    assert e.status == tp.TP_EINVAL and "plan" in str(e), e
plan.close()
torch.cuda.synchronize()
tp.shutdown()  # frees the cached filter tables
tp.shutdown()  # nothing left: still fine
plan = tp.Plan(s.angles, 64, s.center)  # rebuilds the ramp tables
again = tp.fbp_chunk(plan, P, D, F, "f32", kind="shepp").cpu()  # and the window's, on first use
assert torch.equal(first, again)
plan.close()
print("lifecycle ok", flush=True)
"""


def test_shutdown_in_a_fresh_process(tp):
    note("tp_shutdown in a child process")
    r = subprocess.run([sys.executable, "-c", _SHUTDOWN_SCRIPT, ROOT], capture_output=True, text=True, timeout=300,
                       cwd=ROOT)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    assert "lifecycle ok" in r.stdout
