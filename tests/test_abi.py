"""The C ABI: the library loads, exports every declared symbol, and rejects bad
arguments on the host (status + message, nothing enqueued).  No GPU needed:
every call here fails validation before touching the HIP runtime."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tp.h")


@pytest.fixture(scope="module")
def tp():
    from paper_2209_08450_amd import tp as mod
    return mod


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tp_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_hot_path_calls():
    names = declared_functions()
    for n in ["tp_normalize", "tp_filter", "tp_backproject", "tp_radon", "tp_fbp_chunk"]:
        assert n in names


def test_every_declared_symbol_is_exported(tp):
    lib = ctypes.CDLL(tp.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_version(tp):
    assert "gfx950" in tp.version()


def test_null_and_size_errors(tp):
    nul = ctypes.c_void_p()
    st = tp._filter(nul, tp.TP_F32, nul, tp.TP_F32, 4, 16, 0, tp.TP_RAMP, nul)
    assert st == tp.TP_EINVAL and "null" in tp.last_error()
    dummy = ctypes.c_void_p(0x100000)
    st = tp._filter(dummy, tp.TP_F32, ctypes.c_void_p(0x900000), tp.TP_F32, 0, 16, 0, tp.TP_RAMP, nul)
    assert st == tp.TP_EINVAL and "positive" in tp.last_error()
    st = tp._filter(dummy, tp.TP_F32, ctypes.c_void_p(0x900000), tp.TP_F32, 4, 16, 24, tp.TP_RAMP, nul)
    assert st == tp.TP_EINVAL and "power of two" in tp.last_error()
    st = tp._filter(dummy, tp.TP_F32, ctypes.c_void_p(0x900000), tp.TP_F32, 4, 16, 8, tp.TP_RAMP, nul)
    assert st == tp.TP_EINVAL  # pad shorter than the row
    st = tp._filter(dummy, tp.TP_F32, ctypes.c_void_p(0x900000), tp.TP_F32, 4, 16, 0, 7, nul)
    assert st == tp.TP_EUNSUPPORTED and "kind" in tp.last_error()
    st = tp._filter(dummy, 7, ctypes.c_void_p(0x900000), tp.TP_F32, 4, 16, 0, tp.TP_RAMP, nul)
    assert st == tp.TP_EINVAL and "dtype" in tp.last_error()


def test_filter_alias_rules(tp):
    nul = ctypes.c_void_p()
    a = ctypes.c_void_p(0x100000)
    # partial overlap is rejected, and so is in-place with different dtypes
    st = tp._filter(a, tp.TP_F32, ctypes.c_void_p(0x100000 + 32), tp.TP_F32, 4, 16, 0, tp.TP_RAMP, nul)
    assert st == tp.TP_EINVAL and "overlap" in tp.last_error()
    st = tp._filter(a, tp.TP_F32, a, tp.TP_F16, 4, 16, 0, tp.TP_RAMP, nul)
    assert st == tp.TP_EINVAL and "overlap" in tp.last_error()


def test_plan_validation(tp):
    ang = np.zeros(4)
    g = tp.Geometry(4, 16, 0, 8.0, None)
    h = ctypes.c_void_p()
    assert tp._plan_create(ctypes.byref(g), ctypes.byref(h)) == tp.TP_EINVAL
    assert "angles" in tp.last_error()
    g = tp.Geometry(0, 16, 0, 8.0, ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert tp._plan_create(ctypes.byref(g), ctypes.byref(h)) == tp.TP_EINVAL
    g = tp.Geometry(4, 16, 0, float("nan"), ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert tp._plan_create(ctypes.byref(g), ctypes.byref(h)) == tp.TP_EINVAL
    bad = np.array([0.0, np.inf, 1.0, 2.0])
    g = tp.Geometry(4, 16, 0, 8.0, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert tp._plan_create(ctypes.byref(g), ctypes.byref(h)) == tp.TP_EINVAL
    g = tp.Geometry(4, 9000, 0, 8.0, ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert tp._plan_create(ctypes.byref(g), ctypes.byref(h)) == tp.TP_EUNSUPPORTED


def test_plan_null_handles(tp):
    nul = ctypes.c_void_p()
    assert tp._plan_set_tuning(nul, tp.TP_F32, 4, 32) == tp.TP_EINVAL
    assert tp._backproject(nul, nul, 0, 1, 1.0, nul, 0, nul) == tp.TP_EINVAL
    assert tp._radon(nul, nul, 1, nul, nul, 0, nul) == tp.TP_EINVAL
    assert tp._radon_ws(nul, 4) == 0
    assert tp._fbp_chunk_out(nul, nul, 0, nul, 1, nul, 1, 0, 1, tp.TP_RAMP, tp.TP_F16, nul, 0, tp.TP_F16, nul, nul,
                             None) == tp.TP_EINVAL
    assert tp._plan_destroy(nul) == tp.TP_OK


def test_filter_prepare_validation(tp):
    assert tp._filter_prepare(3, tp.TP_RAMP) == tp.TP_EINVAL
    assert tp._filter_prepare(32768, tp.TP_RAMP) == tp.TP_EINVAL
    assert tp._filter_prepare(64, 7) == tp.TP_EUNSUPPORTED


def test_filter_response_validation(tp):
    buf = np.zeros(64)
    ptr = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert tp._filter_response(24, tp.TP_RAMP, ptr) == tp.TP_EINVAL
    assert tp._filter_response(32768, tp.TP_RAMP, ptr) == tp.TP_EINVAL
    assert tp._filter_response(64, 7, ptr) == tp.TP_EUNSUPPORTED
    assert tp._filter_response(64, tp.TP_RAMP, None) == tp.TP_EINVAL
    with pytest.raises(ValueError):
        tp.filter_code("hann")


@pytest.mark.parametrize("kind", ["ramp", "shepp", "parzen"])
def test_filter_response_matches_oracle(tp, kind):
    """The library's FP64 response (closed-form / exact piecewise taps, direct
    DFT sum on the host) against the oracle's (quadrature taps, numpy FFT)."""
    import oracle
    for L in (2, 8, 64, 1024, 8192):
        got = tp.filter_response(L, kind)
        want = oracle.filter_response(L, kind)
        # both FP64; summation order differs, so rounding grows ~ L (largest at Nyquist)
        assert np.max(np.abs(got - want)) < 1e-15 + 1e-16 * L, (kind, L)


def test_normalize_validation(tp):
    nul = ctypes.c_void_p()
    p = ctypes.c_void_p(0x100000)
    assert tp._normalize(nul, 0, p, 1, p, 1, 0, 4, 2, 8, 0, p, p, 1 << 20, nul) == tp.TP_EINVAL
    assert tp._normalize(p, 0, p, 0, p, 1, 0, 4, 2, 8, 0, p, p, 1 << 20, nul) == tp.TP_EINVAL
    assert tp._normalize(p, 0, p, 1, p, 300, 0, 4, 2, 8, 0, p, p, 1 << 20, nul) == tp.TP_EINVAL
    assert tp._normalize(p, 8, p, 1, p, 1, 0, 4, 2, 8, 0, p, p, 1 << 20, nul) == tp.TP_EINVAL  # stride < rows*n
    assert tp._normalize(p, 0, p, 1, p, 1, 0, 4, 2, 8, 0, p, p, 16, nul) == tp.TP_EINVAL  # workspace too small
    assert tp._normalize(p, 0, p, 1, p, 1, 0, 4, 2, 8, 0, p, ctypes.c_void_p(0x100010), 1 << 20,
                         nul) == tp.TP_EINVAL  # misaligned workspace
    assert tp._normalize(p, 0, p, 1, p, 1, 0, 4, 70000, 8, 0, p, p, 1 << 30, nul) == tp.TP_EINVAL
    assert tp._normalize_ws(2, 8) == 512
    assert tp._normalize_ws(0, 8) == 0


def test_normalize_noalloc_validation(tp):
    """Host checks of the allocation-free normaliser, before any device call:
    the raw-data checks of tp_normalize, and sizes beyond its scratch array."""
    nul = ctypes.c_void_p()
    p = ctypes.c_void_p(0x100000)
    f = tp._normalize_noalloc
    assert f(nul, 0, p, 1, p, 1, 0, 4, 2, 8, 0, p, nul) == tp.TP_EINVAL
    assert f(p, 0, p, 0, p, 1, 0, 4, 2, 8, 0, p, nul) == tp.TP_EINVAL
    assert f(p, 0, p, 1, p, 1, 0, 4, 2, 8, 9, p, nul) == tp.TP_EINVAL and "dtype" in tp.last_error()
    assert f(p, 0, p, 1, p, 1, 0, 4, 2, 8, 0, nul, nul) == tp.TP_EINVAL and "sino" in tp.last_error()
    # one row past the limit of n_rows * n_det pixels (2048 x 4096)
    assert f(p, 0, p, 1, p, 1, 0, 4, 2049, 4096, 0, p, nul) == tp.TP_EINVAL
    assert "allocation-free limit" in tp.last_error()
    assert f(p, 0, p, 1, p, 1, 0, 4, 1, 8388609, 0, p, nul) == tp.TP_EINVAL
    assert tp.NOALLOC_MAX_PIXELS == 2048 * 4096


def test_fourier_validation_without_plan(tp):
    nul = ctypes.c_void_p()
    p = ctypes.c_void_p(0x100000)
    assert tp._fourier_ws(nul, 8) == 0
    assert tp._fourier_prepare(nul, tp.TP_RAMP, 0) == tp.TP_EINVAL and "plan" in tp.last_error()
    st = tp._fourier_chunk(nul, p, 0, p, 1, p, 1, 0, 4, tp.TP_RAMP, 0, p, 1 << 20, p, nul)
    assert st == tp.TP_EINVAL and "plan" in tp.last_error()
    arr = (ctypes.c_void_p * 6)()
    st = tp._fourier_chunk_events(nul, p, 0, p, 1, p, 1, 0, 4, tp.TP_RAMP, 0, p, 1 << 20, p, nul, arr)
    assert st == tp.TP_EINVAL


def test_lamino_validation_without_plan(tp):
    nul = ctypes.c_void_p()
    p = ctypes.c_void_p(0x100000)
    assert tp._lamino_prepare(nul, 0.5, 0.0, 8) == tp.TP_EINVAL and "plan" in tp.last_error()
    assert tp._lamino(nul, p, tp.TP_F32, 8, 0.5, 0.0, 8, 0, 8, 1.0, p, nul) == tp.TP_EINVAL


def test_output_tensors_checked_before_the_call(tp):
    # the C ABI gets a bare pointer, so the binding checks a caller's output
    # tensor against what the kernels would write (here on the host: shape,
    # dtype and layout are refused before the device is looked at)
    import torch
    like = torch.empty(1)
    assert tuple(tp._out(None, (2, 3), torch.float32, like).shape) == (2, 3)
    with pytest.raises(ValueError, match="shape"):
        tp._out(torch.empty(2, 4), (2, 3), torch.float32, like)
    with pytest.raises(ValueError, match="shape"):
        tp._out(torch.empty(2, 3, dtype=torch.float16), (2, 3), torch.float32, like)
    with pytest.raises(ValueError, match="shape"):
        tp._out(torch.empty(3, 2).t(), (2, 3), torch.float32, like)  # not contiguous
    with pytest.raises(ValueError, match="must be on"):
        tp._out(torch.empty(2, 3), (2, 3), torch.float32, like)  # a host tensor


# ---------------------------------------------------------------------------
# Lifecycle calls: tp_prepare, tp_tune_load / tp_tune_lookup, tp_shutdown.
# ---------------------------------------------------------------------------
def test_prepare_rejects_bad_arguments(tp):
    nul = ctypes.c_void_p()
    assert tp._prepare(nul, tp.TP_RAMP, tp.TP_F16) == tp.TP_EINVAL
    assert "plan" in tp.last_error()


def _write_table(path, entries):
    import json
    with open(path, "w") as f:
        json.dump(entries, f)


def test_tune_load_reads_the_tuners_cache(tp, tmp_path):
    from paper_2209_08450_amd import tune
    dev = "AMD Instinct MI355X"
    p = str(tmp_path / "tune.json")
    cache = {
        tune.cache_key(dev, "f16", 2048, 2048, 2048, 16): {"choice": [16, 32], "seconds": {"16,32": 0.1,
                                                                                       "8,64": 0.2}},
        tune.cache_key(dev, "f16", 2048, 2048, 2048, 64): {"seconds": {"16,16": 0.1}, "choice": [8, 16]},
        tune.cache_key(dev, "f32", 900, 1024, 1024, 16): {"choice": [16, 8]},
        tune.cache_key("other|gpu", "bf16", 12, 34, 56, 8): {"choice": [4, 64]},
    }
    tune.save_cache(cache, p)  # the tuner's own writer
    tp.tune_load(p)
    # several chunk heights of one shape keep the tallest
    assert tp.tune_lookup(dev, "f16", 2048, 2048, 2048) == (8, 16)
    assert tp.tune_lookup(dev, "f32", 900, 1024, 1024) == (16, 8)
    assert tp.tune_lookup(dev, "f32", 900, 1024, 0) == (16, 8)  # n_vox 0 => n_det
    assert tp.tune_lookup("other|gpu", "bf16", 12, 34, 56) == (4, 64)  # '|' inside the device name
    assert tp.tune_lookup(dev, "bf16", 2048, 2048, 2048) is None
    assert tp.tune_lookup(dev, "f16", 2048, 2048, 1024) is None
    tp.tune_load(None)
    assert tp.tune_lookup(dev, "f32", 900, 1024, 1024) is None


@pytest.mark.parametrize("text,needle", [
    ("[1, 2]", "object"),
    ('{"AMD|f16|na=4|n=8|N=8|rows=2": {"choice": [16, 16]', "expected"),
    ('{"AMD|f16|na=4|n=8|N=8|rows=2": {"choice": [3, 16]}}', "illegal"),
    ('{"AMD|f16|na=4|n=8|N=8|rows=2": {"choice": [16, 16.5]}}', "illegal"),
    ('{"AMD|f32|na=4|n=8|N=8|rows=2": {"choice": [16, 64]}}', "illegal"),  # exceeds LDS
    ('{"AMD|f64|na=4|n=8|N=8|rows=2": {"choice": [16, 16]}}', "key"),
    ('{"AMD|f16|na=0|n=8|N=8|rows=2": {"choice": [16, 16]}}', "key"),
    ('{"f16|na=4|n=8|N=8": {"choice": [16, 16]}}', "key"),
    ('{"AMD|f16|na=4|n=8|N=8|rows=2": {"seconds": {}}}', "choice"),
    ('{"AMD|f16|na=4|n=8|N=8|rows=2": {"choice": [16, 16]}} x', "trailing"),
])
def test_tune_load_rejects_malformed_tables_and_keeps_the_old_one(tp, tmp_path, text, needle):
    good = str(tmp_path / "good.json")
    _write_table(good, {"GPU|f16|na=4|n=8|N=8|rows=2": {"choice": [4, 8]}})
    tp.tune_load(good)
    bad = str(tmp_path / "bad.json")
    with open(bad, "w") as f:
        f.write(text)
    with pytest.raises(tp.TpError) as ei:
        tp.tune_load(bad)
    assert ei.value.status == tp.TP_EINVAL and needle in str(ei.value)
    assert tp.tune_lookup("GPU", "f16", 4, 8, 8) == (4, 8)
    tp.tune_load(None)


def test_tune_load_missing_file(tp, tmp_path):
    with pytest.raises(tp.TpError) as ei:
        tp.tune_load(str(tmp_path / "absent.json"))
    assert "cannot open" in str(ei.value)


def test_tune_load_empty_object_clears(tp, tmp_path):
    p = str(tmp_path / "t.json")
    _write_table(p, {"GPU|f16|na=4|n=8|N=8|rows=2": {"choice": [4, 8]}})
    tp.tune_load(p)
    _write_table(p, {})
    tp.tune_load(p)
    assert tp.tune_lookup("GPU", "f16", 4, 8, 8) is None


def test_shutdown_without_device_state_is_ok(tp):
    # nothing cached on a machine without a GPU: shutdown frees nothing and succeeds
    # (on a GPU machine the lifecycle is tested in a fresh process, test_gpu_lifecycle.py)
    import torch
    if torch.cuda.is_available():
        pytest.skip("device state may exist in this process")
    tp.shutdown()
