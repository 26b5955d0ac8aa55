"""GPU parity of tp_normalize and tp_filter against the FP64 oracle (via the C ABI)."""
import math

import numpy as np
import pytest

import oracle
from paper_2209_08450_amd import synth
from tests._util import max_rel, note, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_08450_amd import tp as mod
    return mod


def _raw(seed, na, nz, n, n_dark=2, n_flat=3, lo=50, hi=4000):
    rng = np.random.default_rng(seed)
    proj = rng.integers(lo, hi, (na, nz, n)).astype(np.uint16)
    dark = rng.integers(90, 110, (n_dark, nz, n)).astype(np.uint16)
    flat = rng.integers(3900, 4100, (n_flat, nz, n)).astype(np.uint16)
    return proj, dark, flat


@pytest.mark.parametrize("shape", [(180, 16, 256), (7, 3, 13), (5, 2, 1), (33, 5, 1000)])
def test_normalize_f32(tp, shape):
    import torch
    na, nz, n = shape
    note(f"normalize f32 {shape}")
    proj, dark, flat = _raw(1, na, nz, n)
    got = to_host(tp.normalize(to_dev(proj), to_dev(dark), to_dev(flat), "f32"))
    torch.cuda.synchronize()
    want = oracle.normalize(proj, dark, flat)
    assert got.shape == want.shape
    # -ln in FP32: the FP32 rounding of D, F and t (relative ~1e-7 of t) is an
    # absolute error ~1e-7 in p; the logarithm adds a few ulp of p
    assert np.max(np.abs(got - want) - 2e-6 * np.abs(want)) < 5e-7


@pytest.mark.parametrize("dt", ["f16", "bf16"])
def test_normalize_half_storage(tp, dt):
    proj, dark, flat = _raw(2, 64, 4, 256)
    note(f"normalize {dt}")
    got = to_host(tp.normalize(to_dev(proj), to_dev(dark), to_dev(flat), dt)).astype(np.float64)
    want = oracle.normalize(proj, dark, flat)
    r = oracle.round_f16(want) if dt == "f16" else oracle.round_bf16(want)
    ulp = 2.0 ** -10 if dt == "f16" else 2.0 ** -7
    # RNE of an FP32 value within ~1e-7 of the FP64 one: equal, or one storage
    # ulp apart where the two straddle a rounding boundary
    assert np.all(np.abs(got - r) <= ulp * np.abs(r) * 1.01 + 1e-6)
    assert np.mean(got == r) > 0.99


def test_normalize_edge_cases(tp):
    na, nz, n = 4, 2, 8
    dark = np.full((1, nz, n), 100, np.uint16)
    flat = np.full((1, nz, n), 4100, np.uint16)
    flat[0, 1, 3] = 100  # dead pixel -> denominator 1
    flat[0, 1, 4] = 60   # flat below dark -> denominator 1
    proj = np.full((na, nz, n), 2100, np.uint16)
    proj[:, 0, 0] = 100  # starved -> clamp
    proj[:, 0, 1] = 0
    proj[:, 1, 3] = 101
    note("normalize edge cases")
    got = to_host(tp.normalize(to_dev(proj), to_dev(dark), to_dev(flat), "f32"))
    want = oracle.normalize(proj, dark, flat)
    assert np.allclose(got, want, rtol=1e-6, atol=1e-6)
    assert abs(got[0, 0, 2] - math.log(2.0)) < 1e-7
    assert abs(got[0, 0, 0] + math.log(1e-6)) < 1e-5


def test_normalize_strided_chunk(tp):
    import torch
    proj, dark, flat = _raw(3, 20, 12, 64)
    P, D, F = to_dev(proj), to_dev(dark), to_dev(flat)
    note("normalize strided chunk")
    got = to_host(tp.normalize(P[:, 5:9, :], D[:, 5:9, :], F[:, 5:9, :], "f32"))
    want = oracle.normalize(proj[:, 5:9], dark[:, 5:9], flat[:, 5:9])
    assert np.max(np.abs(got - want) - 2e-6 * np.abs(want)) < 5e-7
    # the rows outside the chunk are untouched inputs; output is exactly the chunk's
    full = to_host(tp.normalize(P, D, F, "f32"))
    assert np.array_equal(full[5:9], got)
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [1, 2, 3, 5, 12, 64, 100, 256, 1000, 2048, 4096])
def test_filter_f32_matches_oracle(tp, n):
    rng = np.random.default_rng(n)
    lines = 7
    p = rng.standard_normal((lines, n)) + 2.0
    note(f"filter f32 n={n}")
    got = to_host(tp.filter(to_dev(p.astype(np.float32))))
    want = oracle.filter_rows(p.astype(np.float32).astype(np.float64))
    # FP32 FFT: error ~ eps * log2(L) relative to the row norm
    assert rel_l2(got, want) < 2e-6
    assert max_rel(got, want) < 1e-5


def test_filter_explicit_pad_and_in_place(tp):
    import torch
    rng = np.random.default_rng(9)
    p = rng.standard_normal((6, 64)).astype(np.float32)
    note("filter explicit pad, in place")
    t = to_dev(p)
    got = to_host(tp.filter(t, pad_len=64))
    want = oracle.filter_rows(p.astype(np.float64), L=64)
    assert rel_l2(got, want) < 2e-6
    tp.filter(t, out=t)  # in place, default pad
    torch.cuda.synchronize()
    assert rel_l2(to_host(t), oracle.filter_rows(p.astype(np.float64))) < 2e-6


@pytest.mark.parametrize("din,dout", [("f32", "f16"), ("f16", "f32"), ("f32", "bf16"), ("bf16", "bf16")])
def test_filter_dtypes(tp, din, dout):
    import torch
    rng = np.random.default_rng(11)
    p = rng.standard_normal((5, 300)) + 1.0
    t = to_dev(p.astype(np.float32)).to(tp.torch_dtype(tp.dtype_code(din)))
    pin = to_host(t).astype(np.float64)  # the stored input
    note(f"filter {din}->{dout}")
    got = to_host(tp.filter(t, out_dtype=dout)).astype(np.float64)
    want = oracle.filter_rows(pin)
    tol = {"f32": 2e-6, "f16": 1e-3, "bf16": 8e-3}[dout]
    assert rel_l2(got, want) < tol
    # element-wise: rounding a value to the output type moves it by at most
    # half an ulp, 2^-11 (FP16) or 2^-8 (BF16) of its magnitude; FP32 FFT
    # rounding adds ~1e-6 of the largest value
    mx = {"f32": 1e-5, "f16": 4.9e-4 + 1e-5, "bf16": 3.9e-3 + 1e-5}[dout]
    assert max_rel(got, want) < mx


def test_filter_odd_line_count_and_large_l(tp):
    rng = np.random.default_rng(12)
    p = rng.standard_normal((3, 6000)).astype(np.float32)  # L = 16384
    note("filter L=16384, odd lines")
    got = to_host(tp.filter(to_dev(p)))
    assert rel_l2(got, oracle.filter_rows(p.astype(np.float64))) < 3e-6
    assert max_rel(got, oracle.filter_rows(p.astype(np.float64))) < 1e-5


@pytest.mark.parametrize("kind", ["shepp", "parzen"])
@pytest.mark.parametrize("n", [1, 13, 256, 1000, 2048, 4096, 6000])
def test_windowed_filter_matches_oracle(tp, kind, n):
    # n spans the LDS FFT (L < 1024 and L = 16384) and the register FFT
    # (1024 <= L <= 8192)
    rng = np.random.default_rng(1000 + n)
    p = rng.standard_normal((5, n)) + 1.5
    note(f"filter {kind} f32 n={n}")
    got = to_host(tp.filter(to_dev(p.astype(np.float32)), kind=kind))
    want = oracle.filter_rows(p.astype(np.float32).astype(np.float64), kind=kind)
    assert rel_l2(got, want) < 3e-6
    assert max_rel(got, want) < 1e-5


@pytest.mark.parametrize("kind", ["shepp", "parzen"])
def test_windowed_filter_f16_out_and_in_place(tp, kind):
    import torch
    rng = np.random.default_rng(77)
    p = rng.standard_normal((4, 700)).astype(np.float32)
    note(f"filter {kind} f32->f16, in place")
    want = oracle.filter_rows(p.astype(np.float64), kind=kind)
    got16 = to_host(tp.filter(to_dev(p), out_dtype="f16", kind=kind)).astype(np.float64)
    assert rel_l2(got16, want) < 1e-3
    assert max_rel(got16, want) < 4.9e-4 + 1e-5
    t = to_dev(p)
    tp.filter(t, out=t, kind=kind)
    torch.cuda.synchronize()
    assert rel_l2(to_host(t), want) < 3e-6


def test_windows_differ_from_ramp(tp):
    rng = np.random.default_rng(5)
    p = to_dev(rng.standard_normal((3, 128)).astype(np.float32))
    note("filter windows differ")
    r = to_host(tp.filter(p))
    s = to_host(tp.filter(p, kind="shepp"))
    z = to_host(tp.filter(p, kind="parzen"))
    assert rel_l2(s, r) > 1e-2 and rel_l2(z, r) > 1e-2 and rel_l2(z, s) > 1e-2


@pytest.mark.parametrize("kind", ["ramp", "parzen"])
def test_filter_widest_rows(tp, kind):
    # n = 8192: pad length 16384, the largest the filter takes
    rng = np.random.default_rng(81)
    p = rng.standard_normal((3, 8192)) + 1.0
    note(f"filter {kind} n=8192")
    got = to_host(tp.filter(to_dev(p.astype(np.float32)), kind=kind))
    want = oracle.filter_rows(p.astype(np.float32).astype(np.float64), kind=kind)
    assert rel_l2(got, want) < 3e-6
    assert max_rel(got, want) < 1e-5
