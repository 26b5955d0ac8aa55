"""The allocation-free normaliser (tp_normalize_noalloc) against tp_normalize and
the FP64 oracle, through the C ABI: two calls in a row on one device, the
second smaller, in every storage type and on strided chunk views; the first
call also fills the scratch array to its limit."""
import numpy as np
import pytest

import oracle
from tests._util import note, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_08450_amd import tp as mod
    return mod


def _raw(seed, na, nz, n, n_dark=2, n_flat=3):
    rng = np.random.default_rng(seed)
    proj = rng.integers(0, 4096, (na, nz, n)).astype(np.uint16)
    dark = rng.integers(90, 110, (n_dark, nz, n)).astype(np.uint16)
    flat = rng.integers(3900, 4100, (n_flat, nz, n)).astype(np.uint16)
    flat[0, 0, :3] = dark[0, 0, :3]  # dead pixels: denominator clamped to one count
    return proj, dark, flat


def _check_against_oracle(got, proj, dark, flat, dt):
    want = oracle.normalize(proj, dark, flat)
    got = np.asarray(got, dtype=np.float64)
    if dt == "f32":
        assert np.max(np.abs(got - want) - 2e-6 * np.abs(want)) < 5e-7
    else:
        r = oracle.round_f16(want) if dt == "f16" else oracle.round_bf16(want)
        ulp = 2.0 ** -10 if dt == "f16" else 2.0 ** -7
        assert np.all(np.abs(got - r) <= ulp * np.abs(r) * 1.01 + 1e-6)


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
def test_noalloc_equals_normalize_two_calls(tp, dt):
    import torch
    dev = torch.device("cuda:0")
    # first call: 2 angles x 2048 rows x 4096 columns = the scratch array's limit
    # of n_rows * n_det pixels; second call: a ragged 37 x 5 x 1000 scan
    for k, (na, nz, n) in enumerate([(2, 2048, 4096), (37, 5, 1000)]):
        note(f"noalloc {dt} call {k}: {na}x{nz}x{n}")
        proj, dark, flat = _raw(10 + k, na, nz, n)
        p, d, f = to_dev(proj), to_dev(dark), to_dev(flat)
        out = torch.full((nz, na, n), float("nan"), dtype=tp.torch_dtype(tp.dtype_code(dt)), device=dev)
        tp.normalize_noalloc(p, d, f, out)
        ref = tp.normalize(p, d, f, dt)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (dt, k)
        rows = [0, nz // 2, nz - 1]
        _check_against_oracle(to_host(out[rows]), proj[:, rows], dark[:, rows], flat[:, rows], dt)


def test_noalloc_strided_chunk_views(tp):
    import torch
    note("noalloc strided chunk views")
    proj, dark, flat = _raw(20, 24, 40, 256)
    p, d, f = to_dev(proj), to_dev(dark), to_dev(flat)
    prev = None
    for r0, r1 in [(0, 32), (32, 40)]:  # a 32-row chunk, then an 8-row one
        out = torch.empty((r1 - r0, 24, 256), dtype=torch.float32, device="cuda:0")
        tp.normalize_noalloc(p[:, r0:r1], d[:, r0:r1], f[:, r0:r1], out)
        ref = tp.normalize(p[:, r0:r1], d[:, r0:r1], f[:, r0:r1], "f32")
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        _check_against_oracle(to_host(out), proj[:, r0:r1], dark[:, r0:r1], flat[:, r0:r1], "f32")
        if prev is not None:
            assert not torch.equal(out[:1], prev[:1])
        prev = out


def test_noalloc_rejects_sizes_beyond_the_scratch(tp):
    import torch
    note("noalloc limit")
    proj = torch.zeros((1, 2049, 4096), dtype=torch.int16, device="cuda:0")
    frames = torch.zeros((1, 2049, 4096), dtype=torch.int16, device="cuda:0")
    out = torch.empty((2049, 1, 4096), dtype=torch.float32, device="cuda:0")
    with pytest.raises(tp.TpError, match="allocation-free limit"):
        tp.normalize_noalloc(proj, frames, frames, out)
