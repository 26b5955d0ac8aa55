"""The measurement instruments behind the roofline denominators (tp_peak_*):
their work counts and outputs, checked against closed forms and a host
emulation of their access pattern."""
import numpy as np
import pytest

from tests._util import note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_08450_amd import tp as mod
    return mod


def test_peak_fma_counts_and_output(tp):
    import torch
    out = torch.empty(3 * 256, dtype=torch.float32, device="cuda")
    note("peak fma 3 blocks x 50 steps")
    flop = tp.peak_fma(out, 50)
    torch.cuda.synchronize()
    assert flop == 3 * 256 * 50 * 16 * 2
    # every step adds 0.5 * 0.25 = 0.125 exactly: chain c of thread t ends at
    # t + c + 6.25, and the 16 chains sum to 16 t + 120 + 100
    t = np.arange(256, dtype=np.float64)
    assert np.array_equal(out.cpu().numpy().astype(np.float64).reshape(3, 256), np.tile(16 * t + 220, (3, 1)))


def test_peak_dot2_closed_form(tp):
    import torch
    out = torch.empty(2 * 256, dtype=torch.float32, device="cuda")
    note("peak dot2 2 blocks x 100 steps")
    flop = tp.peak_valu("dot2_f16", out, 100)
    torch.cuda.synchronize()
    assert flop == 2 * 256 * 100 * 16 * 4
    # every step adds 0.5 * 0.25 + 0.25 * 0.5 = 0.25 exactly: chain c of thread
    # t ends at t + c + 25, and the 16 chains sum to 16 t + 120 + 400
    t = np.arange(256, dtype=np.float64)
    want = 16 * t + 120 + 16 * 25
    assert np.array_equal(out.cpu().numpy().astype(np.float64).reshape(2, 256), np.tile(want, (2, 1)))


def test_peak_fma_forms_agree(tp):
    import torch
    out = torch.empty(256, dtype=torch.float32, device="cuda")
    note("peak valu forms")
    # the scalar-operand form computes the same chains as the VGPR form
    tp.peak_valu("fma_f32", out, 40)
    a = out.clone()
    tp.peak_valu("fma_f32_sgpr", out, 40)
    assert torch.equal(out, a)
    # fma_mix: every step adds 0.5 (FP16) * 0.25 = 0.125 exactly
    assert tp.peak_valu("fma_mix_f16", out, 64) == 256 * 64 * 16 * 2
    t = np.arange(256, dtype=np.float64)
    assert np.array_equal(out.cpu().numpy().astype(np.float64), 16 * t + 120 + 16 * 8)


def test_peak_lds_reads_match_host_emulation(tp):
    import torch
    iters = 5
    out = torch.empty(2 * 256, dtype=torch.int32, device="cuda")
    note("peak lds 2 blocks x 5 steps")
    nbytes = tp.peak_lds(out, iters)
    torch.cuda.synchronize()
    assert nbytes == 2 * 256 * iters * 16 * 16
    i = np.arange(1024, dtype=np.uint32)
    buf = np.stack([i, 3 * i, 5 * i, 7 * i], axis=1)
    want = np.empty(256, dtype=np.uint32)
    for t in range(256):
        acc = np.zeros(4, dtype=np.uint32)
        idx = t
        for _ in range(iters):
            for u in range(16):
                acc ^= buf[(idx + 64 * u) & 1023]
            idx = (idx + 7) & 1023
        want[t] = acc[0] ^ acc[1] ^ acc[2] ^ acc[3]
    got = out.cpu().numpy().view(np.uint32).reshape(2, 256)
    assert np.array_equal(got, np.tile(want, (2, 1)))


def test_peak_argument_errors(tp):
    import torch
    out = torch.empty(256, dtype=torch.float32, device="cuda")
    with pytest.raises(tp.TpError):
        tp.peak_valu("dot2_f16", out, 0)
    with pytest.raises(tp.TpError):
        tp.peak_lds(torch.empty(256, dtype=torch.int32, device="cuda"), -1)
    with pytest.raises(tp.TpError):
        tp.peak_fma(out[:0], 10)  # no work-groups
