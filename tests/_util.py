"""Helpers shared by the tests (no method arithmetic)."""
from __future__ import annotations

import sys

import numpy as np


def rel_l2(got, want) -> float:
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


def to_dev(a, device="cuda"):
    """numpy -> device tensor; uint16 raw counts travel as int16 bit patterns."""
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint16:
        a = a.view(np.int16)
    return torch.from_numpy(a).to(device)


def to_host(t) -> np.ndarray:
    import torch
    if t.dtype in (torch.float16, torch.bfloat16):
        t = t.float()
    a = t.detach().cpu().numpy()
    return a


def note(msg: str):
    """Print and flush a line naming the case before a GPU step."""
    print(msg, flush=True)
    sys.stdout.flush()


# Element-wise parity: the largest error of a slice relative to the largest
# magnitude of its reference.  Bounds by storage type of the filtered rows:
# FP32 twice the FP32 path's rel-L2 bar (an error field's maximum sits a few
# standard deviations above its RMS, while a slice's maximum is a few times
# its RMS); FP16 the FP16 path's bar applied to the maximum; BF16 eight times
# that (its unit roundoff 2^-8 is eight times FP16's 2^-11).
MAX_REL = {"f32": 2e-5, "f16": 3e-3, "bf16": 2.4e-2}
REL_L2 = {"f32": 1e-5, "f16": 3e-3, "bf16": 2e-2}

# FP16 rows against the oracle's 16-bit mode (same stored rows, binary16
# weights): the kernel rounds weights computed from its FP32 coordinate, the
# oracle from the FP64 one.  They differ by |dw| ~ 1e-6, so a weight rounds
# to a neighbouring binary16 value (spacing u <= 2^-11) with probability
# ~|dw| / u, which puts sqrt(|dw| u) ~ 3e-5 of a tap's value into each term:
# rel-L2 ~ 3e-5 for sums of random rows; the bars leave a factor 3.
F16_MODE_REL_L2 = 1e-4
F16_MODE_MAX_REL = 4e-4


def max_rel(got, want) -> float:
    """max|got - want| / max|want| over the whole array."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    num, den = float(np.max(np.abs(got - want))), float(np.max(np.abs(want)))
    if den == 0.0:  # a slice every ray misses: it must be exactly zero
        return 0.0 if num == 0.0 else float("inf")
    return num / den


def assert_parity(got, want, storage="f32", rel=None, mx=None, label=""):
    """rel-L2 over the array below ``rel`` and, per slice of the leading axis
    (when the array has 3 dimensions, else over the whole array), the
    element-wise max|got - want| / max|want| below ``mx`` (defaults by storage
    type).  Prints both so the run's log records them; returns (rel-L2, worst
    max-rel)."""
    rel = REL_L2[storage] if rel is None else rel
    mx = MAX_REL[storage] if mx is None else mx
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape, (got.shape, want.shape)
    e = rel_l2(got, want)
    slices = [(got[z], want[z]) for z in range(got.shape[0])] if got.ndim == 3 else [(got, want)]
    m = max(max_rel(g, w) for g, w in slices)
    note(f"{label} {storage}: rel-L2 {e:.3e}, max|err|/max|ref| {m:.3e}")
    assert e < rel, (label, storage, e)
    assert m < mx, (label, storage, m)
    return e, m
