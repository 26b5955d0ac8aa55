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
