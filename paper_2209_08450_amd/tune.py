"""Autotuner for the backprojection kernel's tile parameters.

For one geometry, storage type and chunk size it times every legal
(slices per block, angles per block) pair with HIP events on synthetic
filtered rows, keeps the fastest, applies it to the plan and records it in a
JSON cache (path from $TP_TUNE_CACHE, default ~/.cache/tpfbp/tune.json) keyed
by device name, storage type and shape.  Every choice gives bitwise-identical
results, so tuning never changes an answer, only its speed.
"""
from __future__ import annotations

import json
import os
import tempfile

SLICES = (1, 2, 4, 8, 16)
ANGLES = (8, 16, 32, 64)
LDS_BYTES = 160 * 1024
WINDOW = 48


def bin_pitch(group_bytes: int) -> int:
    """LDS bytes between staged bins (padded by 16 when the group is an even
    number, at least 4, of 16-byte bank groups, as the kernel does)."""
    return group_bytes + 16 if group_bytes >= 64 and (group_bytes // 16) % 2 == 0 else group_bytes


def legal(storage: str, k: int, a: int) -> bool:
    # 4 bytes per slice and staged bin for every storage type: FP32, bf16
    # widened to FP32, or an FP16 pair (Q[j], Q[j+1])
    del storage
    return bin_pitch(k * 4) * a * WINDOW + a * 16 <= LDS_BYTES


def candidates(storage: str, slices=SLICES, angles=ANGLES):
    return [(k, a) for k in slices for a in angles if legal(storage, k, a)]


def cache_path() -> str:
    return os.environ.get("TP_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "tpfbp", "tune.json"))


def cache_key(device: str, storage: str, n_angles: int, n_det: int, n_vox: int, rows: int) -> str:
    return f"{device}|{storage}|na={n_angles}|n={n_det}|N={n_vox}|rows={rows}"


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(d: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(path) or ".", prefix=".tune", suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def choose(measure, cands) -> tuple:
    """The candidate with the smallest measure(k, a) (seconds); ties keep the first."""
    best, best_t = None, float("inf")
    timings = {}
    for k, a in cands:
        t = float(measure(k, a))
        timings[f"{k},{a}"] = t
        if t < best_t:
            best, best_t = (k, a), t
    if best is None:
        raise ValueError("no candidates")
    return best, timings


def tune_backproject(plan, storage: str = "f16", rows: int = 16, reps: int = 3, use_cache: bool = True,
                     path: str | None = None, measure=None, device_name: str | None = None):
    """Pick and apply the fastest backprojection tiling for ``plan``.

    Returns (slices_per_block, angles_per_block).  ``measure(k, a)`` may be
    given to replace the on-device timing (it must return seconds).
    """
    if device_name is None:
        import torch
        device_name = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    key = cache_key(device_name, storage, plan.n_angles, plan.n_det, plan.n_vox, rows)
    cache = load_cache(path) if use_cache else {}
    if key in cache:
        k, a = cache[key]["choice"]
        plan.set_tuning(storage, k, a)
        return int(k), int(a)
    if measure is None:
        measure = _device_measure(plan, storage, rows, reps)
    (k, a), timings = choose(measure, candidates(storage))
    plan.set_tuning(storage, k, a)
    if use_cache:
        cache = load_cache(path)
        cache[key] = {"choice": [k, a], "seconds": timings}
        save_cache(cache, path)
    return k, a


def _device_measure(plan, storage, rows, reps):
    import torch

    from . import tp

    g = torch.Generator(device="cuda").manual_seed(1234)
    q = torch.randn((rows, plan.n_angles, plan.n_det), generator=g, device="cuda").to(tp.torch_dtype(
        tp.dtype_code(storage)))
    out = torch.empty((rows, plan.n_vox, plan.n_vox), dtype=torch.float32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def measure(k, a):
        plan.set_tuning(storage, k, a)
        tp.backproject(plan, q, out=out)  # warm-up (first launch sets attributes)
        best = float("inf")
        for _ in range(reps):
            e0.record()
            tp.backproject(plan, q, out=out)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e-3)
        return best

    return measure
