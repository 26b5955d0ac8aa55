#!/usr/bin/env python
"""Benchmark: filtered backprojection of a 2048^3 volume on one MI355X.

Workload (the paper's N = 2048 case, Section 3): 2048 projections over 180
degrees x 2048 detector rows x 2048 columns of 12-bit counts from a seeded
200-ellipsoid phantom (20 darks, 20 flats), reconstructed to 2048^3 float32.
Inputs are generated on the GPU and resident in HBM before timing starts.  A
step is one full FBP of the volume: for each chunk of rows, dark/flat means,
fused normalise + ramp filter, backprojection (tp_fbp_chunk).  Both storage
precisions of the filtered rows are timed: FP16 (the reported value) and FP32.

Printed: ONE JSON line on stdout (progress goes to stderr) with the metric,
per-precision seconds per volume, the FP16/FP32 speed-up, the relative L2 error
of each against the FP64 oracle on full sampled slices, a roofline entry for
the dominant kernel (backprojection) from HIP events around each launch, and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gvoxel-angle updates/s and s per 2048^3 FBP, FP16 vs FP32 at stated L2 error"
UNIT = "Gvoxel-angle updates/s"
# Algorithmic work of one voxel-angle update of the backprojection: detector
# coordinate (1 FMA = 2), interpolation fraction (1), linear interpolation
# (subtract + FMA = 3), accumulation (1).
FLOP_PER_UPDATE = 7
# MI355X fp32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz.
PEAK_FP32_TFLOPS = 157.3


FILTER_NAMES = {"ramp": "ramp filter", "shepp": "Shepp-Logan-windowed ramp filter",
                "parzen": "Parzen-windowed ramp filter"}


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2048, help="detector columns = voxels per side")
    ap.add_argument("--angles", type=int, default=2048)
    ap.add_argument("--rows", type=int, default=2048)
    ap.add_argument("--chunk", type=int, default=256, help="rows per tp_fbp_chunk call")
    ap.add_argument("--storage", default="f16,f32,bf16", help="storage precisions to time (first is reported)")
    ap.add_argument("--precision-slices", type=int, default=32,
                    help="slices sampled for the precision report (rel-L2 and max error vs FP64 per storage)")
    ap.add_argument("--precision-points", type=int, default=2048, help="sampled voxels per precision slice")
    ap.add_argument("--filter", default="ramp", choices=("ramp", "shepp", "parzen"),
                    help="filter window (the paper's tool defaults to parzen; the headline workload is ramp)")
    ap.add_argument("--tuning", default="", help="backprojection tuning K,A (default: plan default)")
    ap.add_argument("--parity-rows", type=int, default=2, help="full slices checked against the oracle")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU-baseline budget: oracle slices are added until this much time is spent (0: skip)")
    ap.add_argument("--pipeline", action="store_true",
                    help="instead: the host-to-host three-stream pipeline over uneven chunks "
                         "(defaults become 3000 angles x 2048 rows x 4096 columns, FP16 storage)")
    ap.add_argument("--pattern", default="32,64,128", help="chunk sizes of the pipeline mode")
    ap.add_argument("--buffers", type=int, default=3,
                    help="pipeline: pinned and device buffers per direction (2: the paper's double buffering)")
    ap.add_argument("--out-dtype", default="f32", choices=("f32", "f16"),
                    help="pipeline mode: precision of the output slices (f16: 16-bit volumes; linear method with FP16 storage, or the Fourier-domain method)")
    ap.add_argument("--io-dir", default="",
                    help="pipeline mode: read the scan from and write the volume to raw files in this directory "
                         "(native reader/writer threads; the files are written first and deleted afterwards)")
    ap.add_argument("--method", default="linear", choices=("linear", "fourier", "lprec"),
                    help="backprojector of the pipeline mode: linear interpolation (tp_fbp_chunk), the "
                         "Fourier-domain method (tp_fourier_fbp_chunk) or the log-polar method "
                         "(tp_lprec_fbp_chunk; 2048^3 in 32-row chunks by default)")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="skip the pipeline section (3000 angles x 2048 rows x 4096 columns host to host, chunks "
                         "32/64/128, FP16 storage)")
    ap.add_argument("--no-ls", action="store_true",
                    help="skip the differentiation section (forward projector, adjoint, 30 LS steps)")
    ap.add_argument("--single-radon", action="store_true",
                    help="instead: one tp_radon of the differentiation workload (128 x 1024^2 x 900), then a 1 GiB "
                         "device copy (a short program for hardware-counter passes)")
    ap.add_argument("--no-fourier", action="store_true",
                    help="skip the Fourier-domain FBP section (tp_fourier_fbp_chunk on the same scan)")
    ap.add_argument("--fourier-half-width", type=int, default=0, help="Gaussian truncation radius (0 = 6)")
    ap.add_argument("--fourier-slices", type=int, default=3, help="slices checked against the oracle's direct sum")
    ap.add_argument("--fourier-points", type=int, default=96, help="sampled voxels per checked slice")
    ap.add_argument("--no-lprec", action="store_true",
                    help="skip the log-polar FBP section (tp_lprec_fbp_chunk on the same scan)")
    ap.add_argument("--lprec-rows", type=int, default=32,
                    help="rows per pass of the log-polar FBP (its workspace: about 1.1 GB per row at 2048^2)")
    ap.add_argument("--lprec-slices", type=int, default=3, help="slices checked against the oracle's direct sum")
    ap.add_argument("--lprec-points", type=int, default=96, help="sampled voxels per checked slice")
    ap.add_argument("--single-lprec", action="store_true",
                    help="instead: one tp_lprec_fbp_chunk of 32 rows of the timed scan shape (a short program for "
                         "hardware-counter passes)")
    ap.add_argument("--no-lamino", action="store_true",
                    help="skip the laminography section (2048^2 x 256 slab from 2048 angles, axis tilted 63 degrees)")
    ap.add_argument("--single-lamino", action="store_true",
                    help="instead: one laminographic backprojection of the bench's slab workload")
    ap.add_argument("--single-fourier", action="store_true",
                    help="instead: one tp_fourier_fbp_chunk of the timed chunk shape, then a 1 GiB device copy "
                         "(a short program for hardware-counter passes)")
    ap.add_argument("--single-launch", action="store_true",
                    help="instead: one tp_fbp_chunk of the timed launch shape, then a 1 GiB device copy "
                         "(a short program for hardware-counter runs; the copy calibrates the byte counters)")
    return ap.parse_args()


PEAK_HBM_GBS = 8000.0
STORAGE_BYTES = {"f32": 4, "f16": 2, "bf16": 2}


def filter_roofline(storage: str, ms_per_volume: float, n_angles: int, rows: int, n_det: int,
                    measured_copy_gbs: float | None = None) -> dict:
    """Roofline entry of k_norm_filter for one volume: algorithmic bytes (2 B
    raw in + the filtered sample out per sample; the dark/flat tables are
    FP32 per row and column, negligible) over its measured time."""
    nbytes = float(n_angles) * rows * n_det * (2 + STORAGE_BYTES[storage])
    gbs = nbytes / (ms_per_volume * 1e-3) / 1e9 if ms_per_volume > 0 else None
    return {"bound": "hbm", "kernel": "k_norm_filter_reg", "achieved": round(gbs, 1) if gbs else None,
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4) if gbs else None,
            "frac_of_measured_copy": round(gbs / measured_copy_gbs, 4) if gbs and measured_copy_gbs else None,
            "bytes_per_volume": nbytes, "ms_per_volume": round(ms_per_volume, 2),
            "note": "moves exactly its algorithmic bytes (FETCH_SIZE / WRITE_SIZE); its time is the FFT arithmetic "
                    "in registers and LDS, about 4 % of a volume's time"}


def host_cpu_model() -> str:
    """The host CPU's model name (for the oracle baseline), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cpu() -> dict:
    """What the host CPU is: lscpu's model, family and topology fields, the
    logical CPU count and the CPUs this process may run on."""
    import subprocess
    info = {"model_name": host_cpu_model(), "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)),
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}
    keys = {"Model name": "lscpu_model_name", "Vendor ID": "vendor", "CPU family": "family", "Model": "model",
            "Socket(s)": "sockets", "Core(s) per socket": "cores_per_socket", "Thread(s) per core": "threads_per_core",
            "CPU max MHz": "max_mhz", "L3 cache": "l3"}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in keys:
                info[keys[k.strip()]] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def measure_peaks(log, copy_bytes: int = 2 << 30, fma_blocks: int = 4096, fma_iters: int = 4096,
                  lds_iters: int = 2048, reps: int = 5):
    """The device rates this library's own kernels reach: a 16-byte-load copy
    (HBM GB/s, read + written bytes), independent multiply-add chains of four
    instruction forms (v_fma_f32 with VGPR operands, the same reading a
    scalar register, v_fma_mix_f32, v_dot2_f32_f16; TFLOP/s and wave64
    instructions per second) and conflict-free 16-byte LDS reads (TB/s summed
    over the CUs).  Best of ``reps`` HIP-event-timed launches after a warm-up."""
    import torch

    from paper_2209_08450_amd import tp
    stream = torch.cuda.current_stream()
    a = torch.ones(copy_bytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    out = torch.empty(fma_blocks * 256, dtype=torch.float32, device="cuda")
    out_i = torch.empty(fma_blocks * 256, dtype=torch.int32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def best(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return min(ts), float(sorted(ts)[len(ts) // 2])

    t_copy, t_copy_med = best(lambda: tp.peak_copy(a, b, stream))
    work = {}
    valu = {}
    for form in tp.VALU_FORMS:
        def run(form=form):
            work[form] = tp.peak_valu(form, out, fma_iters, stream)
        t, t_med = best(run)
        flop_per_inst = 256.0 if form == "dot2_f16" else 128.0  # per wave64 instruction
        valu[form] = {"TFLOPs": round(work[form] / t / 1e12, 2), "TFLOPs_median": round(work[form] / t_med / 1e12, 2),
                      "wave_instructions_per_s": work[form] / t / flop_per_inst}

    def lds():
        work["lds"] = tp.peak_lds(out_i, lds_iters, stream)
    t_lds, _ = best(lds)
    assert torch.equal(b[:1024], a[:1024])
    del a, b, out, out_i
    torch.cuda.empty_cache()
    gbs = 2.0 * copy_bytes / t_copy / 1e9
    lds_tbs = work["lds"] / t_lds / 1e12
    log(f"measured peaks: copy {gbs:.0f} GB/s, " + ", ".join(f"{k} {v['TFLOPs']:.1f} TFLOP/s" for k, v in valu.items())
        + f", LDS reads {lds_tbs:.1f} TB/s")
    return {"hbm_copy_GBs": round(gbs, 1), "hbm_copy_GBs_median": round(2.0 * copy_bytes / t_copy_med / 1e9, 1),
            "copy_bytes": copy_bytes,
            "fp32_fma_nonpacked_TFLOPs": valu["fma_f32"]["TFLOPs"],
            "fp32_fma_nonpacked_TFLOPs_median": valu["fma_f32"]["TFLOPs_median"],
            "valu_wave_instructions_per_s": valu["fma_f32"]["wave_instructions_per_s"],
            "dot2_wave_instructions_per_s": valu["dot2_f16"]["wave_instructions_per_s"],
            "valu_forms": valu,
            "lds_read_TBs": round(lds_tbs, 2),
            "note": "project-written kernels (tp_peak_copy, tp_peak_valu, tp_peak_lds) built like every kernel "
                    f"here; best of {reps} event-timed launches"}


def load_valu_counters(storage: str, chunk: int, n: int, angles: int):
    """VALU wave-instructions per backprojection launch from committed
    rocprofv3 SQ counters, if they were taken on the current kernel source and
    this launch shape."""
    p = os.path.join(ROOT, "profiles", "valu_backproject.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except ValueError:
        return None
    e = d.get(storage)
    if not e or d.get("kernel_sha") != kernel_source_hash():
        return None
    if (e.get("chunk"), e.get("n"), e.get("angles")) != (chunk, n, angles):
        return None
    return e


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_2209_08450_amd", "csrc", "k_backproject.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def load_lamino_traffic():
    """HBM traffic per laminography launch from committed rocprofv3 counters,
    if they were taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic_lamino.json")
    src = os.path.join(ROOT, "paper_2209_08450_amd", "csrc", "k_lamino.hip")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except ValueError:
        return None
    if d.get("kernel_sha") != hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]:
        return None
    e = d.get("f16") or {}
    c = LAMINO
    if (e.get("n"), e.get("angles"), e.get("slices"), e.get("tilt")) != (c["n"], c["angles"], c["slices"], c["tilt"]):
        return None
    return float(e["bytes_per_launch"])


def load_traffic(storage: str, chunk: int, n: int, angles: int):
    """HBM traffic per backprojection launch from committed rocprofv3 counters,
    if they were taken on the current kernel source and this launch shape."""
    p = os.path.join(ROOT, "profiles", "traffic_backproject.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except ValueError:
        return None
    e = d.get(storage)
    if not e or d.get("kernel_sha") != kernel_source_hash():
        return None
    if (e.get("chunk"), e.get("n"), e.get("angles")) != (chunk, n, angles):
        return None
    return float(e["bytes_per_launch"])


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1 "
              "(slices are independent; the path would shard by slice)", file=sys.stderr)
        sys.exit(2)
    if args.pipeline:
        return main_pipeline(args)
    if args.single_launch:
        return main_single_launch(args)
    if args.single_radon:
        return main_single_radon(args)
    if args.single_fourier:
        return main_single_fourier(args)
    if args.single_lprec:
        return main_single_lprec(args)
    if args.single_lamino:
        return main_single_lamino(args)

    import numpy as np
    import torch

    from paper_2209_08450_amd import synth, tp

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, na, rows, chunk = args.n, args.angles, args.rows, min(args.chunk, args.rows)
    storages = [s.strip() for s in args.storage.split(",") if s.strip()]
    center = n / 2.0

    # ---------------- measured denominators of the roofline ----------------
    peaks = measure_peaks(log)

    # ---------------- inputs, resident in HBM ----------------
    t0 = time.time()
    log(f"generating {na} x {rows} x {n} 12-bit scan on the GPU")
    last = [time.time()]

    def progress(done, total):
        if time.time() - last[0] > 10:
            log(f"  generated rows {done}/{total}")
            last[0] = time.time()

    scan = synth.ellipsoid_scan_torch(seed=2, n_angles=na, n_rows=rows, n_det=n, device=dev, center=center,
                                      progress=progress)
    torch.cuda.synchronize()
    log(f"inputs ready in {time.time() - t0:.1f} s: proj {tuple(scan.proj.shape)} "
        f"({scan.proj.numel() * 2 / 1e9:.1f} GB)")

    plan = tp.Plan(scan.angles, n, center)
    if args.tuning:
        k, a = (int(v) for v in args.tuning.split(","))
        for st in storages:
            plan.set_tuning(st, k, a)
    tuning = {st: list(plan.get_tuning(st)) for st in storages}
    vol = torch.empty((rows, n, n), dtype=torch.float32, device=dev)
    ws = torch.empty(max(plan.fbp_workspace_bytes(chunk, s) for s in storages), dtype=torch.uint8, device=dev)
    chunks = [(z0, min(rows, z0 + chunk)) for z0 in range(0, rows, chunk)]
    stream = torch.cuda.current_stream()
    updates = float(n) * n * na * rows

    parity_z = [int(z) for z in np.linspace(rows // 8, rows - rows // 8, args.parity_rows).round()] \
        if args.parity_rows > 0 else []
    # precision report: evenly spaced slices (32 + 64k for 2048 rows), seeded voxel samples
    nps = min(args.precision_slices, rows)
    prec_z = [int((k + 0.5) * rows / nps) for k in range(nps)] if nps > 0 else []
    prng = np.random.default_rng(2048)
    prec_ix = {z: prng.integers(0, n, args.precision_points) for z in prec_z}
    prec_iy = {z: prng.integers(0, n, args.precision_points) for z in prec_z}
    results = {}
    for st in storages:
        # events per chunk: before darkflat, before norm+filter, before BP, after BP
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in chunks]
        for row in evs:
            for e in row:
                e.record(stream)  # create the underlying HIP events

        def step(record):
            for ci, (z0, z1) in enumerate(chunks):
                tp.fbp_chunk(plan, scan.proj[:, z0:z1], scan.dark[:, z0:z1], scan.flat[:, z0:z1], st,
                             out=vol[z0:z1], workspace=ws, events=evs[ci] if record else None, kind=args.filter)

        for _ in range(args.warmup):
            step(False)
        torch.cuda.synchronize()
        log(f"[{st}] warmup done; timing {args.steps} steps")
        stage = np.zeros(3)
        bp_times = []
        t_start = time.perf_counter()
        for s_i in range(args.steps):
            step(True)
            torch.cuda.synchronize()
            for row in evs:
                d = [row[i].elapsed_time(row[i + 1]) for i in range(3)]
                stage += d
                bp_times.append(d[2])
            log(f"[{st}] step {s_i + 1}/{args.steps} done")
        t_total = time.perf_counter() - t_start
        sec = t_total / args.steps
        samples = {z: vol[z].detach().cpu().numpy().astype(np.float64) for z in parity_z}
        points = {z: vol[z][torch.from_numpy(prec_iy[z]).to(dev), torch.from_numpy(prec_ix[z]).to(dev)]
                  .cpu().numpy().astype(np.float64) for z in prec_z}
        results[st] = {
            "s_per_volume": sec,
            "gups": updates / sec / 1e9,
            "stage_ms_per_step": {"darkflat": stage[0] / args.steps, "norm_filter": stage[1] / args.steps,
                                  "backproject": stage[2] / args.steps},
            "bp_launch_ms": float(np.mean(bp_times)),
            "samples": samples,
            "points": points,
        }
        log(f"[{st}] {sec:.3f} s per volume, {updates / sec / 1e9:.1f} Gupd/s, "
            f"BP launch {np.mean(bp_times):.2f} ms")

    # ---------------- FP64 oracle: parity slices and CPU baseline ----------------
    import oracle

    def oracle_slice(z):
        p = scan.proj[:, z, :].cpu().numpy().view(np.uint16)[:, None, :]
        d = scan.dark[:, z, :].cpu().numpy().view(np.uint16)[:, None, :]
        f = scan.flat[:, z, :].cpu().numpy().view(np.uint16)[:, None, :]
        t1 = time.perf_counter()
        v = oracle.fbp(p, d, f, scan.angles, center, kind=args.filter)[0]
        return v, time.perf_counter() - t1

    rel = {st: None for st in storages}
    cpu_t, cpu_slices = 0.0, 0
    ref = {}
    for z in parity_z:
        log(f"oracle FBP of slice {z} ({oracle.num_threads()} threads)")
        ref[z], dt = oracle_slice(z)
        cpu_t += dt
        cpu_slices += 1
    for st in storages:
        if parity_z:
            num = sum(np.sum((results[st]["samples"][z] - ref[z]) ** 2) for z in parity_z)
            den = sum(np.sum(ref[z] ** 2) for z in parity_z)
            rel[st] = float(math.sqrt(num / den))
            log(f"[{st}] rel-L2 vs FP64 oracle on slices {parity_z}: {rel[st]:.3e}")
    precision = None
    if prec_z:
        log(f"oracle FBP at {args.precision_points} voxels of each of {len(prec_z)} slices")
        want = {}
        for z in prec_z:
            p = scan.proj[:, z, :].cpu().numpy().view(np.uint16)
            d = scan.dark[:, z, :].cpu().numpy().view(np.uint16)
            f = scan.flat[:, z, :].cpu().numpy().view(np.uint16)
            want[z] = oracle.fbp_points(p, d, f, scan.angles, center, n, prec_ix[z], prec_iy[z], kind=args.filter)
        w_all = np.concatenate([want[z] for z in prec_z])
        precision = {"slices": prec_z if len(prec_z) <= 8 else f"{len(prec_z)} evenly spaced, {prec_z[0]} + "
                     f"{prec_z[1] - prec_z[0]}k", "points_per_slice": args.precision_points}
        for st in storages:
            g_all = np.concatenate([results[st]["points"][z] for z in prec_z])
            err = g_all - w_all
            precision[st] = {"rel_l2": float(np.linalg.norm(err) / np.linalg.norm(w_all)),
                             "max_abs_over_max_ref": float(np.max(np.abs(err)) / np.max(np.abs(w_all)))}
            log(f"[{st}] sampled precision: rel-L2 {precision[st]['rel_l2']:.3e}, "
                f"max|err|/max|ref| {precision[st]['max_abs_over_max_ref']:.3e}")
    cpu = None
    if args.cpu_seconds > 0:
        extra = [z for z in range(0, rows, max(1, rows // 16)) if z not in parity_z]
        while (cpu_t < args.cpu_seconds or cpu_slices == 0) and extra:
            z = extra.pop(0)
            log(f"oracle FBP of slice {z} for the CPU baseline")
            _, dt = oracle_slice(z)
            cpu_t += dt
            cpu_slices += 1
        cpu_updates = float(n) * n * na * cpu_slices
        cpu = {"value": round(cpu_updates / cpu_t / 1e9, 4), "unit": UNIT, "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{cpu_slices} full slices of the workload ({na} angles x {n} cols -> {n}^2; "
                         f"normalise, filter, backproject in FP64), {cpu_t:.1f} s",
               "s_per_volume_extrapolated": round(cpu_t / cpu_slices * rows, 1), "cpu_model": host_cpu_model(),
               "host": host_cpu()}
        cpu["single_thread"] = oracle_single_thread(scan, center, n, na, rows, args, log)

    # ---------------- Fourier-domain FBP on the same scan ----------------
    fourier = None
    if not args.no_fourier:
        fourier = bench_fourier(args, scan, plan, vol, chunks, stream, updates, log)

    # ---------------- log-polar FBP on the same scan ----------------
    lprec = None
    if not args.no_lprec:
        lprec = bench_lprec(args, scan, plan, vol, stream, updates, log)

    # ---------------- laminography (tilted axis) ----------------
    lamino = None
    if not args.no_lamino:
        del scan, vol
        torch.cuda.empty_cache()
        lamino = bench_lamino(args, log)

    # ---------------- differentiation form: forward projector and least squares ----------------
    ls = None
    if not args.no_ls:
        ls = bench_ls(plan_cls=tp.Plan, log=log)

    # ---------------- batching form: host-to-host three-stream pipeline ----------------
    pipe = None
    if not args.no_pipeline:
        if lamino is None:
            del scan, vol
            torch.cuda.empty_cache()
        pipe = pipeline_run(dev, 4096, 3000, 2048, "f16", (32, 64, 128), "linear", args.filter, "", log,
                            buffers=args.buffers)
        pipe = {k: pipe[k] for k in ("value", "unit", "config", "s_host_to_host", "s_compute_only_resident",
                                      "compute_over_host_to_host", "h2d_GB", "d2h_GB", "vs_fp64_oracle_sampled",
                                      "bitwise_equal_to_resident_compute")}
        pipe["note"] = ("PCIe-inclusive: raw counts from pageable host memory through pinned buffers to the device "
                        "and slices back to pinned host memory; value = updates per host-to-host second")

    # ---------------- report ----------------
    head = storages[0]
    r = results[head]
    bp_updates = float(n) * n * na * chunk
    achieved = FLOP_PER_UPDATE * bp_updates / (r["bp_launch_ms"] * 1e-3) / 1e12
    traffic = load_traffic(head, chunk, n, na)
    valu = load_valu_counters(head, chunk, n, na)
    if valu is not None:
        insts = float(valu["valu_insts_per_launch"])
        t_launch = r["bp_launch_ms"] * 1e-3
        # FP16 rows: one v_dot2 per slice and voxel-angle (per wave: one per 64
        # updates), issued at the dot2 rate; every other VALU instruction at the
        # FP32 FMA rate.  LDS: the bytes the taps read per update (an FP16 pair,
        # or two FP32 values).
        dot2 = bp_updates / 64.0 if head == "f16" else 0.0
        t_valu = dot2 / peaks["dot2_wave_instructions_per_s"] + (insts - dot2) / peaks["valu_wave_instructions_per_s"]
        lds_bytes = bp_updates * (4.0 if head == "f16" else 8.0)
        valu = {"valu_insts_per_launch": insts, "valu_insts_per_update": round(insts * 64 / bp_updates, 3),
                "dot2_insts_per_launch": dot2,
                "valu_busy_frac": round(t_valu / t_launch, 4),
                "lds_tap_bytes_per_launch": lds_bytes,
                "lds_busy_frac": round(lds_bytes / t_launch / (peaks["lds_read_TBs"] * 1e12), 4),
                "source": "profiles/valu_backproject.json (rocprofv3 SQ_INSTS_VALU on this kernel source); "
                          "busy fractions: issue time at the measured dot2 and FP32 FMA rates, tap bytes at the "
                          "measured LDS read rate, over the launch time"}
    out = {
        "metric": METRIC,
        "value": round(r["gups"], 3),
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["s_per_volume"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"fbp {n}x{n}x{rows} volume from {na} angles x {rows} rows x {n} cols "
                               f"12-bit ellipsoid scan, {FILTER_NAMES[args.filter]}, linear-interpolation "
                               f"backprojection",
                   "storage": head, "chunk_rows": chunk, "bp_tuning": tuning},
        "s_per_volume": {st: round(results[st]["s_per_volume"], 4) for st in storages},
        "gups": {st: round(results[st]["gups"], 2) for st in storages},
        "rel_l2_vs_fp64_oracle": rel,
        "precision_sampled_vs_fp64_oracle": precision,
        "stage_ms_per_step": {st: {k: round(v, 2) for k, v in results[st]["stage_ms_per_step"].items()}
                              for st in storages},
        "roofline": {"bound": "alu", "kernel": "k_backproject", "achieved": round(achieved, 2),
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "frac_of_measured_fma_rate": round(achieved / peaks["fp32_fma_nonpacked_TFLOPs"], 4),
                     "traffic": traffic,
                     "launch_ms": round(r["bp_launch_ms"], 3),
                     "flop_per_launch": FLOP_PER_UPDATE * bp_updates,
                     "executed": valu,
                     "note": "achieved = 7 algorithmic flop per voxel-angle update / launch time; the kernel "
                             "shares the coordinate, fraction and weights of a voxel and angle over 16 slices and "
                             "(FP16 rows) adds both taps of a slice with one v_dot2, so it issues fewer VALU "
                             "instructions than 7 flop per update (see executed)"},
        "measured_peaks": peaks,
        # the fused normalise + filter kernel: HBM-class work (uint16 raw sample
        # in, one filtered sample out in the storage type, per sample of the
        # scan), from the HIP events around its launches
        "filter_roofline": {st: filter_roofline(st, results[st]["stage_ms_per_step"]["norm_filter"], na, rows, n,
                                                peaks["hbm_copy_GBs"])
                            for st in storages},
        "cpu_baseline": cpu,
        "differentiation": ls,
        "fourierrec": fourier,
        "lprec": lprec,
        "laminography": lamino,
        "pipeline": pipe,
        "paper_context": {"linerec_fp32_2048cubed_total_s_A100_incl_io": 80.0},
    }
    if "f16" in results and "f32" in results:
        out["speedup_f16_vs_f32"] = round(results["f32"]["s_per_volume"] / results["f16"]["s_per_volume"], 3)
    print(json.dumps(out), flush=True)
    plan.close()


def oracle_single_thread(scan, center, n, na, rows, args, log):
    """The oracle on one thread: one slice's normalise + filter (numpy FP64),
    timed, then its backprojection at whole rows of voxels (C, FP64, one
    OpenMP thread) until about ``args.cpu_seconds / 2`` is spent; the slice
    time is extrapolated from the sampled rows."""
    import numpy as np

    import oracle
    z = rows // 2
    p = scan.proj[:, z, :].cpu().numpy().view(np.uint16)
    d = scan.dark[:, z, :].cpu().numpy().view(np.uint16)
    f = scan.flat[:, z, :].cpu().numpy().view(np.uint16)
    before = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        q = oracle.filter_rows(oracle.normalize(p[:, None, :], d[:, None, :], f[:, None, :])[0], kind=args.filter)
        t_filter = time.perf_counter() - t0
        t_bp, vox_rows, step = 0.0, 0, 8
        budget = max(2.0, 0.5 * args.cpu_seconds)
        while t_bp < budget and vox_rows < n:
            k = min(step, n - vox_rows)
            iy, ix = np.meshgrid(np.arange(vox_rows, vox_rows + k), np.arange(n), indexing="ij")
            t1 = time.perf_counter()
            oracle.backproject_points(q, scan.angles, center, n, ix.ravel(), iy.ravel())
            t_bp += time.perf_counter() - t1
            vox_rows += k
            step *= 2
    finally:
        oracle.set_num_threads(before)
    s_slice = t_filter + t_bp * n / vox_rows
    log(f"oracle on one thread: filter {t_filter:.2f} s, backprojection of {vox_rows} voxel rows {t_bp:.2f} s, "
        f"{s_slice:.1f} s per slice")
    return {"value": round(float(n) * n * na / s_slice / 1e9, 4), "unit": UNIT, "cores": 1, "kind": "oracle",
            "sample": f"slice {z}: normalise + filter of its {na} rows ({t_filter:.2f} s), backprojection of "
                      f"{vox_rows} of its {n} voxel rows ({t_bp:.2f} s); slice time extrapolated to "
                      f"{s_slice:.1f} s",
            "s_per_volume_extrapolated": round(s_slice * rows, 1)}


def fourier_flop_per_pair(n_angles: int, pad_len: int, half_width: int) -> float:
    """Algorithmic work of the gather for one pair of slices: every polar
    sample (n_angles x (pad_len + 1)) meets the (2 half_width)^2 grid points
    of its truncated Gaussian (one grid point per sample along the ray at the
    paper's sizes); per meeting 2 flop for the weight (two-ratio recurrence)
    and 4 for the complex-by-real multiply-accumulate."""
    return float(n_angles) * (pad_len + 1) * (2 * half_width) ** 2 * 6


def bench_fourier(args, scan, plan, vol, chunks, stream, updates, log):
    """Fourier-domain FBP (tp_fourier_fbp_chunk) of the resident scan in the
    same chunks: time per volume, per-stage times, the gather's roofline and
    parity at sampled voxels against the oracle's direct sum (which is also
    timed on the host)."""
    import numpy as np
    import torch

    import oracle
    from paper_2209_08450_amd import tp

    n, na, rows = plan.n_det, plan.n_angles, vol.shape[0]
    chunk = chunks[0][1] - chunks[0][0]
    hw = args.fourier_half_width or 6
    plan.fourier_prepare(args.filter, hw)
    ws = torch.empty(plan.fourier_workspace_bytes(chunk), dtype=torch.uint8, device=vol.device)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in chunks]
    for row in evs:
        for e in row:
            e.record(stream)

    def step(record):
        for ci, (z0, z1) in enumerate(chunks):
            tp.fourier_fbp_chunk(plan, scan.proj[:, z0:z1], scan.dark[:, z0:z1], scan.flat[:, z0:z1],
                                 out=vol[z0:z1], workspace=ws, events=evs[ci] if record else None, kind=args.filter,
                                 half_width=hw)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log(f"[fourier] warmup done; timing {args.steps} steps")
    stage = np.zeros(5)
    grid_ms = []
    t0 = time.perf_counter()
    for s_i in range(args.steps):
        step(True)
        torch.cuda.synchronize()
        for row in evs:
            d = [row[i].elapsed_time(row[i + 1]) for i in range(5)]
            stage += d
            grid_ms.append(d[2])
        log(f"[fourier] step {s_i + 1}/{args.steps} done")
    sec = (time.perf_counter() - t0) / args.steps
    L = tp.pad_len(n)
    flop = fourier_flop_per_pair(na, L, hw) * ((chunk + 1) // 2)
    achieved = flop / (np.mean(grid_ms) * 1e-3) / 1e12
    log(f"[fourier] {sec:.3f} s per volume, gather {np.mean(grid_ms):.2f} ms per chunk "
        f"({achieved:.1f} TFLOP/s algorithmic)")
    # parity at sampled voxels; the same oracle evaluations time the CPU side
    ns = min(args.fourier_slices, rows)
    zs = [int((k + 0.5) * rows / ns) for k in range(ns)] if ns > 0 else []
    rng = np.random.default_rng(4096)
    errs, num, den, cpu_t, cpu_pts = [], 0.0, 0.0, 0.0, 0
    for z in zs:
        ix = rng.integers(0, n, args.fourier_points)
        iy = rng.integers(0, n, args.fourier_points)
        got = vol[z][torch.from_numpy(iy).to(vol.device), torch.from_numpy(ix).to(vol.device)].cpu().numpy()
        p = scan.proj[:, z, :].cpu().numpy().view(np.uint16)
        d = scan.dark[:, z, :].cpu().numpy().view(np.uint16)
        f = scan.flat[:, z, :].cpu().numpy().view(np.uint16)
        log(f"[fourier] oracle direct sum at {args.fourier_points} voxels of slice {z}")
        t1 = time.perf_counter()
        want = oracle.fourier_fbp_points(p, d, f, scan.angles, plan.center, n, ix, iy, kind=args.filter)
        cpu_t += time.perf_counter() - t1
        cpu_pts += len(ix)
        e = got.astype(np.float64) - want
        num += float(np.sum(e ** 2))
        den += float(np.sum(want ** 2))
        errs.append(float(np.max(np.abs(e)) / np.max(np.abs(want))))
    rel = math.sqrt(num / den) if den > 0 else None
    if rel is not None:
        log(f"[fourier] rel-L2 vs FP64 direct sum at sampled voxels: {rel:.3e}")
    return {
        "method": "Fourier-domain backprojection: polar spectra, Gaussian gather onto a 2x oversampled grid, "
                  "2-D inverse FFT, deconvolution",
        "half_width": hw,
        "s_per_volume": round(sec, 4),
        "gups_equivalent": round(updates / sec / 1e9, 2),
        "stage_ms_per_step": {k: round(v / args.steps, 2) for k, v in
                              zip(("darkflat", "spectra", "grid", "ifft_rows", "ifft_cols"), stage)},
        "rel_l2_vs_fp64_direct_sum_sampled": rel,
        "max_abs_over_max_ref_per_slice": errs,
        "parity_sample": f"{args.fourier_points} voxels of each of slices {zs}",
        "roofline_gather": {"bound": "alu", "kernel": "k_fr_grid", "achieved": round(achieved, 2),
                            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                            "launch_ms": round(float(np.mean(grid_ms)), 3), "flop_per_launch": flop},
        "cpu_oracle": {"value": round(cpu_pts * na / cpu_t / 1e9, 6) if cpu_t > 0 else None,
                       "unit": "Gvoxel-angle updates/s", "cores": oracle.num_threads(),
                       "sample": f"direct sum at {cpu_pts} voxels ({L + 1} terms per voxel-angle), {cpu_t:.1f} s"},
    }


def lprec_conv_flop_per_pair(g: dict) -> float:
    """Algorithmic work of the log-polar convolution kernel per pair of slices:
    for every span and sigma frequency, the angle column's FFT (length NA/M),
    the product with the kernel's transform (NA complex multiplies) and the
    inverse FFT (length NA); 5 n log2 n real flop per complex FFT of length n,
    6 per complex multiply."""
    na_c = g["NA"] // g["M"]
    fft = lambda n: 5.0 * n * math.log2(n)
    return float(g["spans"]) * g["Ns"] * (fft(na_c) + 6.0 * g["NA"] + fft(g["NA"]))


def lprec_conv_bytes_per_pair(g: dict) -> float:
    """Algorithmic bytes of the convolution kernel per pair: the angle columns
    read (spans x Ns x n_span complex FP32) and the kept rows written
    (spans x rows x Ns complex FP32)."""
    return 8.0 * g["spans"] * g["Ns"] * (g["n_span"] + g["rows"])


def bench_lprec(args, scan, plan, vol, stream, updates, log):
    """Log-polar FBP (tp_lprec_fbp_chunk) of the resident scan, in passes of
    --lprec-rows rows: time per volume, per-stage times of one pass, the
    convolution kernel's roofline and parity at sampled voxels against the
    oracle's direct sum of trigonometric interpolants (the sum it
    approximates)."""
    import numpy as np
    import torch

    import oracle
    from paper_2209_08450_amd import tp

    n, na, rows = plan.n_det, plan.n_angles, vol.shape[0]
    chunk = args.lprec_rows
    plan.lprec_prepare(args.filter)
    g = tp.lprec_grid(na, plan.n_vox)
    ws = torch.empty(plan.lprec_workspace_bytes(chunk), dtype=torch.uint8, device=vol.device)
    chunks = [(z0, min(rows, z0 + chunk)) for z0 in range(0, rows, chunk)]
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
    for e in evs:
        e.record(stream)

    def step(record):
        for ci, (z0, z1) in enumerate(chunks):
            tp.lprec_fbp_chunk(plan, scan.proj[:, z0:z1], scan.dark[:, z0:z1], scan.flat[:, z0:z1], out=vol[z0:z1],
                               workspace=ws, events=evs if (record and ci == 0) else None, kind=args.filter)

    # a few steps only: one volume takes seconds
    steps, warmup = max(1, min(args.steps, 3)), min(args.warmup, 1)
    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    log(f"[lprec] warmup done; timing {steps} steps")
    stage = np.zeros(6)
    t0 = time.perf_counter()
    for s_i in range(steps):
        step(True)
        torch.cuda.synchronize()
        stage += [evs[i].elapsed_time(evs[i + 1]) for i in range(6)]
        log(f"[lprec] step {s_i + 1}/{steps} done")
    sec = (time.perf_counter() - t0) / steps
    stage /= steps
    pairs = (chunk + 1) // 2
    conv_ms = float(stage[3])
    flop = lprec_conv_flop_per_pair(g) * pairs
    achieved = flop / (conv_ms * 1e-3) / 1e12
    gbs = lprec_conv_bytes_per_pair(g) * pairs / (conv_ms * 1e-3) / 1e9
    log(f"[lprec] {sec:.3f} s per volume; convolution {conv_ms:.2f} ms per {chunk}-row pass "
        f"({achieved:.1f} TFLOP/s, {gbs:.0f} GB/s algorithmic)")
    ns = min(args.lprec_slices, rows)
    zs = [int((k + 0.5) * rows / ns) for k in range(ns)] if ns > 0 else []
    rng = np.random.default_rng(8192)
    errs, num, den, cpu_t, cpu_pts = [], 0.0, 0.0, 0.0, 0
    for z in zs:
        ix = rng.integers(0, n, args.lprec_points)
        iy = rng.integers(0, n, args.lprec_points)
        got = vol[z][torch.from_numpy(iy).to(vol.device), torch.from_numpy(ix).to(vol.device)].cpu().numpy()
        p = scan.proj[:, z, :].cpu().numpy().view(np.uint16)
        d = scan.dark[:, z, :].cpu().numpy().view(np.uint16)
        f = scan.flat[:, z, :].cpu().numpy().view(np.uint16)
        log(f"[lprec] oracle direct sum at {args.lprec_points} voxels of slice {z}")
        t1 = time.perf_counter()
        want = oracle.fourier_fbp_points(p, d, f, scan.angles, plan.center, n, ix, iy, kind=args.filter)
        cpu_t += time.perf_counter() - t1
        cpu_pts += len(ix)
        e = got.astype(np.float64) - want
        num += float(np.sum(e ** 2))
        den += float(np.sum(want ** 2))
        errs.append(float(np.max(np.abs(e)) / np.max(np.abs(want))))
    rel = math.sqrt(num / den) if den > 0 else None
    if rel is not None:
        log(f"[lprec] rel-L2 vs FP64 direct sum at sampled voxels: {rel:.3e}")
    return {
        "method": "log-polar backprojection: half-sample quintic row splines, per span of angles a convolution in "
                  "(angle, log-radius) by FFTs, quintic spline evaluation at the voxels",
        "grid": {k: g[k] for k in ("spans", "n_span", "Ns", "NA", "M", "rows", "nj", "os", "eps")},
        "s_per_volume": round(sec, 4),
        "gups_equivalent": round(updates / sec / 1e9, 2),
        "rows_per_pass": chunk,
        "steps": steps,
        "stage_ms_first_pass": {k: round(float(v), 2) for k, v in
                                zip(("darkflat", "row_splines", "logradial_fft", "conv", "sigma_ifft", "interp"),
                                    stage)},
        "rel_l2_vs_fp64_direct_sum_sampled": rel,
        "max_abs_over_max_ref_per_slice": errs,
        "parity_sample": f"{args.lprec_points} voxels of each of slices {zs}",
        "roofline_conv": {"bound": "alu", "kernel": "k_lp_conv", "achieved": round(achieved, 2),
                          "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                          "hbm_GBs_algorithmic": round(gbs, 1), "launch_ms": round(conv_ms, 3),
                          "flop_per_launch": flop},
        "cpu_oracle_direct_sum": {"value": round(cpu_pts * na / cpu_t / 1e9, 6) if cpu_t > 0 else None,
                                  "unit": "Gvoxel-angle updates/s", "cores": oracle.num_threads(),
                                  "sample": f"direct sum at {cpu_pts} voxels, {cpu_t:.1f} s"},
    }


def main_single_lprec(args):
    import torch

    from paper_2209_08450_amd import synth, tp

    n, na, rows = args.n, args.angles, 32
    scan = synth.ellipsoid_scan_torch(seed=2, n_angles=na, n_rows=rows, n_det=n, device="cuda", center=n / 2.0)
    plan = tp.Plan(scan.angles, n, n / 2.0)
    plan.lprec_prepare(args.filter)
    vol = torch.empty((rows, n, n), dtype=torch.float32, device="cuda")
    ws = torch.empty(plan.lprec_workspace_bytes(rows), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    tp.lprec_fbp_chunk(plan, scan.proj, scan.dark, scan.flat, out=vol, workspace=ws, kind=args.filter)
    torch.cuda.synchronize()
    print(json.dumps({"single_lprec": {"rows": rows, "n": n, "angles": na, "grid": tp.lprec_grid(na, n)}}),
          flush=True)
    plan.close()


LAMINO = dict(n=2048, rows=2048, angles=2048, slices=256, tilt=1.1, center_v=1023.5)
LAMINO_FLOP_PER_UPDATE = 8  # bilinear: 3 lerps (2 each); accumulate 1; row coordinate 1


def lamino_setup(dev):
    """The laminography workload: random FP16 filtered projections of a
    2048 x 2048 detector at 2048 angles over a full turn, axis tilted by
    1.1 rad (63 degrees) from the beam, reconstructed into a 256-slice slab of
    2048^2 (timing does not depend on the values; parity is checked against
    the oracle at sampled voxels)."""
    import numpy as np
    import torch

    from paper_2209_08450_amd import tp

    c = LAMINO
    ang = np.arange(c["angles"]) * 2 * math.pi / c["angles"]
    g = torch.Generator(device=dev).manual_seed(63)
    filt = torch.randn((c["angles"], c["rows"], c["n"]), generator=g, device=dev, dtype=torch.float16)
    plan = tp.Plan(ang, c["n"], c["n"] / 2 - 0.5, c["n"])
    tp.lamino_prepare(plan, c["tilt"], c["center_v"], c["slices"])
    return plan, filt, ang


def bench_lamino(args, log):
    """Laminographic backprojection of the slab workload: time per call (HIP
    events on the launch stream), updates/s, roofline; parity on two full
    slices against the FP64 oracle, which is timed on the host meanwhile."""
    import numpy as np
    import torch

    import oracle
    from paper_2209_08450_amd import tp

    dev = torch.device("cuda:0")
    c = LAMINO
    plan, filt, ang = lamino_setup(dev)
    out = torch.empty((c["slices"], c["n"], c["n"]), dtype=torch.float32, device=dev)

    def run():
        tp.lamino_backproject(plan, filt, c["tilt"], c["center_v"], c["slices"], out=out)

    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(max(args.steps, 2)):
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    updates = float(c["n"]) ** 2 * c["slices"] * c["angles"]
    achieved = LAMINO_FLOP_PER_UPDATE * updates / (ms * 1e-3) / 1e12
    log(f"[lamino] {ms:.1f} ms per call, {updates / (ms * 1e-3) / 1e12:.2f}e12 updates/s, "
        f"{achieved:.1f} TFLOP/s algorithmic")
    # parity at full detector and slab size from every 32nd angle (64 angles):
    # the whole slab on the GPU, 24 evenly spaced full slices (first and last
    # included) by the FP64 oracle, which is also the host baseline (timed on
    # the host's threads, about 10 s on 16)
    sub = slice(0, c["angles"], 32)
    n_sub = len(range(0, c["angles"], 32))
    plan_s = tp.Plan(ang[sub], c["n"], plan.center, c["n"])
    filt_s = filt[sub].contiguous()
    tp.lamino_backproject(plan_s, filt_s, c["tilt"], c["center_v"], c["slices"], out=out)
    zs = [int(z) for z in np.linspace(0, c["slices"] - 1, 24).round()]
    got = out[zs].cpu().numpy().astype(np.float64)
    q = filt_s.float().cpu().numpy().astype(np.float64)
    del filt_s
    iz, iy, ix = np.meshgrid(np.array(zs), np.arange(c["n"]), np.arange(c["n"]), indexing="ij")
    t0 = time.time()
    want = oracle.lamino_backproject_points(q, ang[sub], plan.center, c["center_v"], c["tilt"], c["n"],
                                            c["slices"], ix.ravel(), iy.ravel(), iz.ravel()).reshape(got.shape)
    cpu_t = time.time() - t0
    del q
    rel = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    mx = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    cpu_updates = float(got.size) * n_sub
    log(f"[lamino] rel-L2 vs FP64 oracle ({len(zs)} full slices, {n_sub} angles): {rel:.2e}, max {mx:.2e}; "
        f"oracle {cpu_updates / cpu_t / 1e6:.1f}e6 updates/s on {oracle.num_threads()} threads ({cpu_t:.1f} s)")
    plan_s.close()
    plan.close()
    return {
        "workload": f"{c['slices']} x {c['n']}^2 slab from {c['angles']} angles over 360 degrees of a "
                    f"{c['rows']} x {c['n']} detector, axis tilted {c['tilt']} rad from the beam, FP16 projections",
        "ms_per_call": round(ms, 3),
        "gups": round(updates / (ms * 1e-3) / 1e9, 1),
        "rel_l2_vs_fp64_oracle": rel,
        "max_err_over_max_ref": mx,
        "parity_sample": f"{len(zs)} evenly spaced slices in full ({len(zs)} x {c['n']}^2 voxels), the same slab "
                         f"from every 32nd angle ({n_sub} angles)",
        "cpu_oracle": {"value": round(cpu_updates / cpu_t / 1e9, 6), "unit": "Gvoxel-angle updates/s",
                       "cores": oracle.num_threads(), "kind": "oracle",
                       "sample": f"the parity sample: {int(cpu_updates):d} voxel-angle updates, {cpu_t:.1f} s"},
        "roofline": {"bound": "alu", "kernel": "k_lamino", "achieved": round(achieved, 2), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "flop_per_update": LAMINO_FLOP_PER_UPDATE, "traffic": load_lamino_traffic()},
    }


def main_single_lamino(args):
    """One laminographic backprojection of the slab workload, then a 1 GiB
    device copy (a short program for profiler and counter runs)."""
    import torch

    from paper_2209_08450_amd import tp

    dev = torch.device("cuda:0")
    c = LAMINO
    plan, filt, ang = lamino_setup(dev)
    out = torch.empty((c["slices"], c["n"], c["n"]), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    tp.lamino_backproject(plan, filt, c["tilt"], c["center_v"], c["slices"], out=out)
    torch.cuda.synchronize()
    del out, filt
    a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)  # calibration copy: 1 GiB read + 1 GiB written
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    log("single laminographic backprojection done")
    plan.close()


def main_single_fourier(args):
    """One tp_fourier_fbp_chunk of the timed chunk shape, then a 1 GiB device copy (counter calibration)."""
    import torch

    from paper_2209_08450_amd import synth, tp

    dev = torch.device("cuda:0")
    n, na, rows = args.n, args.angles, args.chunk
    scan = synth.ellipsoid_scan_torch(seed=2, n_angles=na, n_rows=rows, n_det=n, device=dev, center=n / 2.0)
    plan = tp.Plan(scan.angles, n, n / 2.0)
    hw = args.fourier_half_width or 6
    plan.fourier_prepare(args.filter, hw)
    ws = torch.empty(plan.fourier_workspace_bytes(rows), dtype=torch.uint8, device=dev)
    vol = torch.empty((rows, n, n), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    tp.fourier_fbp_chunk(plan, scan.proj, scan.dark, scan.flat, out=vol, workspace=ws, kind=args.filter,
                         half_width=hw)
    torch.cuda.synchronize()
    a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"single Fourier chunk {na} x {rows} x {n} done")
    plan.close()


def bench_ls(plan_cls, log, n_slices=128, n_vox=1024, n_angles=900, steps=30):
    """Forward projector R (tp_radon), its adjoint (tp_backproject, scale 1) and
    30 gradient least-squares steps on 128 slices of 1024^2 from 900 angles of
    noisy ellipsoid data; parity of R on one slice against the FP64 oracle and
    the oracle's R timed on the host."""
    import numpy as np
    import torch

    import oracle
    from paper_2209_08450_amd import autograd, synth, tp

    y, ang, c = synth.ls_problem_torch(seed=4, n_slices=n_slices, n_vox=n_vox, n_angles=n_angles, device="cuda")
    plan = plan_cls(ang, n_vox, c)
    g = torch.Generator(device="cuda").manual_seed(7)
    x = torch.rand((n_slices, n_vox, n_vox), generator=g, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    t_r = timed(lambda: tp.radon(plan, x))
    t_bp = timed(lambda: tp.backproject(plan, y, scale=1.0))
    upd = float(n_slices) * n_vox * n_vox * n_angles
    log(f"forward projector {t_r:.2f} ms, adjoint {t_bp:.2f} ms per call ({n_slices}x{n_vox}^2x{n_angles})")
    eta = autograd.step_size(plan)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, losses = autograd.ls_solve(plan, y, steps=steps, eta=eta)
    torch.cuda.synchronize()
    t_ls = time.perf_counter() - t0
    log(f"{steps} LS steps: {t_ls:.2f} s, loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    # parity of R on one slice, and the oracle's R on the host
    z = n_slices // 2
    xs = x[z:z + 1].cpu().numpy().astype(np.float64)
    got = tp.radon(plan, x[z:z + 1].contiguous()).cpu().numpy().astype(np.float64)
    t1 = time.perf_counter()
    want = oracle.radon(xs, ang, c, n_vox)
    t_cpu = time.perf_counter() - t1
    rel = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    achieved = FLOP_PER_UPDATE * upd / (t_r * 1e-3) / 1e12
    plan.close()
    return {
        "workload": f"{n_slices} slices x {n_vox}^2 from {n_angles} angles, noisy ellipsoid line integrals",
        "radon_ms": round(t_r, 3), "radon_gups": round(upd / t_r / 1e6, 1),
        "adjoint_ms": round(t_bp, 3), "adjoint_gups": round(upd / t_bp / 1e6, 1),
        "ls_steps": steps, "ls_s": round(t_ls, 3), "loss_first": losses[0], "loss_last": losses[-1],
        "loss_monotone": all(b <= a * (1 + 1e-6) for a, b in zip(losses, losses[1:])),
        "radon_rel_l2_vs_fp64_oracle_one_slice": rel,
        "radon_roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": PEAK_FP32_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4)},
        "radon_cpu_oracle": {"value": round(float(n_vox) * n_vox * n_angles / t_cpu / 1e9, 3), "unit": UNIT,
                             "cores": oracle.num_threads(), "sample": f"one slice, {t_cpu:.1f} s"},
    }


def main_single_launch(args):
    import torch

    from paper_2209_08450_amd import synth, tp

    st = args.storage.split(",")[0]
    n, na, rows = args.n, args.angles, args.chunk
    scan = synth.ellipsoid_scan_torch(seed=2, n_angles=na, n_rows=rows, n_det=n, device="cuda", center=n / 2.0)
    plan = tp.Plan(scan.angles, n, n / 2.0)
    vol = torch.empty((rows, n, n), dtype=torch.float32, device="cuda")
    ws = torch.empty(plan.fbp_workspace_bytes(rows, st), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    tp.fbp_chunk(plan, scan.proj, scan.dark, scan.flat, st, out=vol, workspace=ws, kind=args.filter)
    torch.cuda.synchronize()
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)  # 1 GiB read + 1 GiB written
    torch.cuda.synchronize()
    print(json.dumps({"single_launch": {"storage": st, "rows": rows, "n": n, "angles": na,
                                        "tuning": list(plan.get_tuning(st)), "copy_bytes": 1 << 30}}), flush=True)
    plan.close()


def main_single_radon(args):
    import torch

    from paper_2209_08450_amd import synth, tp

    y, ang, c = synth.ls_problem_torch(seed=4, n_slices=128, n_vox=1024, n_angles=900, device="cuda")
    plan = tp.Plan(ang, 1024, c)
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randn((128, 1024, 1024), generator=g, device="cuda")
    ws = torch.empty(max(256, plan.radon_workspace_bytes(128)), dtype=torch.uint8, device="cuda")
    out = torch.empty((128, 900, 1024), device="cuda")
    torch.cuda.synchronize()
    tp.radon(plan, x, out=out, workspace=ws)
    torch.cuda.synchronize()
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)  # 1 GiB read + 1 GiB written
    torch.cuda.synchronize()
    print(json.dumps({"single_radon": {"slices": 128, "n": 1024, "angles": 900, "copy_bytes": 1 << 30}}),
          flush=True)
    plan.close()


def cfg5_check_rows(chunks, rows: int, n_even: int = 10):
    """Slices the pipeline is checked on: the first and last row of the first
    three chunks and ``n_even`` evenly spaced rows."""
    zs = [z for z0, z1 in chunks[:3] for z in (z0, z1 - 1)]
    zs += [int((k + 0.5) * rows / n_even) for k in range(n_even)]
    return sorted(set(zs))


def pipeline_run(dev, n, na, rows, st, pattern, method, kind, io_dir, log, points=256, out_dtype="f32", buffers=3):
    """Host-pinned to host-pinned reconstruction through the three-stream
    pipeline (copy-in, compute, copy-out) over uneven chunks, with per-chunk
    graphs and the autotuned backprojection tiling; the same chunks are also
    timed with inputs resident on the device to show how much of the copy
    time the overlap hides.  Checked against the FP64 oracle at ``points``
    voxels of each check slice, and bitwise against the resident computation
    on the check slices of the first three chunks.  ``out_dtype`` 'f16': FP16
    slices (the 16-bit mode's output; half the copy-out and write bytes).
    Returns the record."""
    import concurrent.futures as cf

    import numpy as np
    import torch

    import oracle
    from paper_2209_08450_amd import pipeline, synth, tp, tune

    center = n / 2.0
    log(f"pipeline: generating {na} x {rows} x {n} scan on the GPU")
    scan = synth.ellipsoid_scan_torch(seed=5, n_angles=na, n_rows=rows, n_det=n, device=dev, center=center)
    torch.cuda.synchronize()
    plan = tp.Plan(scan.angles, n, center)
    fourier = method == "fourier"
    lprec = method == "lprec"
    if fourier:
        plan.fourier_prepare(kind, 0)
        k = a = None
    elif lprec:
        plan.lprec_prepare(kind)
        k = a = None
    else:
        k, a = tune.tune_backproject(plan, st, rows=16, use_cache=False)
        log(f"autotuned backprojection ({st}): slices {k}, angles {a}")
    chunks = pipeline.uneven_chunks(rows, pattern)
    updates = float(n) * n * na * rows
    check_z = cfg5_check_rows(chunks, rows)
    early_z = [z for z in check_z if z < chunks[min(2, len(chunks) - 1)][1]]

    def compute(z0, z1, out, ws):
        if fourier:
            tp.fourier_fbp_chunk(plan, scan.proj[:, z0:z1], scan.dark[:, z0:z1], scan.flat[:, z0:z1], out=out,
                                 workspace=ws, kind=kind, out_dtype=out_dtype)
        elif lprec:
            tp.lprec_fbp_chunk(plan, scan.proj[:, z0:z1], scan.dark[:, z0:z1], scan.flat[:, z0:z1], out=out,
                               workspace=ws, kind=kind)
        else:
            tp.fbp_chunk(plan, scan.proj[:, z0:z1], scan.dark[:, z0:z1], scan.flat[:, z0:z1], st, out=out,
                         workspace=ws, kind=kind, out_dtype=out_dtype)

    odt = torch.float16 if out_dtype == "f16" else torch.float32
    out_bytes = 2 if out_dtype == "f16" else 4
    # compute only, inputs resident on the device, same chunks
    vol_c = torch.empty((max(pattern), n, n), dtype=odt, device=dev)
    if fourier:
        ws_bytes = plan.fourier_workspace_bytes(max(pattern))
    elif lprec:
        ws_bytes = plan.lprec_workspace_bytes(max(pattern))
    else:
        ws_bytes = plan.fbp_workspace_bytes(max(pattern), st)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    resident = {}
    for z0, z1 in chunks[:3]:
        compute(z0, z1, vol_c[: z1 - z0], ws)
        for z in early_z:
            if z0 <= z < z1:
                resident[z] = vol_c[z - z0].cpu().numpy().copy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for z0, z1 in chunks:
        compute(z0, z1, vol_c[: z1 - z0], ws)
    torch.cuda.synchronize()
    t_compute = time.perf_counter() - t0
    log(f"compute only: {t_compute:.2f} s")
    del vol_c, ws

    # host copies of the raw data (pageable memory, as read from storage)
    log("copying the scan to host memory")
    proj_h = scan.proj.cpu().numpy()
    dark_h = scan.dark.cpu().numpy()
    flat_h = scan.flat.cpu().numpy()
    del scan
    torch.cuda.empty_cache()
    pool = cf.ThreadPoolExecutor(16)

    def source(z0, z1, p, d, f):
        pn, dn, fn = p.numpy(), d.numpy(), f.numpy()
        parts = np.array_split(np.arange(na), 16)
        list(pool.map(lambda idx: np.copyto(pn[idx[0]:idx[-1] + 1], proj_h[idx[0]:idx[-1] + 1, z0:z1]),
                      [q for q in parts if q.size]))
        np.copyto(dn, dark_h[:, z0:z1])
        np.copyto(fn, flat_h[:, z0:z1])

    kept = {}
    checksum = [0.0]

    def sink(z0, z1, vol):
        v = vol.numpy()
        checksum[0] += float(v[:, ::64, ::64].sum(dtype=np.float64))
        for z in check_z:
            if z0 <= z < z1:
                kept[z] = v[z - z0].copy()

    io = None
    if io_dir:
        # storage on both ends: the raw scan is written to files first (not
        # timed), then the pipeline reads row chunks from them and writes the
        # slices into one volume file with the native reader/writer threads
        os.makedirs(io_dir, exist_ok=True)
        paths = {k: os.path.join(io_dir, f"tp_bench_{k}.raw") for k in ("proj", "dark", "flat", "vol")}
        t1 = time.perf_counter()
        for name, arr in (("proj", proj_h), ("dark", dark_h), ("flat", flat_h)):
            tp.io_create(paths[name], arr.nbytes)
            tp.io_write_slices(paths[name], 0, arr.reshape(-1), arr.nbytes, threads=16)
            # on the drive and out of the page cache, so the pipeline's reads
            # come from the drive
            fd = os.open(paths[name], os.O_RDONLY)
            os.fsync(fd)
            os.posix_fadvise(fd, 0, 0, os.POSIX_FADV_DONTNEED)
            os.close(fd)
        log(f"scan written to {io_dir} in {time.perf_counter() - t1:.1f} s")
        source = pipeline.FileSource(paths["proj"], paths["dark"], paths["flat"], na, rows, n, dark_h.shape[0],
                                     flat_h.shape[0], threads=16)
        file_sink = pipeline.FileSink(paths["vol"], rows, n, threads=16, elem_bytes=out_bytes)

        def sink(z0, z1, vol):  # noqa: F811 (the file variant)
            file_sink(z0, z1, vol)
            v = vol.numpy()
            checksum[0] += float(v[:, ::64, ::64].sum(dtype=np.float64))

        io = paths

    pl = pipeline.ChunkPipeline(plan, max_rows=max(pattern), n_dark=dark_h.shape[0], n_flat=flat_h.shape[0],
                                storage=st, use_graphs=True, kind=kind, method=method, out_dtype=out_dtype,
                                buffers=buffers)
    pl.prepare(chunks)
    log(f"pipeline: {len(chunks)} chunks, {pl.stats.graphs_captured} graphs; running")
    t_run = time.perf_counter()
    stats = pl.run(chunks, source, sink)
    if io:
        file_sink.flush()  # the volume is on the drive before the clock stops
        stats.seconds = time.perf_counter() - t_run
    log(f"pipeline: {stats.seconds:.2f} s " + ("file to file" if io else "host to host"))
    if io:
        vol_file = np.memmap(io["vol"], dtype=np.float16 if out_dtype == "f16" else np.float32, mode="r",
                             shape=(rows, n, n))
        for z in check_z:
            kept[z] = np.array(vol_file[z])
        del vol_file
    bitwise = all(np.array_equal(kept[z], resident[z]) for z in early_z)
    rng = np.random.default_rng(0)
    # the Fourier-domain and log-polar methods are checked against the exact sum of
    # trigonometric interpolants, which sums L + 1 terms per voxel and angle
    npts = min(points, 64) if (fourier or lprec) else points
    per_slice, g_all, w_all = [], [], []
    log(f"oracle at {npts} voxels of each of {len(check_z)} slices")
    for z in check_z:
        ix, iy = rng.integers(0, n, npts), rng.integers(0, n, npts)
        ref = oracle.fourier_fbp_points if (fourier or lprec) else oracle.fbp_points
        want = ref(proj_h[:, z].view(np.uint16), dark_h[:, z].view(np.uint16), flat_h[:, z].view(np.uint16),
                   plan.angles, center, n, ix, iy, kind=kind)
        got = kept[z][iy, ix].astype(np.float64)
        per_slice.append({"z": z, "rel_l2": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
                          "max_abs_over_max_ref": float(np.max(np.abs(got - want)) / np.max(np.abs(want)))})
        g_all.append(got)
        w_all.append(want)
    g_all, w_all = np.concatenate(g_all), np.concatenate(w_all)
    h2d = (proj_h.nbytes + dark_h.nbytes + flat_h.nbytes) / 1e9
    d2h = rows * n * n * out_bytes / 1e9
    out = {
        "metric": "Gvoxel-angle updates/s host-pinned to host-pinned (three-stream pipeline, uneven chunks)",
        "value": round(updates / stats.seconds / 1e9, 2),
        "unit": UNIT,
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"fbp {n}x{n}x{rows} from {na} angles x {rows} rows x {n} cols 12-bit ellipsoid scan, "
                               f"{FILTER_NAMES[kind]}, "
                               + ("Fourier-domain backprojection" if fourier else
                                  "log-polar backprojection" if lprec else "linear-interpolation backprojection"),
                   "storage": None if (fourier or lprec) else st, "slices_out": out_dtype,
                   "chunks": list(pattern), "n_chunks": len(chunks), "buffers": buffers,
                   "graphs": stats.graphs_captured, "bp_tuning": None if (fourier or lprec) else [k, a]},
        "s_host_to_host" if not io else "s_file_to_file": round(stats.seconds, 3),
        "s_compute_only_resident": round(t_compute, 3),
        "compute_over_host_to_host": round(t_compute / stats.seconds, 3),
        "h2d_GB": round(h2d, 2), "d2h_GB": round(d2h, 2),
        "vs_fp64_oracle_sampled": {"points_per_slice": npts, "slices": check_z,
                                   "rel_l2": float(np.linalg.norm(g_all - w_all) / np.linalg.norm(w_all)),
                                   "max_abs_over_max_ref": float(np.max(np.abs(g_all - w_all)) / np.max(np.abs(w_all))),
                                   "per_slice": per_slice},
        "bitwise_equal_to_resident_compute": {"slices": early_z, "equal": bool(bitwise)},
        "checksum_strided": checksum[0],
    }
    if io:
        out["metric"] = "Gvoxel-angle updates/s file to file (storage reads, three-stream pipeline, storage writes)"
        out["storage"] = {"read_GB": round(h2d, 2), "write_GB": round(d2h, 2),
                          "read_write_GB_per_s": round((h2d + d2h) / stats.seconds, 2), "dir": io_dir}
        for path in io.values():
            os.remove(path)
    pool.shutdown()
    plan.close()
    return out


def main_pipeline(args):
    """The pipeline mode on its own (``--pipeline``): its record is the printed line."""
    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # defaults: 3000 angles x 4096 columns host to host; with --io-dir the 2048^3
    # scan (its files and the volume take ~52 GB of storage)
    # (the log-polar method: 2048^3 in 32-row chunks, its grid at 4096 columns
    # from 3000 angles exceeds the angle transform's length)
    lp = args.method == "lprec"
    n = args.n if (args.n != 2048 or args.io_dir or lp) else 4096
    na = args.angles if (args.angles != 2048 or args.io_dir or lp) else 3000
    st = args.storage.split(",")[0] if args.storage != "f16,f32,bf16" else "f16"
    pattern = tuple(int(v) for v in args.pattern.split(","))
    if lp and args.pattern == "32,64,128":
        pattern = (32,)
    out = pipeline_run(dev, n, na, args.rows, st, pattern, args.method, args.filter, args.io_dir, log,
                       out_dtype=args.out_dtype, buffers=args.buffers)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
