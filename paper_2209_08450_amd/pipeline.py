"""Asynchronous chunk pipeline (paper Section 2.3).

Chunks of detector rows (uneven sizes allowed) flow host -> device -> host
through three HIP streams: copy-in, compute, copy-out.  B pinned host
buffers and B device buffers on each side (B = 2 is the paper's double
buffering) let the copy-in of chunk k+1 and the copy-out of chunk k-1 overlap
the reconstruction of chunk k; instead of a full synchronisation after every
chunk, events order exactly the hazards that exist (chunk k uses buffer k%B):

  copy-in(k)   waits compute(k-B)   (device input buffer free)
  compute(k)   waits copy-in(k) and copy-out(k-B) (device output buffer free)
  copy-out(k)  waits compute(k) and the sink's release of chunk k-B's pinned
               output buffer
  host fill(k) waits copy-in(k-B)   (pinned input buffer free)

With uneven chunks a third buffer pays: after a large chunk, the next two
small ones would otherwise wait for its copy-out (and the host fill of the
chunk after them behind it), leaving the GPU idle.

Each chunk's three kernels (dark/flat means, fused normalise + filter,
backprojection) are captured once per (chunk size, buffer) as a HIP graph and
replayed.  A producer callback fills the pinned input views on the host; a
sink callback consumes each finished pinned output view on a worker thread.
Slices are independent, so results are bitwise equal to one monolithic
tp_fbp_chunk call over all rows.
"""
from __future__ import annotations

import os
import queue
import threading
from dataclasses import dataclass

import torch

from . import tp


def uneven_chunks(n_rows: int, pattern=(32, 64, 128), start_row: int = 0):
    """[(z0, z1), ...] covering [start_row, n_rows) with sizes cycling through
    ``pattern``; the last chunk is truncated.  Every row is covered once."""
    out, z, i = [], int(start_row), 0
    while z < n_rows:
        c = int(pattern[i % len(pattern)])
        if c <= 0:
            raise ValueError("chunk sizes must be positive")
        out.append((z, min(n_rows, z + c)))
        z += c
        i += 1
    return out


class FileSource:
    """Pipeline source that reads each chunk's rows from raw projection-major
    files (uint16 [n_angles][n_rows][n_det], dark and flat [frames][n_rows][n_det])
    straight into the pipeline's pinned buffers with tp_io_read_rows: the
    storage side of the paper's Section 2.3 pipeline, in native threads."""

    def __init__(self, proj_path, dark_path, flat_path, n_angles: int, n_rows: int, n_det: int, n_dark: int,
                 n_flat: int, threads: int = 16):
        self.paths = (str(proj_path), str(dark_path), str(flat_path))
        self.shape = (int(n_angles), int(n_rows), int(n_det), int(n_dark), int(n_flat))
        self.threads = int(threads)

    def __call__(self, z0, z1, p, d, f):
        na, nr, n, nd, nf = self.shape
        tp.io_read_rows(self.paths[0], na, nr, n, z0, z1, p, threads=self.threads)
        tp.io_read_rows(self.paths[1], nd, nr, n, z0, z1, d, threads=self.threads)
        tp.io_read_rows(self.paths[2], nf, nr, n, z0, z1, f, threads=self.threads)


class FileSink:
    """Pipeline sink that writes each chunk's slices ([rows][N][N], float32 or,
    with ``elem_bytes=2``, FP16) into one raw volume file with
    tp_io_write_slices; the file is created at its full size first."""

    def __init__(self, path, n_rows: int, n_vox: int, threads: int = 16, elem_bytes: int = 4):
        self.path = str(path)
        if elem_bytes not in (2, 4):
            raise ValueError("elem_bytes must be 2 (FP16 slices) or 4 (float32)")
        self.slice_bytes = int(n_vox) * int(n_vox) * int(elem_bytes)
        self.threads = int(threads)
        tp.io_create(self.path, int(n_rows) * self.slice_bytes)

    def __call__(self, z0, z1, vol):
        tp.io_write_slices(self.path, z0, vol, self.slice_bytes, threads=self.threads)

    def flush(self):
        """Force the written slices out to the drive (fsync)."""
        fd = os.open(self.path, os.O_RDONLY)
        try:
            os.fsync(fd)
        finally:
            os.close(fd)


@dataclass
class PipelineStats:
    chunks: int = 0
    rows: int = 0
    graphs_captured: int = 0
    graph_replays: int = 0
    seconds: float = 0.0


class ChunkPipeline:
    """Three-stream, multi-buffered FBP over row chunks.

    plan: tp.Plan of the scan geometry; max_rows: largest chunk; n_dark/n_flat:
    frames per chunk; storage: 'f16' / 'f32' / 'bf16' for the filtered rows;
    kind: filter window ('ramp', 'shepp', 'parzen'); use_graphs: capture each (size, buffer) once and replay it; poison: fill
    device and pinned buffers with NaN before each use (a missing dependency
    then shows as NaN in the result).  method: 'linear' (tp_fbp_chunk),
    'fourier' (tp_fourier_fbp_chunk; storage is then unused and half_width
    sets its Gaussian's truncation radius) or 'lprec' (tp_lprec_fbp_chunk,
    equally spaced angles; lprec = (spans, oversampling, origin margin), zeros
    for the defaults; one pass per chunk).  The Fourier-domain and log-polar
    methods carry two slices as one complex sequence: chunks of even sizes keep
    the pairs of one monolithic call.  buffers: pinned and device buffers
    per direction (each holds one chunk of max_rows; 2 is the paper's double
    buffering, the default 3 keeps the GPU busy behind uneven chunks).
    """

    def __init__(self, plan: "tp.Plan", max_rows: int, n_dark: int, n_flat: int, storage="f16",
                 use_graphs: bool = True, poison: bool = False, device=None, kind="ramp", method="linear",
                 half_width: int = 0, out_dtype="f32", buffers: int = 3, lprec=(0, 0.0, 0.0)):
        self.plan = plan
        if int(buffers) < 2:
            raise ValueError(f"buffers must be at least 2, not {buffers}")
        self.nbuf = nb = int(buffers)
        self.kind = kind
        tp.filter_code(kind)  # reject unknown names early
        if method not in ("linear", "fourier", "lprec"):
            raise ValueError(f"method must be 'linear', 'fourier' or 'lprec', not {method!r}")
        self.method = method
        self.half_width = int(half_width)
        spans, lp_os, lp_eps = lprec
        self.lprec = (int(spans), float(lp_os), float(lp_eps))
        if out_dtype not in ("f32", "f16"):
            raise ValueError(f"out_dtype must be 'f32' or 'f16', not {out_dtype!r}")
        if out_dtype == "f16" and (method == "lprec" or (method == "linear" and storage != "f16")):
            raise ValueError("FP16 slices come from the linear method with FP16 storage (the 16-bit mode) "
                             "or from the Fourier-domain method")
        self.out_dtype = out_dtype
        odt = torch.float16 if out_dtype == "f16" else torch.float32
        if method == "fourier":
            plan.fourier_prepare(kind, self.half_width)  # tables before any capture
        elif method == "lprec":
            plan.lprec_prepare(kind, *self.lprec)
        self.device = torch.device(device or f"cuda:{torch.cuda.current_device()}")
        self.max_rows = int(max_rows)
        self.n_dark, self.n_flat = int(n_dark), int(n_flat)
        self.storage = storage
        self.use_graphs = use_graphs
        self.poison = poison
        na, n, N = plan.n_angles, plan.n_det, plan.n_vox
        r = self.max_rows
        i16 = torch.int16

        def pinned(numel, dtype):
            return torch.empty(numel, dtype=dtype, pin_memory=True)

        def dev(numel, dtype):
            return torch.empty(numel, dtype=dtype, device=self.device)

        self.pin_in = [pinned(na * r * n, i16) for _ in range(nb)]
        self.pin_dark = [pinned(self.n_dark * r * n, i16) for _ in range(nb)]
        self.pin_flat = [pinned(self.n_flat * r * n, i16) for _ in range(nb)]
        self.pin_out = [pinned(r * N * N, odt) for _ in range(nb)]
        self.dev_in = [dev(na * r * n, i16) for _ in range(nb)]
        self.dev_dark = [dev(self.n_dark * r * n, i16) for _ in range(nb)]
        self.dev_flat = [dev(self.n_flat * r * n, i16) for _ in range(nb)]
        self.dev_out = [dev(r * N * N, odt) for _ in range(nb)]
        if method == "fourier":
            ws_bytes = plan.fourier_workspace_bytes(r)
        elif method == "lprec":
            ws_bytes = plan.lprec_workspace_bytes(r, *self.lprec)
            if ws_bytes == 0:
                raise ValueError("the log-polar method needs equally spaced angles theta_0 + a pi / n_angles")
        else:
            ws_bytes = plan.fbp_workspace_bytes(r, storage)
        self.ws = dev(max(256, ws_bytes), torch.uint8)
        # streams at default priority
        self.s_h2d = torch.cuda.Stream(device=self.device)
        self.s_comp = torch.cuda.Stream(device=self.device)
        self.s_d2h = torch.cuda.Stream(device=self.device)
        self._graphs = {}
        self.stats = PipelineStats()

    # -- views of the flat buffers for a chunk of c rows (contiguous) --
    def _views(self, b, c):
        na, n, N = self.plan.n_angles, self.plan.n_det, self.plan.n_vox
        return dict(
            pin_in=self.pin_in[b][: na * c * n].view(na, c, n),
            pin_dark=self.pin_dark[b][: self.n_dark * c * n].view(self.n_dark, c, n),
            pin_flat=self.pin_flat[b][: self.n_flat * c * n].view(self.n_flat, c, n),
            pin_out=self.pin_out[b][: c * N * N].view(c, N, N),
            dev_in=self.dev_in[b][: na * c * n].view(na, c, n),
            dev_dark=self.dev_dark[b][: self.n_dark * c * n].view(self.n_dark, c, n),
            dev_flat=self.dev_flat[b][: self.n_flat * c * n].view(self.n_flat, c, n),
            dev_out=self.dev_out[b][: c * N * N].view(c, N, N),
        )

    def _compute(self, v):
        if self.method == "fourier":
            tp.fourier_fbp_chunk(self.plan, v["dev_in"], v["dev_dark"], v["dev_flat"], out=v["dev_out"],
                                 workspace=self.ws, kind=self.kind, half_width=self.half_width,
                                 out_dtype=self.out_dtype)
        elif self.method == "lprec":
            spans, lp_os, lp_eps = self.lprec
            tp.lprec_fbp_chunk(self.plan, v["dev_in"], v["dev_dark"], v["dev_flat"], out=v["dev_out"],
                               workspace=self.ws, kind=self.kind, spans=spans, os=lp_os, eps=lp_eps)
        else:
            tp.fbp_chunk(self.plan, v["dev_in"], v["dev_dark"], v["dev_flat"], self.storage, out=v["dev_out"],
                         workspace=self.ws, kind=self.kind, out_dtype=self.out_dtype)

    def prepare(self, chunks):
        """Capture the graphs of every (chunk size, buffer) the run will use.

        Each is run once eagerly first (on whatever the buffers hold), so that
        one-time setup such as kernel attributes happens outside the capture.
        """
        if not self.use_graphs:
            return
        for b, c in sorted({(k % self.nbuf, z1 - z0) for k, (z0, z1) in enumerate(chunks)}):
            if (b, c) in self._graphs:
                continue
            v = self._views(b, c)
            with torch.cuda.stream(self.s_comp):
                self._compute(v)
            self.s_comp.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=self.s_comp, capture_error_mode="thread_local"):
                self._compute(v)
            self._graphs[(b, c)] = g
            self.stats.graphs_captured += 1

    def run(self, chunks, source, sink):
        """Reconstruct ``chunks`` [(z0, z1), ...].

        source(z0, z1, proj, dark, flat): fill the pinned uint16 views
            proj [n_angles][c][n_det], dark [n_dark][c][n_det], flat [n_flat][c][n_det]
            (int16 tensors holding uint16 bit patterns) with rows z0..z1.
        sink(z0, z1, vol): consume the pinned view vol [c][N][N] (float32, or FP16
            with out_dtype 'f16'); it is
            reused for a later chunk once sink returns.
        """
        import time

        for z0, z1 in chunks:
            if not 0 < z1 - z0 <= self.max_rows:
                raise ValueError(f"chunk ({z0}, {z1}) exceeds max_rows={self.max_rows}")
        self.prepare(chunks)
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        ev = lambda: torch.cuda.Event()  # noqa: E731
        nb = self.nbuf
        h2d_done = [None] * nb
        comp_done = [None] * nb
        d2h_done = [None] * nb
        out_free = [threading.Event() for _ in range(nb)]
        for e in out_free:
            e.set()
        work = queue.Queue()
        errors = []

        def sink_worker():
            while True:
                item = work.get()
                if item is None:
                    return
                b, z0, z1, done_ev, view = item
                try:
                    done_ev.synchronize()
                    sink(z0, z1, view)
                except Exception as exc:  # report after the loop drains
                    errors.append((z0, z1, exc))
                finally:
                    out_free[b].set()

        worker = threading.Thread(target=sink_worker, daemon=True)
        worker.start()
        try:
            for k, (z0, z1) in enumerate(chunks):
                if errors:
                    break
                b, c = k % nb, z1 - z0
                v = self._views(b, c)
                # host fill of pinned input b: its previous copy-in must be done
                if h2d_done[b] is not None:
                    h2d_done[b].synchronize()
                if self.poison:
                    v["pin_in"].fill_(-1)
                try:
                    source(z0, z1, v["pin_in"], v["pin_dark"], v["pin_flat"])
                except Exception as exc:
                    raise RuntimeError(f"source failed on chunk {k} (rows [{z0}, {z1}))") from exc
                # copy-in
                if comp_done[b] is not None:
                    self.s_h2d.wait_event(comp_done[b])
                with torch.cuda.stream(self.s_h2d):
                    if self.poison:
                        v["dev_in"].fill_(-1)
                    v["dev_in"].copy_(v["pin_in"], non_blocking=True)
                    v["dev_dark"].copy_(v["pin_dark"], non_blocking=True)
                    v["dev_flat"].copy_(v["pin_flat"], non_blocking=True)
                    h2d_done[b] = ev()
                    h2d_done[b].record(self.s_h2d)
                # compute
                self.s_comp.wait_event(h2d_done[b])
                if d2h_done[b] is not None:
                    self.s_comp.wait_event(d2h_done[b])
                if self.use_graphs:
                    g = self._graphs[(b, c)]
                    if self.poison:
                        with torch.cuda.stream(self.s_comp):
                            v["dev_out"].fill_(float("nan"))
                    with torch.cuda.stream(self.s_comp):
                        g.replay()
                    self.stats.graph_replays += 1
                else:
                    with torch.cuda.stream(self.s_comp):
                        if self.poison:
                            v["dev_out"].fill_(float("nan"))
                        self._compute(v)
                comp_done[b] = ev()
                comp_done[b].record(self.s_comp)
                # copy-out, once the sink has released pinned output b
                out_free[b].wait()
                out_free[b].clear()
                self.s_d2h.wait_event(comp_done[b])
                with torch.cuda.stream(self.s_d2h):
                    if self.poison:
                        v["pin_out"].fill_(float("nan"))  # host op: ordered by out_free
                    v["pin_out"].copy_(v["dev_out"], non_blocking=True)
                    d2h_done[b] = ev()
                    d2h_done[b].record(self.s_d2h)
                work.put((b, z0, z1, d2h_done[b], v["pin_out"]))
                self.stats.chunks += 1
                self.stats.rows += c
        finally:
            work.put(None)
            worker.join()
            torch.cuda.synchronize(self.device)
        self.stats.seconds = time.perf_counter() - t0
        if errors:
            z0, z1, exc = errors[0]
            raise RuntimeError(f"sink failed on chunk rows [{z0}, {z1})") from exc
        return self.stats
