"""ctypes binding of libtp.so (C ABI in include/tp.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device buffers are torch tensors on the current HIP device; work is
enqueued on ``torch.cuda.current_stream()`` unless a stream is given.  A
negative status raises ``TpError`` with the library's message.  There is no
fallback: if libtp.so is missing this module fails to import.
"""
from __future__ import annotations

import ctypes
import math
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TP_LIBRARY", os.path.join(_HERE, "libtp.so"))

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libtp.so not found at {LIB_PATH}; build it with "
                      f"`python -c 'import __graft_entry__ as g; g.build()'`")

_lib = ctypes.CDLL(LIB_PATH)

TP_OK, TP_EINVAL, TP_EUNSUPPORTED, TP_EHIP, TP_ENOMEM = 0, -1, -2, -3, -4
TP_F32, TP_F16, TP_BF16 = 0, 1, 2
TP_RAMP, TP_SHEPP, TP_PARZEN = 0, 1, 2
FILTERS = {"ramp": TP_RAMP, "shepp": TP_SHEPP, "parzen": TP_PARZEN}

_c_i32, _c_i64, _c_sz, _c_vp, _c_f, _c_d = (ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t,
                                            ctypes.c_void_p, ctypes.c_float, ctypes.c_double)


class Geometry(ctypes.Structure):
    _fields_ = [("n_angles", ctypes.c_int32), ("n_det", ctypes.c_int32), ("n_vox", ctypes.c_int32),
                ("center", ctypes.c_double), ("angles", ctypes.POINTER(ctypes.c_double))]


def _proto(name, restype, *args):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(args)
    return f


_plan_create = _proto("tp_plan_create", _c_i32, ctypes.POINTER(Geometry), ctypes.POINTER(_c_vp))
_plan_destroy = _proto("tp_plan_destroy", _c_i32, _c_vp)
_plan_set_tuning = _proto("tp_plan_set_tuning", _c_i32, _c_vp, _c_i32, _c_i32, _c_i32)
_plan_get_tuning = _proto("tp_plan_get_tuning", _c_i32, _c_vp, _c_i32, ctypes.POINTER(_c_i32),
                          ctypes.POINTER(_c_i32))
_filter_prepare = _proto("tp_filter_prepare", _c_i32, _c_i32, _c_i32)
_prepare = _proto("tp_prepare", _c_i32, _c_vp, _c_i32, _c_i32)
_tune_load = _proto("tp_tune_load", _c_i32, ctypes.c_char_p)
_tune_lookup = _proto("tp_tune_lookup", _c_i32, ctypes.c_char_p, _c_i32, _c_i32, _c_i32, _c_i32,
                      ctypes.POINTER(_c_i32), ctypes.POINTER(_c_i32))
_shutdown = _proto("tp_shutdown", _c_i32)
_filter_response = _proto("tp_filter_response", _c_i32, _c_i32, _c_i32, ctypes.POINTER(_c_d))
_normalize_ws = _proto("tp_normalize_workspace_bytes", _c_sz, _c_i32, _c_i32)
_normalize = _proto("tp_normalize", _c_i32, _c_vp, _c_i64, _c_vp, _c_i32, _c_vp, _c_i32, _c_i64, _c_i32, _c_i32,
                    _c_i32, _c_i32, _c_vp, _c_vp, _c_sz, _c_vp)
_normalize_noalloc = _proto("tp_normalize_noalloc", _c_i32, _c_vp, _c_i64, _c_vp, _c_i32, _c_vp, _c_i32, _c_i64,
                            _c_i32, _c_i32, _c_i32, _c_i32, _c_vp, _c_vp)
_filter = _proto("tp_filter", _c_i32, _c_vp, _c_i32, _c_vp, _c_i32, _c_i64, _c_i32, _c_i32, _c_i32, _c_vp)
_backproject = _proto("tp_backproject", _c_i32, _c_vp, _c_vp, _c_i32, _c_i32, _c_f, _c_vp, _c_i32, _c_vp)
_radon = _proto("tp_radon", _c_i32, _c_vp, _c_vp, _c_i32, _c_vp, _c_vp, _c_sz, _c_vp)
_radon_ws = _proto("tp_radon_workspace_bytes", _c_sz, _c_vp, _c_i32)
_fbp_ws = _proto("tp_fbp_workspace_bytes", _c_sz, _c_vp, _c_i32, _c_i32)
_fbp_chunk = _proto("tp_fbp_chunk", _c_i32, _c_vp, _c_vp, _c_i64, _c_vp, _c_i32, _c_vp, _c_i32, _c_i64, _c_i32,
                    _c_i32, _c_i32, _c_vp, _c_sz, _c_vp, _c_vp)
_fbp_chunk_events = _proto("tp_fbp_chunk_events", _c_i32, _c_vp, _c_vp, _c_i64, _c_vp, _c_i32, _c_vp, _c_i32, _c_i64,
                           _c_i32, _c_i32, _c_i32, _c_vp, _c_sz, _c_vp, _c_vp, ctypes.POINTER(_c_vp))
_fbp_chunk_out = _proto("tp_fbp_chunk_out", _c_i32, _c_vp, _c_vp, _c_i64, _c_vp, _c_i32, _c_vp, _c_i32, _c_i64,
                        _c_i32, _c_i32, _c_i32, _c_vp, _c_sz, _c_i32, _c_vp, _c_vp, ctypes.POINTER(_c_vp))
_fourier_ws = _proto("tp_fourier_workspace_bytes", _c_sz, _c_vp, _c_i32)
_fourier_prepare = _proto("tp_fourier_prepare", _c_i32, _c_vp, _c_i32, _c_i32)
_fourier_chunk = _proto("tp_fourier_fbp_chunk", _c_i32, _c_vp, _c_vp, _c_i64, _c_vp, _c_i32, _c_vp, _c_i32, _c_i64,
                        _c_i32, _c_i32, _c_i32, _c_vp, _c_sz, _c_vp, _c_vp)
_fourier_chunk_events = _proto("tp_fourier_fbp_chunk_events", _c_i32, _c_vp, _c_vp, _c_i64, _c_vp, _c_i32, _c_vp,
                               _c_i32, _c_i64, _c_i32, _c_i32, _c_i32, _c_vp, _c_sz, _c_vp, _c_vp,
                               ctypes.POINTER(_c_vp))
_fourier_chunk_out = _proto("tp_fourier_fbp_chunk_out", _c_i32, _c_vp, _c_vp, _c_i64, _c_vp, _c_i32, _c_vp,
                            _c_i32, _c_i64, _c_i32, _c_i32, _c_i32, _c_vp, _c_sz, _c_i32, _c_vp, _c_vp,
                            ctypes.POINTER(_c_vp))


class LprecGrid(ctypes.Structure):
    """tp_lprec_grid: sizes and geometry of the log-polar grids."""
    _fields_ = [(k, ctypes.c_int32) for k in ("spans", "n_span", "Ns", "M", "NA", "D", "rows", "m_lo", "d_lo",
                                             "j_lo", "nj")] + \
               [(k, ctypes.c_double) for k in ("os", "eps", "dtheta", "R", "phi0", "a0", "s_min", "s_max", "delta",
                                              "sigma0", "dpsi")]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lprec_grid = _proto("tp_lprec_grid_query", _c_i32, _c_i32, _c_i32, _c_i32, _c_d, _c_d, ctypes.POINTER(LprecGrid))
_lprec_ws = _proto("tp_lprec_workspace_bytes", _c_sz, _c_vp, _c_i32, _c_i32, _c_d, _c_d)
_lprec_prepare = _proto("tp_lprec_prepare", _c_i32, _c_vp, _c_i32, _c_i32, _c_d, _c_d)
_lprec_chunk = _proto("tp_lprec_fbp_chunk", _c_i32, _c_vp, _c_vp, _c_i64, _c_vp, _c_i32, _c_vp, _c_i32, _c_i64,
                      _c_i32, _c_i32, _c_i32, _c_d, _c_d, _c_vp, _c_sz, _c_vp, _c_vp)
_lprec_chunk_events = _proto("tp_lprec_fbp_chunk_events", _c_i32, _c_vp, _c_vp, _c_i64, _c_vp, _c_i32, _c_vp,
                             _c_i32, _c_i64, _c_i32, _c_i32, _c_i32, _c_d, _c_d, _c_vp, _c_sz, _c_vp, _c_vp,
                             ctypes.POINTER(_c_vp))
_lamino_prepare = _proto("tp_lamino_prepare", _c_i32, _c_vp, _c_d, _c_d, _c_i32)
_lamino = _proto("tp_lamino_backproject", _c_i32, _c_vp, _c_vp, _c_i32, _c_i32, _c_d, _c_d, _c_i32, _c_i32, _c_i32,
                 _c_f, _c_vp, _c_vp)
_io_read_rows = _proto("tp_io_read_rows", _c_i32, ctypes.c_char_p, _c_i64, _c_i32, _c_i32, _c_i32, _c_i32, _c_i32,
                       _c_i32, _c_vp, _c_i32)
_io_write_slices = _proto("tp_io_write_slices", _c_i32, ctypes.c_char_p, _c_i64, _c_i64, _c_i32, _c_i64, _c_vp,
                          _c_i32)
_io_create = _proto("tp_io_create", _c_i32, ctypes.c_char_p, _c_i64)
_io_last_error = _proto("tp_io_last_error", ctypes.c_char_p)
_peak_copy = _proto("tp_peak_copy", _c_i32, _c_vp, _c_vp, _c_i64, _c_vp)
_peak_fma = _proto("tp_peak_fma", _c_i32, _c_vp, _c_i32, _c_i32, ctypes.POINTER(_c_i64), _c_vp)
_peak_valu = _proto("tp_peak_valu", _c_i32, _c_i32, _c_vp, _c_i32, _c_i32, ctypes.POINTER(_c_i64), _c_vp)
_peak_lds = _proto("tp_peak_lds", _c_i32, _c_vp, _c_i32, _c_i32, ctypes.POINTER(_c_i64), _c_vp)
_last_error = _proto("tp_last_error", ctypes.c_char_p)
_version = _proto("tp_version", ctypes.c_char_p)


class TpError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"tp status {status}: {message}")
        self.status = status


def last_error() -> str:
    return _last_error().decode()


def version() -> str:
    return _version().decode()


def _check(status: int):
    if status != TP_OK:
        raise TpError(status, last_error())


def raw_function(name: str):
    """The exported C function ``name`` (for ABI tests)."""
    return getattr(_lib, name)


# ---------------------------------------------------------------------------
# torch helpers (torch provides device memory and streams only)
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def dtype_code(dt) -> int:
    torch = _torch()
    if dt in (torch.float32, "f32", TP_F32):
        return TP_F32
    if dt in (torch.float16, "f16", TP_F16):
        return TP_F16
    if dt in (torch.bfloat16, "bf16", TP_BF16):
        return TP_BF16
    raise ValueError(f"unsupported storage dtype {dt!r}")


def torch_dtype(code: int):
    torch = _torch()
    return {TP_F32: torch.float32, TP_F16: torch.float16, TP_BF16: torch.bfloat16}[code]


def _stream_ptr(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _out(out, shape, dtype, like, name="out"):
    """A caller's output tensor checked against what the kernels will write
    (the C ABI receives a bare pointer), or a new one on ``like``'s device."""
    torch = _torch()
    shape = tuple(int(v) for v in shape)
    if out is None:
        return torch.empty(shape, dtype=dtype, device=like.device)
    if out.dtype != dtype or tuple(out.shape) != shape or not out.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {list(shape)}, "
                         f"got {out.dtype} {list(out.shape)}")
    if not out.is_cuda or out.device != like.device:
        raise ValueError(f"{name} must be on {like.device}")
    return out


def _raw_strides(t, name, n_det):
    """(pointer, outer stride) of a [outer][rows][n_det] uint16 view with packed rows."""
    torch = _torch()
    if t.dtype not in (torch.uint16, torch.int16):
        raise ValueError(f"{name} must be uint16 raw counts")
    if t.dim() != 3 or t.shape[2] != n_det or t.stride(2) != 1 or (t.shape[1] > 1 and t.stride(1) != n_det):
        raise ValueError(f"{name} must be [k][rows][n_det] with contiguous rows")
    return _dev(t, name), int(t.stride(0))


def _workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------------------
# Plans
# ---------------------------------------------------------------------------
class Plan:
    """Geometry tables on the current device (tp_plan_create)."""

    def __init__(self, angles, n_det: int, center: float, n_vox: int = 0):
        self.angles = np.ascontiguousarray(angles, dtype=np.float64)
        self.n_angles = int(self.angles.shape[0])
        self.n_det = int(n_det)
        self.n_vox = int(n_vox) if n_vox else int(n_det)
        self.center = float(center)
        g = Geometry(self.n_angles, self.n_det, int(n_vox), self.center,
                     self.angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        h = _c_vp()
        _check(_plan_create(ctypes.byref(g), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def set_tuning(self, storage, slices_per_block: int, angles_per_block: int):
        """Backprojection (slices per block, angles per block) for one storage type."""
        _check(_plan_set_tuning(self._h, dtype_code(storage), int(slices_per_block), int(angles_per_block)))

    def get_tuning(self, storage):
        k, a = _c_i32(), _c_i32()
        _check(_plan_get_tuning(self._h, dtype_code(storage), ctypes.byref(k), ctypes.byref(a)))
        return int(k.value), int(a.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(_plan_destroy(self._h))
            self._h = _c_vp()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():  # the HIP runtime may already be gone
            return
        try:
            self.close()
        except Exception:
            pass

    def fbp_workspace_bytes(self, n_rows: int, storage) -> int:
        return int(_fbp_ws(self._h, int(n_rows), dtype_code(storage)))

    def radon_workspace_bytes(self, n_rows: int) -> int:
        return int(_radon_ws(self._h, int(n_rows)))

    def fourier_workspace_bytes(self, n_rows: int) -> int:
        """Workspace for the Fourier-domain FBP of n_rows rows in one pass."""
        return int(_fourier_ws(self._h, int(n_rows)))

    def prepare(self, kind="ramp", storage="f16"):
        """Build what the hot calls need for (kind, storage) before graph capture (tp_prepare)."""
        _check(_prepare(self._h, filter_code(kind), dtype_code(storage)))

    def fourier_prepare(self, kind="ramp", half_width: int = 0):
        """Build the Fourier-domain path's tables (before graph capture)."""
        _check(_fourier_prepare(self._h, filter_code(kind), int(half_width)))

    def lprec_workspace_bytes(self, n_rows: int, spans: int = 0, os: float = 0.0, eps: float = 0.0) -> int:
        """Workspace for the log-polar FBP of n_rows rows in one pass (0: unsupported plan)."""
        return int(_lprec_ws(self._h, int(n_rows), int(spans), float(os), float(eps)))

    def lprec_prepare(self, kind="ramp", spans: int = 0, os: float = 0.0, eps: float = 0.0):
        """Build the log-polar path's tables (before graph capture)."""
        _check(_lprec_prepare(self._h, filter_code(kind), int(spans), float(os), float(eps)))


def tune_load(path) -> None:
    """Load the autotuner's JSON table of backprojection tilings (None clears it); plans
    created afterwards start from the recorded tilings of their device and shape."""
    _check(_tune_load(None if path is None else os.fsencode(path)))


def tune_lookup(device_name: str, storage, n_angles: int, n_det: int, n_vox: int = 0):
    """(slices_per_block, angles_per_block) the loaded table holds for a shape, or None."""
    k, a = _c_i32(), _c_i32()
    st = _tune_lookup(device_name.encode(), dtype_code(storage), int(n_angles), int(n_det), int(n_vox),
                      ctypes.byref(k), ctypes.byref(a))
    if st != TP_OK:
        return None
    return int(k.value), int(a.value)


def shutdown() -> None:
    """Free the library's cached filter tables on every device and clear the tuning
    table (every plan must have been closed)."""
    _check(_shutdown())


def filter_code(kind) -> int:
    """Filter window code from a name ('ramp', 'shepp', 'parzen') or a code."""
    if isinstance(kind, str):
        if kind not in FILTERS:
            raise ValueError(f"unknown filter {kind!r}; choose from {sorted(FILTERS)}")
        return FILTERS[kind]
    return int(kind)


def filter_prepare(pad_len: int, kind="ramp"):
    _check(_filter_prepare(int(pad_len), filter_code(kind)))


def filter_response(pad_len: int, kind="ramp") -> np.ndarray:
    """The library's FP64 filter response H[0..pad_len) (host only, no device)."""
    out = np.empty(int(pad_len), dtype=np.float64)
    _check(_filter_response(int(pad_len), filter_code(kind), out.ctypes.data_as(ctypes.POINTER(_c_d))))
    return out


def pad_len(n_det: int) -> int:
    return 1 << int(math.ceil(math.log2(2 * n_det)))


# ---------------------------------------------------------------------------
# Hot-path calls
# ---------------------------------------------------------------------------
def normalize(proj, dark, flat, out_dtype="f32", out=None, workspace=None, stream=None):
    """Raw uint16 [n_angles][rows][n_det] -> -log sinogram [rows][n_angles][n_det]."""
    torch = _torch()
    n_angles, n_rows, n_det = (int(s) for s in proj.shape)
    pp, ps = _raw_strides(proj, "proj", n_det)
    dp, fs = _raw_strides(dark, "dark", n_det)
    fp, fs2 = _raw_strides(flat, "flat", n_det)
    if fs != fs2:
        raise ValueError("dark and flat must share one frame stride")
    if dark.shape[1] != n_rows or flat.shape[1] != n_rows:
        raise ValueError("dark/flat rows must match proj rows")
    code = dtype_code(out_dtype)
    out = _out(out, (n_rows, n_angles, n_det), torch_dtype(code), proj)
    ws_need = int(_normalize_ws(n_rows, n_det))
    if workspace is None:
        workspace = _workspace(ws_need, proj.device)
    _check(_normalize(pp, ps, dp, int(dark.shape[0]), fp, int(flat.shape[0]), fs, n_angles, n_rows, n_det, code,
                      _dev(out, "out"), _dev(workspace, "workspace"), workspace.numel() * workspace.element_size(),
                      _stream_ptr(stream)))
    return out


NOALLOC_MAX_PIXELS = 1 << 23


def normalize_noalloc(proj, dark, flat, out, stream=None):
    """``normalize`` through the allocation-free entry point: the caller passes
    the output sinogram (``out``, [rows][n_angles][n_det] of F32/F16/BF16); the
    library's per-device scratch array holds the dark/flat tables, so the call
    allocates nothing.  Calls that overlap on one device race."""
    n_angles, n_rows, n_det = (int(s) for s in proj.shape)
    pp, ps = _raw_strides(proj, "proj", n_det)
    dp, fs = _raw_strides(dark, "dark", n_det)
    fp, fs2 = _raw_strides(flat, "flat", n_det)
    if fs != fs2:
        raise ValueError("dark and flat must share one frame stride")
    if dark.shape[1] != n_rows or flat.shape[1] != n_rows:
        raise ValueError("dark/flat rows must match proj rows")
    if out is None:
        raise ValueError("normalize_noalloc needs a caller-supplied output")
    code = dtype_code(out.dtype)
    _out(out, (n_rows, n_angles, n_det), torch_dtype(code), proj)
    _check(_normalize_noalloc(pp, ps, dp, int(dark.shape[0]), fp, int(flat.shape[0]), fs, n_angles, n_rows, n_det,
                              code, _dev(out, "out"), _stream_ptr(stream)))
    return out


def filter(sino, out_dtype=None, out=None, pad_len: int = 0, kind="ramp", stream=None):
    """Filter every row of ``sino`` [..., n_det] (ramp, or ramp with the Shepp-Logan
    or Parzen window); returns the filtered rows."""
    torch = _torch()
    if not sino.is_contiguous():
        raise ValueError("sino must be contiguous")
    in_code = dtype_code(sino.dtype)
    out_code = in_code if out_dtype is None else dtype_code(out_dtype)
    n_det = int(sino.shape[-1])
    n_lines = int(sino.numel() // n_det)
    out = _out(out, sino.shape, torch_dtype(out_code), sino)
    _check(_filter(_dev(sino, "sino"), in_code, _dev(out, "out"), out_code, n_lines, n_det, int(pad_len),
                   filter_code(kind), _stream_ptr(stream)))
    return out


def backproject(plan: Plan, filt, scale=None, out=None, accumulate: bool = False, stream=None):
    """Filtered rows [rows][n_angles][n_det] -> volume [rows][N][N] (float32)."""
    torch = _torch()
    if filt.dim() != 3 or tuple(filt.shape[1:]) != (plan.n_angles, plan.n_det) or not filt.is_contiguous():
        raise ValueError(f"filt must be contiguous [rows][{plan.n_angles}][{plan.n_det}]")
    n_rows = int(filt.shape[0])
    if scale is None:
        scale = math.pi / plan.n_angles
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs out")
        out = torch.empty((n_rows, plan.n_vox, plan.n_vox), dtype=torch.float32, device=filt.device)
    if out.dtype != torch.float32 or not out.is_contiguous() or tuple(out.shape) != (n_rows, plan.n_vox, plan.n_vox):
        raise ValueError("out must be contiguous float32 [rows][N][N]")
    _check(_backproject(plan.handle, _dev(filt, "filt"), dtype_code(filt.dtype), n_rows, float(scale),
                        _dev(out, "out"), 1 if accumulate else 0, _stream_ptr(stream)))
    return out


def radon(plan: Plan, vol, out=None, workspace=None, stream=None):
    """Volume [rows][N][N] float32 -> projections [rows][n_angles][n_det] float32.

    ``workspace``: optional device buffer of at least
    ``plan.radon_workspace_bytes(rows)`` bytes (allocated when omitted).
    """
    torch = _torch()
    if vol.dtype != torch.float32 or vol.dim() != 3 or tuple(vol.shape[1:]) != (plan.n_vox, plan.n_vox) \
            or not vol.is_contiguous():
        raise ValueError(f"vol must be contiguous float32 [rows][{plan.n_vox}][{plan.n_vox}]")
    n_rows = int(vol.shape[0])
    out = _out(out, (n_rows, plan.n_angles, plan.n_det), torch.float32, vol)
    need = plan.radon_workspace_bytes(n_rows)
    if workspace is None and need > 0:
        workspace = _workspace(need, vol.device)
    ws_ptr = _dev(workspace, "workspace") if workspace is not None else None
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(_radon(plan.handle, _dev(vol, "vol"), n_rows, _dev(out, "out"), ws_ptr, ws_bytes, _stream_ptr(stream)))
    return out


def fbp_chunk(plan: Plan, proj, dark, flat, storage="f32", out=None, workspace=None, stream=None, events=None,
              kind="ramp", out_dtype=None):
    """Raw counts of a row chunk -> reconstructed slices [rows][N][N].

    ``kind``: filter window, 'ramp', 'shepp' or 'parzen' (or its code).

    ``out_dtype``: 'f32' (default) or 'f16' (the 16-bit mode's FP16 slices,
    storage 'f16' only); ``out``, when given, must have that type.

    ``events``: optional list of four recorded-once ``torch.cuda.Event`` objects
    (or None entries) marked before the dark/flat means, the fused
    normalise+filter and the backprojection, and after it.
    """
    torch = _torch()
    n_angles, n_rows, n_det = (int(s) for s in proj.shape)
    if n_angles != plan.n_angles or n_det != plan.n_det:
        raise ValueError("proj does not match the plan geometry")
    pp, ps = _raw_strides(proj, "proj", n_det)
    dp, fs = _raw_strides(dark, "dark", n_det)
    fp, fs2 = _raw_strides(flat, "flat", n_det)
    if fs != fs2:
        raise ValueError("dark and flat must share one frame stride")
    if dark.shape[1] != n_rows or flat.shape[1] != n_rows:
        raise ValueError("dark/flat rows must match proj rows")
    code = dtype_code(storage)
    kcode = filter_code(kind)
    need = plan.fbp_workspace_bytes(n_rows, code)
    if workspace is None:
        workspace = _workspace(need, proj.device)
    vcode = dtype_code("f32" if out_dtype is None else out_dtype)
    tdt = torch.float16 if vcode == dtype_code("f16") else torch.float32
    out = _out(out, (n_rows, plan.n_vox, plan.n_vox), tdt, proj)
    arr = None
    if events is not None:
        if len(events) != 4:
            raise ValueError("events must hold four entries")
        arr = (_c_vp * 4)(*[_c_vp(e.cuda_event) if e is not None else _c_vp() for e in events])
        if any(e is not None and not e.cuda_event for e in events):
            raise ValueError("record each event once before passing it (torch creates it lazily)")
    _check(_fbp_chunk_out(plan.handle, pp, ps, dp, int(dark.shape[0]), fp, int(flat.shape[0]), fs, n_rows, kcode,
                          code, _dev(workspace, "workspace"), workspace.numel() * workspace.element_size(), vcode,
                          _dev(out, "out"), _stream_ptr(stream), arr))
    return out


def fourier_fbp_chunk(plan: Plan, proj, dark, flat, out=None, workspace=None, stream=None, events=None,
                      kind="ramp", half_width: int = 0, out_dtype="f32"):
    """Raw counts of a row chunk -> Fourier-domain FBP slices [rows][N][N]
    (float32, or float16 with ``out_dtype`` 'f16': each voxel's FP32 value
    rounded once; tp_fourier_fbp_chunk_out).

    Same inputs as ``fbp_chunk``; the backprojection uses the trigonometric
    interpolant of each padded filtered row, evaluated by gridding polar
    spectra onto a Cartesian frequency grid (tp_fourier_fbp_chunk).
    ``half_width``: Gaussian truncation radius in grid points (0 = 6).
    ``workspace``: default ``plan.fourier_workspace_bytes(rows)`` bytes (one
    pass); a smaller one runs the rows in several passes.
    ``events``: optional list of six recorded-once ``torch.cuda.Event``
    objects (or None entries), marked before the dark/flat means, the
    spectra, the gather, the two inverse-FFT passes, and after the first pass.
    """
    torch = _torch()
    n_angles, n_rows, n_det = (int(s) for s in proj.shape)
    if n_angles != plan.n_angles or n_det != plan.n_det:
        raise ValueError("proj does not match the plan geometry")
    pp, ps = _raw_strides(proj, "proj", n_det)
    dp, fs = _raw_strides(dark, "dark", n_det)
    fp, fs2 = _raw_strides(flat, "flat", n_det)
    if fs != fs2:
        raise ValueError("dark and flat must share one frame stride")
    if dark.shape[1] != n_rows or flat.shape[1] != n_rows:
        raise ValueError("dark/flat rows must match proj rows")
    kcode = filter_code(kind)
    if workspace is None:
        workspace = _workspace(plan.fourier_workspace_bytes(n_rows), proj.device)
    if out_dtype not in ("f32", "f16"):
        raise ValueError(f"out_dtype must be 'f32' or 'f16', not {out_dtype!r}")
    half = out_dtype == "f16"
    out = _out(out, (n_rows, plan.n_vox, plan.n_vox), torch.float16 if half else torch.float32, proj)
    args = (plan.handle, pp, ps, dp, int(dark.shape[0]), fp, int(flat.shape[0]), fs, n_rows, kcode, int(half_width),
            _dev(workspace, "workspace"), workspace.numel() * workspace.element_size(), _dev(out, "out"),
            _stream_ptr(stream))
    if half:
        if events is not None:
            raise ValueError("stage events are for FP32 slices")
        _check(_fourier_chunk_out(*args[:13], dtype_code("f16"), *args[13:], None))
    elif events is None:
        _check(_fourier_chunk(*args))
    else:
        if len(events) != 6:
            raise ValueError("events must hold six entries")
        if any(e is not None and not e.cuda_event for e in events):
            raise ValueError("record each event once before passing it (torch creates it lazily)")
        arr = (_c_vp * 6)(*[_c_vp(e.cuda_event) if e is not None else _c_vp() for e in events])
        _check(_fourier_chunk_events(*args, arr))
    return out


def lprec_grid(n_angles: int, n_vox: int, spans: int = 0, os: float = 0.0, eps: float = 0.0) -> dict:
    """The log-polar grid the library picks (host only, tp_lprec_grid_query)."""
    g = LprecGrid()
    _check(_lprec_grid(int(n_angles), int(n_vox), int(spans), float(os), float(eps), ctypes.byref(g)))
    return g.as_dict()


def lprec_fbp_chunk(plan: Plan, proj, dark, flat, out=None, workspace=None, stream=None, events=None,
                    kind="ramp", spans: int = 0, os: float = 0.0, eps: float = 0.0):
    """Raw counts of a row chunk -> log-polar FBP slices [rows][N][N] (float32)
    (tp_lprec_fbp_chunk).  Same inputs as ``fbp_chunk``; the plan's angles must
    be theta_0 + a pi / n_angles.  ``spans``, ``os``, ``eps``: span count,
    grid oversampling and origin margin (0: 3, 1.0, 1.0).  ``workspace``:
    default ``plan.lprec_workspace_bytes(rows, ...)`` (one pass).  ``events``:
    optional list of seven recorded-once ``torch.cuda.Event`` objects (or
    None entries) marking the stages of the first pass."""
    torch = _torch()
    n_angles, n_rows, n_det = (int(s) for s in proj.shape)
    if n_angles != plan.n_angles or n_det != plan.n_det:
        raise ValueError("proj does not match the plan geometry")
    pp, ps = _raw_strides(proj, "proj", n_det)
    dp, fs = _raw_strides(dark, "dark", n_det)
    fp, fs2 = _raw_strides(flat, "flat", n_det)
    if fs != fs2:
        raise ValueError("dark and flat must share one frame stride")
    if dark.shape[1] != n_rows or flat.shape[1] != n_rows:
        raise ValueError("dark/flat rows must match proj rows")
    kcode = filter_code(kind)
    if workspace is None:
        need = plan.lprec_workspace_bytes(n_rows, spans, os, eps)
        if need == 0:
            _check(_lprec_prepare(plan.handle, kcode, int(spans), float(os), float(eps)))
        workspace = _workspace(need, proj.device)
    out = _out(out, (n_rows, plan.n_vox, plan.n_vox), torch.float32, proj)
    args = (plan.handle, pp, ps, dp, int(dark.shape[0]), fp, int(flat.shape[0]), fs, n_rows, kcode, int(spans),
            float(os), float(eps), _dev(workspace, "workspace"), workspace.numel() * workspace.element_size(),
            _dev(out, "out"), _stream_ptr(stream))
    if events is None:
        _check(_lprec_chunk(*args))
    else:
        if len(events) != 7:
            raise ValueError("events must hold seven entries")
        if any(e is not None and not e.cuda_event for e in events):
            raise ValueError("record each event once before passing it (torch creates it lazily)")
        arr = (_c_vp * 7)(*[_c_vp(e.cuda_event) if e is not None else _c_vp() for e in events])
        _check(_lprec_chunk_events(*args, arr))
    return out


# ---------------------------------------------------------------------------
# Laminography
# ---------------------------------------------------------------------------
def lamino_prepare(plan: Plan, tilt: float, center_v: float, n_slices: int):
    """Build the laminographic tables for (tilt, center_v, n_slices) (tp_lamino_prepare)."""
    _check(_lamino_prepare(plan.handle, float(tilt), float(center_v), int(n_slices)))


def lamino_backproject(plan: Plan, filt, tilt: float, center_v: float, n_slices: int, z0: int = 0, nz=None,
                       scale=None, out=None, stream=None):
    """Laminographic backprojection of filtered projections filt [n_angles][det_rows][n_det]
    (device, float32 / float16 / bfloat16) into slices z0 .. z0+nz-1 of an n_slices-slice
    volume: out [nz][N][N] float32 (tp_lamino_backproject).  tilt: angle of the rotation
    axis to the beam in (0, pi), pi/2 = tomography; scale defaults to pi / n_angles."""
    torch = _torch()
    if filt.dim() != 3 or filt.shape[0] != plan.n_angles or filt.shape[2] != plan.n_det or not filt.is_contiguous():
        raise ValueError("filt must be a contiguous [n_angles][det_rows][n_det] device tensor")
    nz = int(n_slices) - int(z0) if nz is None else int(nz)
    out = _out(out, (nz, plan.n_vox, plan.n_vox), torch.float32, filt)
    scale = math.pi / plan.n_angles if scale is None else float(scale)
    _check(_lamino(plan.handle, _dev(filt, "filt"), dtype_code(filt.dtype), int(filt.shape[1]), float(tilt),
                   float(center_v), int(n_slices), int(z0), nz, scale, _dev(out, "out"), _stream_ptr(stream)))
    return out


# ---------------------------------------------------------------------------
# Storage reads and writes (host buffers: numpy arrays or CPU tensors)
# ---------------------------------------------------------------------------
def _host_ptr(buf, writable: bool):
    if isinstance(buf, np.ndarray):
        if not buf.flags.c_contiguous or (writable and not buf.flags.writeable):
            raise ValueError("host buffer must be C-contiguous" + (" and writable" if writable else ""))
        return ctypes.c_void_p(buf.ctypes.data), buf.nbytes
    if getattr(buf, "is_cuda", False):
        raise ValueError("storage calls take host buffers")
    if not buf.is_contiguous():
        raise ValueError("host buffer must be contiguous")
    return ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()


def _io_check(status: int):
    if status != TP_OK:
        raise TpError(status, _io_last_error().decode())


def io_read_rows(path, n_outer: int, n_rows: int, n_det: int, z0: int, z1: int, dst, threads: int = 8,
                 header_bytes: int = 0, elem_bytes: int = 2):
    """Rows [z0, z1) of a projection-major file [n_outer][n_rows][n_det] into
    dst [n_outer][z1 - z0][n_det] (tp_io_read_rows)."""
    ptr, nbytes = _host_ptr(dst, True)
    if nbytes < n_outer * (z1 - z0) * n_det * elem_bytes:
        raise ValueError("destination buffer too small")
    _io_check(_io_read_rows(os.fsencode(str(path)), int(header_bytes), int(n_outer), int(n_rows), int(n_det), int(z0),
                            int(z1), int(elem_bytes), ptr, int(threads)))
    return dst


def io_write_slices(path, first_slice: int, src, slice_bytes: int, threads: int = 8, header_bytes: int = 0):
    """Slices src [n][...] (n * slice_bytes bytes) at slice first_slice of the file (tp_io_write_slices)."""
    ptr, nbytes = _host_ptr(src, False)
    if nbytes % slice_bytes:
        raise ValueError("source is not a whole number of slices")
    _io_check(_io_write_slices(os.fsencode(str(path)), int(header_bytes), int(first_slice), nbytes // slice_bytes,
                               int(slice_bytes), ptr, int(threads)))


def io_create(path, nbytes: int):
    """Create (or truncate) a file of nbytes bytes (tp_io_create)."""
    _io_check(_io_create(os.fsencode(str(path)), int(nbytes)))


# ---------------------------------------------------------------------------
# Measurement instruments (roofline denominators)
# ---------------------------------------------------------------------------
def peak_copy(src, dst, stream=None):
    """Enqueue a device copy of src into dst (same byte size, a multiple of 16)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst must have the same size in bytes")
    _check(_peak_copy(_dev(src, "src"), _dev(dst, "dst"), nbytes, _stream_ptr(stream)))
    return nbytes


def peak_fma(out, iters: int, stream=None) -> int:
    """Enqueue the FMA-chain kernel over out.numel() // 256 work-groups; returns its flop count."""
    blocks = out.numel() // 256
    flop = _c_i64()
    _check(_peak_fma(_dev(out, "out"), int(blocks), int(iters), ctypes.byref(flop), _stream_ptr(stream)))
    return int(flop.value)


VALU_FORMS = {"fma_f32": 0, "fma_f32_sgpr": 1, "fma_mix_f16": 2, "dot2_f16": 3}


def peak_valu(form: str, out, iters: int, stream=None) -> int:
    """Enqueue the multiply-add chain kernel of one instruction form (``VALU_FORMS``) over
    out.numel() // 256 work-groups (float32 out); returns its flop count."""
    blocks = out.numel() // 256
    flop = _c_i64()
    _check(_peak_valu(VALU_FORMS[form], _dev(out, "out"), int(blocks), int(iters), ctypes.byref(flop),
                      _stream_ptr(stream)))
    return int(flop.value)


def peak_lds(out, iters: int, stream=None) -> int:
    """Enqueue the LDS read kernel (32-bit out, out.numel() // 256 work-groups); returns the bytes read."""
    blocks = out.numel() // 256
    nbytes = _c_i64()
    _check(_peak_lds(_dev(out, "out"), int(blocks), int(iters), ctypes.byref(nbytes), _stream_ptr(stream)))
    return int(nbytes.value)
