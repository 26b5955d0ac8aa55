"""MI355X-native filtered backprojection for parallel-beam tomography.

The hot path of arXiv 2209.08450 (TomocuPy): dark/flat correction and -log,
ramp filtering of detector rows by FFT, and direct backprojection with linear
interpolation ("LineRec"), plus its exact transpose (forward projection) for
gradient-based least squares.  Every step runs in hand-written HIP kernels for
gfx950 behind the C ABI declared in ``include/tp.h`` (library ``libtp.so``);
this package is the thin ctypes binding over it (``tp``), a torch autograd
wrapper (``autograd``), the three-stream chunk pipeline (``pipeline``) and the
tile autotuner (``tune``).  ``synth`` holds the seeded synthetic inputs.

Submodules are imported lazily so that ``synth`` works without the HIP library.
"""
import importlib

__all__ = ["tp", "synth", "autograd", "pipeline", "tune"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
