"""FP64 CPU oracle for the filtered-backprojection hot path (TEST INFRASTRUCTURE).

This package is a plain, slow, obviously-correct reference.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
it.  The product library (``paper_2209_08450_amd``) never imports, links or
calls anything here, and nothing here imports the product library: the two
share no code, tables or constants.  Inputs reach both sides only through the
seeded generators in ``paper_2209_08450_amd.synth``, which contain none of the
method's arithmetic.

Functions follow the paper (arXiv 2209.08450):

* ``dark_flat_mean`` / ``normalize``  -- dark/flat-field correction and the
  negative logarithm (Section 2.2, pre-processing list).
* ``pad_len`` / ``ramp_kernel`` / ``ramp_response`` / ``filter_rows`` /
  ``filter_rows_direct`` -- padded one-dimensional filtering of detector rows
  by FFT (Section 2.2; padding discussion in Section 3).
* ``filter_window`` / ``filter_kernel`` / ``filter_response`` -- the
  Shepp-Logan and Parzen windows on the ramp (the filter choices of the
  command-line interface, Section 2.4; Parzen for every result of Section 3).
* ``backproject`` / ``backproject_points`` -- direct discretisation of the
  backprojection line integral with linear interpolation ("LineRec",
  Sections 2.2 and 3).
* ``radon`` -- its exact transpose (forward projector; the paper names
  iterative methods as the use of such a pair in Sections 1 and 5).
* ``fbp`` -- the composition, with optional FP16/BF16 rounding of stored
  filtered rows (Section 2.1 on 16-bit storage).
* ``fourier_backproject`` / ``fourier_fbp`` -- the Fourier-domain
  backprojection ("FourierRec", Sections 2.2 and 3): each padded filtered row
  evaluated along the ray by its trigonometric interpolant, summed directly.
* ``lamino_backproject`` -- the direct backprojector in laminographic
  geometry (tilted rotation axis, bilinear interpolation; Section 2.2 names
  this use of the direct method).
* ``power_lambda_max`` / ``ls_solve`` -- gradient least squares with the pair.
* ``lprec.lprec_backproject`` / ``lprec.lprec_fbp`` -- the log-polar-based
  backprojection ("LpRec", Sections 2.2 and 3): per span of angles, a
  convolution in log-polar coordinates by FFTs between B-spline
  interpolations to and from the log-polar grid (module ``oracle.lprec``).

Parity status: every function here is pinned by closed forms, invariants or
brute force in ``tests/test_oracle_*.py`` except where noted in a function's
docstring.
"""
from .fbp import (  # noqa: F401
    MIN_TRANSMISSION,
    dark_flat_mean,
    normalize,
    pad_len,
    ramp_kernel,
    ramp_response,
    FILTERS,
    filter_window,
    filter_kernel,
    filter_response,
    pad_rows,
    filter_rows,
    filter_rows_direct,
    round_binary16,
    round_f16,
    round_bf16,
    backproject,
    backproject_points,
    radon,
    fbp,
    fbp_points,
    filter_rows_padded,
    fourier_backproject,
    fourier_backproject_points,
    fourier_fbp,
    fourier_fbp_points,
    lamino_backproject,
    lamino_backproject_points,
    power_lambda_max,
    ls_gradient,
    ls_solve,
    num_threads,
    set_num_threads,
)
from . import lprec  # noqa: F401,E402
