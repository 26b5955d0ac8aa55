"""Log-polar-based backprojection ("LpRec") in FP64 (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; the product library never imports it.

The paper (Sections 2.2 and 3) lists the method as its third backprojector:
the backprojection over a range of equally spaced angles is a convolution in
log-polar coordinates, evaluated with FFTs, with cubic-spline interpolations
to and from the log-polar grid done in the image domain.  It gives no grids,
origin shift or spline details; the reading implemented here (also stated in
the library's header) is:

1. Rows.  Each padded filtered row y_a (length L) is represented by its
   trigonometric interpolant (the sum the Fourier-domain oracle evaluates),
   resampled at half-sample spacing by zero-padding its spectrum to 2L (the
   Nyquist term split evenly), and turned into periodic B-spline coefficients
   of degree ``deg`` by dividing that spectrum by the B-spline's sampled
   transform (degree 5: (66 + 52 cos w + 2 cos 2w) / 120).

2. Spans.  The n_angles equally spaced angles theta_a = theta_0 + a pi /
   n_angles are split into ``spans`` consecutive groups of n_span =
   ceil(n_angles / spans) slots (missing slots of the last group are empty).
   Span p is rotated by its centre angle beta_p so that its angles sit at
   phi_k = (k - (n_span - 1) / 2) dtheta, |phi_k| <= phi_max.

3. Origin shift.  In span coordinates the image (every voxel centre within R
   of the axis point) is moved by a0 = (1 + eps) R / cos(phi_max) along the
   first axis, so every ray offset s'' = x''.(cos phi, sin phi) of an image
   point is at least eps R > 0.  Writing x'' = e^rho (cos psi, sin psi), the
   span's backprojection becomes
       F_p(psi, rho) = dtheta sum_k G_k(rho + log cos(psi - phi_k)),
       G_k(sigma) = Y_a(e^sigma - a0 cos phi_k + pos0),
   a convolution in (angle, log-radius).

4. Log-polar grid.  sigma_j = sigma_0 + j delta, j < Ns (a power of two,
   >= 1024), spread so that [log(eps R), log(a0 + R)] occupies
   [margin, Ns - 1 - margin] at a spacing of at most 1 / (os * (a0 + R)).
   G_k is evaluated there by the B-spline of step 1 and multiplied by a
   raised-cosine taper that is 1 on that range and 0 within 2 points of the
   ends.  Angles: psi_m = phi_0 + m dpsi, dpsi = dtheta / M, M the power of
   two with dpsi <= 1 / (os (a0 + R)); rows m_lo..m_hi cover
   |psi| <= asin(R / a0) plus ``margin_a`` rows each side.

5. Convolution.  Along sigma the shift by log cos(d dpsi) is exact for the
   sampled band: DFT over j, multiply by exp(2 pi i eta ell(d) / (delta Ns))
   (eta signed; the Nyquist term takes the cosine).  Along psi the sum over k
   is a linear convolution of the sequence Ghat_k placed at every M-th index
   with that kernel over d = m - M k, done by FFTs of length NA (a power of
   two, >= rows + M (n_span - 1)).

6. Prefilters.  Both inverse transforms divide by the sampled B-spline
   transform of their length, so the inverse FFTs return B-spline
   coefficients C(m, j) of F_p (the scale dtheta included).

7. Evaluation.  A voxel (ix, iy), x = ix - N//2, y = iy - N//2, is mapped
   into every span's frame (rho, psi) and the tensor-product B-spline of
   degree ``deg`` is evaluated there; the spans are summed.

Parity status: pinned in ``tests/test_oracle_lprec.py`` -- convergence to the
direct sum of trigonometric interpolants as the oversampling grows, the
convolution step against a direct sum at grid nodes, the row splines against
FFT-upsampled rows, B-spline evaluation at grid nodes, constant rows, the
sizing constraints.
"""
from __future__ import annotations

import math

import numpy as np

SIGMA_MARGIN = 12    # grid points of sigma padding (taper) beyond the data range
ANGLE_MARGIN = 16    # psi rows beyond the image sector
WINDOW_MARGIN = 4    # sigma points kept beyond the image's rho range
MIN_FFT = 1024
MAX_FFT = 16384


def _pow2_at_least(v: int) -> int:
    return 1 << max(0, int(math.ceil(math.log2(max(v, 1)))))


def lprec_params(n_angles: int, N: int, spans: int = 3, os: float = 1.0, eps: float = 1.0) -> dict:
    """Grid sizes and geometry of the log-polar backprojection (steps 2-4 of the
    module docstring) for n_angles equally spaced angles over a half turn and
    an N x N slice."""
    if spans < 2:
        raise ValueError("need at least two spans")
    dtheta = math.pi / n_angles
    half = N // 2
    R = math.sqrt(2.0) * half + 2.0
    n_span = -(-n_angles // spans)
    phi_max = 0.5 * (n_span - 1) * dtheta
    a0 = (1.0 + eps) * R / math.cos(phi_max)
    s_min = a0 * math.cos(phi_max) - R
    s_max = a0 + R
    lo, hi = math.log(s_min), math.log(s_max)
    n_need = int(math.ceil((hi - lo) * os * s_max)) + 2 * SIGMA_MARGIN + 1
    Ns = max(MIN_FFT, _pow2_at_least(n_need))
    delta = (hi - lo) / (Ns - 1 - 2 * SIGMA_MARGIN)
    sigma0 = lo - SIGMA_MARGIN * delta
    M = _pow2_at_least(int(math.ceil(os * dtheta * s_max)))
    dpsi = dtheta / M
    phi0 = -phi_max
    psi_max = math.asin(R / a0)
    m_lo = int(math.floor((-psi_max - phi0) / dpsi)) - ANGLE_MARGIN
    m_hi = int(math.ceil((psi_max - phi0) / dpsi)) + ANGLE_MARGIN
    rows = m_hi - m_lo + 1
    D = rows + M * (n_span - 1)
    NA = max(MIN_FFT, _pow2_at_least(D))
    d_lo = m_lo - M * (n_span - 1)
    if (d_lo * dpsi <= -math.pi / 2) or ((d_lo + D - 1) * dpsi >= math.pi / 2):
        raise ValueError("angular margin does not fit below 90 degrees; increase eps")
    j_lo = int(math.floor((math.log(a0 - R) - sigma0) / delta)) - WINDOW_MARGIN
    j_hi = int(math.ceil((math.log(a0 + R) - sigma0) / delta)) + WINDOW_MARGIN
    return dict(n_angles=n_angles, N=N, spans=spans, os=os, eps=eps, dtheta=dtheta, R=R, n_span=n_span,
                phi_max=phi_max, phi0=phi0, a0=a0, s_min=s_min, s_max=s_max, Ns=Ns, delta=delta, sigma0=sigma0,
                M=M, dpsi=dpsi, psi_max=psi_max, m_lo=m_lo, rows=rows, D=D, NA=NA, d_lo=d_lo,
                j_lo=j_lo, nj=j_hi - j_lo + 1)


def bspline_hat(k, n: int, deg: int = 5):
    """Sampled transform sum_m beta(m) exp(-2 pi i k m / n) of the centred
    B-spline of degree 3 or 5 (real, even)."""
    w = 2.0 * np.pi * np.asarray(k, dtype=np.float64) / n
    if deg == 3:
        return (4.0 + 2.0 * np.cos(w)) / 6.0
    if deg == 5:
        return (66.0 + 52.0 * np.cos(w) + 2.0 * np.cos(2.0 * w)) / 120.0
    raise ValueError("degree 3 or 5")


def bspline_weights(t, deg: int = 5):
    """Weights beta(t - i) of the taps i = -(deg // 2) .. deg // 2 + 1 around a
    point at fraction t in [0, 1) past its floor (closed forms of the centred
    B-splines).  Returns (offsets, [weights])."""
    t = np.asarray(t, dtype=np.float64)
    if deg == 3:
        offs = (-1, 0, 1, 2)
    elif deg == 5:
        offs = (-2, -1, 0, 1, 2, 3)
    else:
        raise ValueError("degree 3 or 5")
    ws = []
    for o in offs:
        x = np.abs(t - o)
        if deg == 3:
            w = np.where(x < 1.0, 2.0 / 3.0 - x * x + 0.5 * x ** 3, np.where(x < 2.0, (2.0 - x) ** 3 / 6.0, 0.0))
        else:
            w = np.where(x < 1.0, 11.0 / 20.0 - x ** 2 / 2.0 + x ** 4 / 4.0 - x ** 5 / 12.0,
                         np.where(x < 2.0, 17.0 / 40.0 + 5.0 * x / 8.0 - 7.0 * x ** 2 / 4.0 + 5.0 * x ** 3 / 4.0
                                  - 3.0 * x ** 4 / 8.0 + x ** 5 / 24.0,
                                  np.where(x < 3.0, (3.0 - x) ** 5 / 120.0, 0.0)))
        ws.append(w)
    return offs, ws


def row_splines(y: np.ndarray, deg: int = 5) -> np.ndarray:
    """Step 1: periodic B-spline coefficients, at half-sample spacing, of the
    trigonometric interpolant of each padded row y [..., L] -> [..., 2L]."""
    y = np.asarray(y, dtype=np.float64)
    L = y.shape[-1]
    Y = np.fft.fft(y, axis=-1)
    Z = np.zeros(y.shape[:-1] + (2 * L,), dtype=complex)
    h = L // 2
    Z[..., :h] = Y[..., :h]
    Z[..., 2 * L - h + 1:] = Y[..., h + 1:]
    Z[..., h] = 0.5 * Y[..., h]
    Z[..., 2 * L - h] = 0.5 * Y[..., h]
    k = np.fft.fftfreq(2 * L) * (2 * L)
    return np.fft.ifft(2.0 * Z / bspline_hat(k, 2 * L, deg), axis=-1).real


def spline_eval_periodic(c: np.ndarray, u, deg: int = 5):
    """sum_i c[(floor(u) + i) mod n] beta(u - floor(u) - i) for one coefficient row c."""
    n = c.shape[-1]
    u = np.asarray(u, dtype=np.float64)
    i0 = np.floor(u).astype(np.int64)
    offs, ws = bspline_weights(u - i0, deg)
    out = np.zeros(u.shape)
    for o, w in zip(offs, ws):
        out += w * c[(i0 + o) % n]
    return out


def taper(Ns: int) -> np.ndarray:
    """Raised cosine: 0 at j <= 2 and j >= Ns - 3, 1 on [SIGMA_MARGIN, Ns - 1 - SIGMA_MARGIN]."""
    j = np.arange(Ns, dtype=np.float64)
    ramp = SIGMA_MARGIN - 2
    tl = np.clip((j - 2.0) / ramp, 0.0, 1.0)
    th = np.clip((Ns - 3.0 - j) / ramp, 0.0, 1.0)
    return np.minimum(0.5 - 0.5 * np.cos(np.pi * tl), 0.5 - 0.5 * np.cos(np.pi * th))


def span_angles(pr: dict, theta0: float, p: int):
    """(beta_p, [a for each slot k or -1 when empty]) of span p."""
    n_span, na = pr["n_span"], pr["n_angles"]
    beta = theta0 + (p * n_span + 0.5 * (n_span - 1)) * pr["dtheta"]
    slots = [p * n_span + k if p * n_span + k < na else -1 for k in range(n_span)]
    return beta, slots


def log_radial_samples(c_rows: np.ndarray, pr: dict, slots, pos0: float, deg: int = 5) -> np.ndarray:
    """Steps 3-4: G_k(sigma_j) (tapered) for the slots of one span [n_span][Ns]."""
    Ns, dth = pr["Ns"], pr["dtheta"]
    sig = pr["sigma0"] + pr["delta"] * np.arange(Ns)
    es = np.exp(sig)
    w = taper(Ns)
    G = np.zeros((len(slots), Ns))
    for k, a in enumerate(slots):
        if a < 0:
            continue
        phi = (k - 0.5 * (pr["n_span"] - 1)) * dth
        u = 2.0 * (es - pr["a0"] * math.cos(phi) + pos0)
        G[k] = w * spline_eval_periodic(c_rows[a], u, deg)
    return G


def shift_kernel(pr: dict) -> np.ndarray:
    """K[d', eta] = exp(2 pi i eta ell(d) / (delta Ns)), ell(d) = log cos(d dpsi),
    d = d' + d_lo for d' < D (zero beyond), eta signed; cosine at Nyquist. [NA][Ns]."""
    Ns, D, NA = pr["Ns"], pr["D"], pr["NA"]
    d = pr["d_lo"] + np.arange(D)
    ell = np.log(np.cos(d * pr["dpsi"]))
    eta = np.fft.fftfreq(Ns) * Ns
    K = np.zeros((NA, Ns), dtype=complex)
    K[:D] = np.exp(2j * np.pi * np.outer(ell, eta) / (pr["delta"] * Ns))
    K[:D, Ns // 2] = np.cos(np.pi * ell / pr["delta"])
    return K


def span_coefficients(G: np.ndarray, pr: dict, deg: int = 5, K: np.ndarray | None = None) -> np.ndarray:
    """Steps 5-6: B-spline coefficients C[m - m_lo][j] of F_p on the log-polar
    grid, rows m_lo..m_hi, all Ns sigma points (scale dtheta included)."""
    Ns, NA, M, n_span, rows = pr["Ns"], pr["NA"], pr["M"], pr["n_span"], pr["rows"]
    Gh = np.fft.fft(G, axis=-1)
    Z = np.zeros((NA, Ns), dtype=complex)
    Z[0:M * n_span:M] = Gh
    if K is None:
        K = shift_kernel(pr)
    nu = np.fft.fftfreq(NA) * NA
    eta = np.fft.fftfreq(Ns) * Ns
    conv = np.fft.ifft(np.fft.fft(Z, axis=0) * np.fft.fft(K, axis=0) / bspline_hat(nu, NA, deg)[:, None], axis=0)
    first = M * (n_span - 1)
    Fh = conv[first:first + rows]
    return pr["dtheta"] * np.fft.ifft(Fh / bspline_hat(eta, Ns, deg)[None, :], axis=1).real


def span_points(C: np.ndarray, pr: dict, beta: float, ix, iy, deg: int = 5) -> np.ndarray:
    """Step 7: the span's spline at voxels (ix, iy)."""
    half = pr["N"] // 2
    x = np.asarray(ix, dtype=np.float64) - half
    y = np.asarray(iy, dtype=np.float64) - half
    cb, sb = math.cos(beta), math.sin(beta)
    xp = cb * x + sb * y + pr["a0"]
    yp = -sb * x + cb * y
    rho = 0.5 * np.log(xp * xp + yp * yp)
    psi = np.arctan2(yp, xp)
    tj = (rho - pr["sigma0"]) / pr["delta"]
    tm = (psi - pr["phi0"]) / pr["dpsi"] - pr["m_lo"]
    j0 = np.floor(tj).astype(np.int64)
    m0 = np.floor(tm).astype(np.int64)
    offs, wj = bspline_weights(tj - j0, deg)
    _, wm = bspline_weights(tm - m0, deg)
    assert np.all(m0 + offs[0] >= 0) and np.all(m0 + offs[-1] < pr["rows"])
    assert np.all(j0 + offs[0] >= pr["j_lo"]) and np.all(j0 + offs[-1] < pr["j_lo"] + pr["nj"])
    out = np.zeros(x.shape)
    for oi, a in zip(offs, wm):
        for oj, b in zip(offs, wj):
            out += a * b * C[m0 + oi, j0 + oj]
    return out


def lprec_backproject_points(y: np.ndarray, theta0: float, pos0: float, N: int, ix, iy, spans: int = 3,
                             os: float = 1.0, eps: float = 1.0, deg: int = 5) -> np.ndarray:
    """Log-polar backprojection of one slice's padded filtered rows y [n_angles][L]
    (angles theta0 + a pi / n_angles) at voxels (ix, iy); pos0 = centre + pad
    offset.  Approximates ``fourier_backproject_points`` (scale pi / n_angles)."""
    y = np.asarray(y, dtype=np.float64)
    pr = lprec_params(y.shape[0], N, spans, os, eps)
    c_rows = row_splines(y, deg)
    K = shift_kernel(pr)
    out = np.zeros(np.asarray(ix).shape)
    for p in range(spans):
        beta, slots = span_angles(pr, theta0, p)
        G = log_radial_samples(c_rows, pr, slots, pos0, deg)
        C = span_coefficients(G, pr, deg, K)
        out += span_points(C, pr, beta, ix, iy, deg)
    return out


def lprec_backproject(y: np.ndarray, theta0: float, pos0: float, N: int, **kw) -> np.ndarray:
    """``lprec_backproject_points`` at every voxel: y [nz][n_angles][L] -> [nz][N][N]."""
    y = np.asarray(y, dtype=np.float64)
    if y.ndim == 2:
        y = y[None]
    iy, ix = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    return np.stack([lprec_backproject_points(y[z], theta0, pos0, N, ix.ravel(), iy.ravel(), **kw).reshape(N, N)
                     for z in range(y.shape[0])])


def lprec_fbp(proj, dark, flat, theta0: float, center: float, N: int | None = None, kind: str = "ramp", **kw):
    """LpRec FBP: normalise, pad, filter, then the log-polar backprojection."""
    from .fbp import filter_rows_padded, normalize

    p = normalize(proj, dark, flat)
    n = p.shape[-1]
    y, off = filter_rows_padded(p, kind=kind)
    return lprec_backproject(y, theta0, center + off, n if N is None else N, **kw)
