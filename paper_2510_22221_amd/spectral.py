"""Spectral analysis of probe traces: spectra, ESPRIT modes, Kittel and
anti-crossing fits (arXiv:2510.22221, Results: the Fourier-transformed E_x
spectra of Fig. 3d/3e, the ESPRIT frequencies and Q factors of Fig. 4e/4f,
the Kittel law for the film's resonance, and eq. omega_pm for the two hybrid
modes).

Host-side post-processing of the traces that the GPU probes record; none of it
is on the time-stepping path.  Frequencies are in Hz, times in s.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np

MU0 = 4e-7 * np.pi


# ---------------------------------------------------------------------------
# spectra
# ---------------------------------------------------------------------------
def spectrum(x, dt: float, pad: int = 8, window: str = "hann", detrend: bool = True):
    """One-sided magnitude spectrum |X(f)| of a real trace (zero-padded to
    pad * len(x) samples); returns (f, |X|)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if n < 2:
        raise ValueError("trace too short")
    if detrend:
        x = x - x.mean()
    w = np.hanning(n) if window == "hann" else np.ones(n)
    nfft = max(n, int(pad) * n)
    X = np.fft.rfft(x * w, nfft)
    f = np.fft.rfftfreq(nfft, dt)
    return f, np.abs(X)


def peak_frequencies(x, dt: float, n_peaks: int = 2, pad: int = 16, fmin: float = 0.0,
                     fmax: Optional[float] = None):
    """Frequencies of the n_peaks largest local maxima of the spectrum in
    [fmin, fmax], each refined by a parabola through the log magnitudes of the
    peak bin and its neighbours; sorted ascending."""
    f, a = spectrum(x, dt, pad=pad)
    sel = (f >= fmin) & (f <= (fmax if fmax is not None else f[-1]))
    la = np.log(a + 1e-300)
    cand = [k for k in range(1, f.size - 1) if sel[k] and a[k] >= a[k - 1] and a[k] > a[k + 1]]
    cand.sort(key=lambda k: -a[k])
    out = []
    df = f[1] - f[0]
    for k in cand[:n_peaks]:
        y0, y1, y2 = la[k - 1], la[k], la[k + 1]
        den = y0 - 2.0 * y1 + y2
        off = 0.5 * (y0 - y2) / den if den != 0 else 0.0
        out.append(f[k] + off * df)
    return np.sort(np.array(out))


# ---------------------------------------------------------------------------
# ESPRIT (Roy and Kailath's rotational-invariance method)
# ---------------------------------------------------------------------------
@dataclass
class Modes:
    f: np.ndarray       # frequency, Hz (ascending)
    Q: np.ndarray       # quality factor pi f / sigma (inf when undamped)
    sigma: np.ndarray   # amplitude decay rate, 1/s
    amp: np.ndarray     # amplitude of the real cosine (2 |a_k| for a real trace)
    phase: np.ndarray   # phase of the cosine at the first sample, rad


def esprit(x, dt: float, n_modes: int, L: Optional[int] = None, stride: int = 1,
           max_rows: int = 2048) -> Modes:
    """Frequencies, decay rates, Q and amplitudes of the n_modes damped
    sinusoids that best explain a real trace.

    The trace (taken every `stride` samples) is arranged in a Hankel matrix
    with L rows; the leading 2 n_modes left singular vectors span the signal
    subspace, whose shift invariance (rows 1.. equal rows ..-1 times a
    matrix) gives the poles z_k as eigenvalues of the least-squares shift
    matrix.  f = arg z / (2 pi dt'), sigma = -ln|z| / dt', Q = pi f / sigma;
    the complex amplitudes come from a least-squares Vandermonde fit."""
    x = np.asarray(x, dtype=np.float64)[::max(1, int(stride))]
    dts = dt * max(1, int(stride))
    n = x.size
    K = 2 * int(n_modes)
    if n < 2 * K + 2:
        raise ValueError("trace too short for the requested number of modes")
    if L is None:
        L = min(n // 2, max_rows)
    L = max(K + 1, min(L, n - K))
    cols = n - L + 1
    idx = np.arange(L)[:, None] + np.arange(cols)[None, :]
    H = x[idx]
    U, s, _ = np.linalg.svd(H, full_matrices=False)
    Us = U[:, :K]
    Phi, *_ = np.linalg.lstsq(Us[:-1], Us[1:], rcond=None)
    z = np.linalg.eigvals(Phi)
    # Vandermonde fit of the complex amplitudes over the whole trace
    V = z[None, :] ** np.arange(n)[:, None]
    a, *_ = np.linalg.lstsq(V, x.astype(np.complex128), rcond=None)
    f = np.angle(z) / (2.0 * np.pi * dts)
    keep = f > 0
    z, a, f = z[keep], a[keep], f[keep]
    order = np.argsort(f)
    z, a, f = z[order][:n_modes], a[order][:n_modes], f[order][:n_modes]
    sigma = -np.log(np.abs(z)) / dts
    with np.errstate(divide="ignore"):
        Q = np.where(sigma > 0, np.pi * f / np.where(sigma > 0, sigma, 1.0), np.inf)
    return Modes(f=f, Q=Q, sigma=sigma, amp=2.0 * np.abs(a), phase=np.angle(a))


# ---------------------------------------------------------------------------
# resonance laws
# ---------------------------------------------------------------------------
def kittel_inplane(H0, Ms, mu0_gamma=MU0 * 1.76e11):
    """In-plane film FMR (Kittel law): f = (mu0 |gamma| / 2 pi)
    sqrt(H0 (H0 + Ms)), SI units (A/m)."""
    H0 = np.asarray(H0, dtype=np.float64)
    return mu0_gamma / (2.0 * np.pi) * np.sqrt(H0 * (H0 + Ms))


def kittel_inplane_cgs(H0_Oe, four_pi_Ms_G, gamma_over_2pi_Hz_per_Oe=2.8e6):
    """The same law in the Gaussian units the paper quotes it in:
    f = (gamma / 2 pi) sqrt(H0 (H0 + 4 pi Ms))."""
    H0 = np.asarray(H0_Oe, dtype=np.float64)
    return gamma_over_2pi_Hz_per_Oe * np.sqrt(H0 * (H0 + four_pi_Ms_G))


def kittel_perpendicular(H0, Ms, mu0_gamma=MU0 * 1.76e11):
    """Film magnetised along its normal: f = (mu0 |gamma| / 2 pi)(H0 - Ms)."""
    H0 = np.asarray(H0, dtype=np.float64)
    return mu0_gamma / (2.0 * np.pi) * (H0 - Ms)


def omega_pm(fp, delta, g):
    """Eq. omega_pm: the two hybrid-mode frequencies
    fp + delta/2 -+ sqrt(delta^2 + 4 g^2)/2 (lower, upper); any consistent
    unit (Hz or rad/s)."""
    fp = np.asarray(fp, dtype=np.float64)
    delta = np.asarray(delta, dtype=np.float64)
    r = np.sqrt(delta * delta + 4.0 * g * g) / 2.0
    c = fp + delta / 2.0
    return c - r, c + r


@dataclass
class AntiCrossingFit:
    fp: float           # photon (resonator) frequency
    g: float            # coupling of eq. omega_pm (minimum splitting 2 g)
    scale: float        # multiplier of the magnon branch fm(H0)
    residual_rms: float
    offset: float = 0.0  # added to the magnon branch (fit_offset)


def fit_anticrossing(H0, f_lower, f_upper, fm_of_H0, fp0: float, g0: float, fit_scale: bool = False,
                     fit_offset: bool = False):
    """Least-squares fit of eq. omega_pm to the two branches measured over a
    bias sweep, with the detuning delta(H0) = s fm(H0) + c - fp taken from a
    magnon law fm (for example kittel_inplane); fits fp, g (and s when
    fit_scale, c when fit_offset: a magnon branch linear in the law, for
    static demagnetising and surface shifts the law leaves out)."""
    from scipy.optimize import least_squares

    H0 = np.asarray(H0, dtype=np.float64)
    lo = np.asarray(f_lower, dtype=np.float64)
    hi = np.asarray(f_upper, dtype=np.float64)
    fm = np.asarray(fm_of_H0(H0), dtype=np.float64)
    unit = float(max(abs(fp0), 1.0))

    def unpack(v):
        q = 2
        s = 1.0
        if fit_scale:
            s = v[q]
            q += 1
        c = v[q] * unit if fit_offset else 0.0
        return v[0] * unit, v[1] * unit, s, c

    def resid(v):
        fp, g, s, c = unpack(v)
        a, b = omega_pm(fp, s * fm + c - fp, g)
        return np.concatenate([a - lo, b - hi]) / unit

    v0 = [fp0 / unit, g0 / unit] + ([1.0] if fit_scale else []) + ([0.0] if fit_offset else [])
    r = least_squares(resid, v0, xtol=1e-15, ftol=1e-15, gtol=1e-15)
    fp, g, s, c = unpack(r.x)
    return AntiCrossingFit(fp=float(fp), g=float(abs(g)), scale=float(s),
                           residual_rms=float(np.sqrt(np.mean(r.fun ** 2)) * unit), offset=float(c))


def sweep_branches(traces: Sequence[np.ndarray], dt: float, n_modes: int = 2, stride: int = 1,
                   fmin: float = 0.0, fmax: Optional[float] = None, min_separation: float = 0.0,
                   max_rows: int = 2048) -> np.ndarray:
    """ESPRIT frequencies (n_traces x n_modes, ascending per trace) of a bias
    sweep's probe traces, restricted to [fmin, fmax]: per trace the strongest
    modes taken in order of amplitude, skipping any closer than
    `min_separation` (relative) to one already taken (a mode the fit splits
    into a close pair counts once); missing modes are NaN."""
    out = np.full((len(traces), n_modes), np.nan)
    for q, x in enumerate(traces):
        x = np.asarray(x, dtype=np.float64)
        m = esprit(x - x.mean(), dt, n_modes + 2, stride=stride, max_rows=max_rows)
        sel = (m.f >= fmin) & (m.f <= (fmax if fmax is not None else np.inf))
        f = m.f[sel]
        a = m.amp[sel]
        top = []
        for k in np.argsort(-a):
            if all(abs(f[k] - t) > min_separation * t for t in top):
                top.append(f[k])
            if len(top) == n_modes:
                break
        top = np.sort(top)
        out[q, :top.size] = top
    return out


def mode_splitting(f_lower, f_upper) -> Tuple[float, int]:
    """Minimum distance between the two branches over a sweep and its index."""
    d = np.asarray(f_upper) - np.asarray(f_lower)
    q = int(np.nanargmin(d))
    return float(d[q]), q
