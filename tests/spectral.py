"""Frequency extraction for probe traces (test helper).

A single-tone least-squares fit: the periodogram peak seeds the search, then
the frequency minimising the residual of x(t) ~ a cos(2 pi f t) +
b sin(2 pi f t) + c (+ d t) is found by bounded scalar minimisation.
"""
import numpy as np
from scipy.optimize import minimize_scalar


def tone_frequency(x, dt, drift=False, pad=16):
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    t = np.arange(n) * dt
    xc = x - x.mean()
    spec = np.abs(np.fft.rfft(xc * np.hanning(n), pad * n))
    k = int(np.argmax(spec[1:])) + 1
    f_seed = k / (pad * n * dt)
    cols = [np.ones(n)] + ([t / t[-1]] if drift else [])

    def resid(f):
        A = np.stack([np.cos(2 * np.pi * f * t), np.sin(2 * np.pi * f * t)] + cols, 1)
        coef, *_ = np.linalg.lstsq(A, x, rcond=None)
        r = A @ coef - x
        return float(r @ r)

    df = 2.0 / (n * dt)
    res = minimize_scalar(resid, bounds=(max(f_seed - df, 1e-30), f_seed + df), method="bounded",
                          options={"xatol": f_seed * 1e-12, "maxiter": 500})
    return float(res.x)
