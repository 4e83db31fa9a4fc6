"""Plain definitions for checking the spectral tools (TEST INFRASTRUCTURE
ONLY; shares no code with the package).

* dft_mag: |sum_n w_n x_n exp(-2 pi i f n dt)| by direct summation, the
  definition of the windowed discrete-time Fourier transform the spectra of
  Results (Fig. 3d/3e) are samples of.
* omega_pm_oracle: eq. omega_pm written out term by term.
* kittel_oracle: the Kittel law of Results, (gamma/2pi) sqrt(H0 (H0 + 4 pi
  Ms)), in Gaussian units.
"""
import math

import numpy as np


def dft_mag(x, dt, freqs, window="hann"):
    x = [float(v) for v in x]
    n = len(x)
    mean = sum(x) / n
    w = [0.5 - 0.5 * math.cos(2.0 * math.pi * q / (n - 1)) for q in range(n)] if window == "hann" else [1.0] * n
    out = []
    for f in freqs:
        re = im = 0.0
        for q in range(n):
            ph = 2.0 * math.pi * f * q * dt
            v = (x[q] - mean) * w[q]
            re += v * math.cos(ph)
            im -= v * math.sin(ph)
        out.append(math.hypot(re, im))
    return np.array(out)


def omega_pm_oracle(wp, delta, g):
    root = math.sqrt(delta ** 2 + 4.0 * g ** 2)
    return wp + delta / 2.0 - root / 2.0, wp + delta / 2.0 + root / 2.0


def kittel_oracle(H0_Oe, four_pi_Ms_G, gamma_over_2pi=2.8e6):
    return gamma_over_2pi * math.sqrt(H0_Oe * (H0_Oe + four_pi_Ms_G))
