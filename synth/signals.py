"""Seeded synthetic probe traces for the spectral tools: sums of damped
cosines x(t) = sum_k A_k exp(-sigma_k t) cos(2 pi f_k t + phi_k), optionally
with white noise.  Inputs only (no analysis arithmetic)."""
from __future__ import annotations

import numpy as np

SEED = 22221


def damped_cosines(n: int, dt: float, f, sigma, amp, phase=None, noise: float = 0.0, seed: int = SEED):
    t = np.arange(n) * dt
    f = np.atleast_1d(np.asarray(f, dtype=np.float64))
    sigma = np.broadcast_to(np.asarray(sigma, dtype=np.float64), f.shape)
    amp = np.broadcast_to(np.asarray(amp, dtype=np.float64), f.shape)
    phase = np.zeros_like(f) if phase is None else np.broadcast_to(np.asarray(phase, dtype=np.float64), f.shape)
    x = np.zeros(n)
    for k in range(f.size):
        x += amp[k] * np.exp(-sigma[k] * t) * np.cos(2.0 * np.pi * f[k] * t + phase[k])
    if noise > 0:
        x += noise * np.random.default_rng(seed).standard_normal(n)
    return x
