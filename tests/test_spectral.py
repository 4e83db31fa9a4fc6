"""Spectral tools (spectra, ESPRIT, Kittel and anti-crossing fits) against
plain definitions, exact synthetic signals and the paper's printed numbers.
CPU only."""
import json
import os

import numpy as np
import pytest

from oracle import spectral_oracle as SO
from paper_2510_22221_amd import spectral as S
from synth import signals as G

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_spectrum_equals_direct_dft():
    x = G.damped_cosines(257, 1e-12, [31e9, 77e9], [1e9, 4e9], [1.0, 0.4], [0.3, -1.1], noise=0.05)
    f, a = S.spectrum(x, 1e-12, pad=2)
    pick = [0, 3, 17, 64, 129, 255]
    ref = SO.dft_mag(x, 1e-12, f[pick])
    assert np.allclose(a[pick], ref, rtol=1e-10, atol=1e-12 * ref.max())


def test_peak_frequency_of_a_tone_between_bins():
    dt, n = 1e-12, 4000
    f0 = 12.3456789e9
    x = G.damped_cosines(n, dt, [f0], [0.0], [1.0], [0.4])
    (f,) = S.peak_frequencies(x, dt, 1, pad=16)
    assert abs(f - f0) < 0.02 / (n * dt)


def test_esprit_recovers_two_damped_modes_exactly():
    # the paper's hybrid-mode frequencies with unequal Q and amplitude
    dt, n = 5e-12, 800
    f = np.array([14.95e9, 15.65e9])
    Q = np.array([800.0, 300.0])
    sigma = np.pi * f / Q
    amp, ph = np.array([1.0, 0.35]), np.array([0.2, -2.0])
    x = G.damped_cosines(n, dt, f, sigma, amp, ph)
    m = S.esprit(x, dt, 2)
    assert np.allclose(m.f, f, rtol=1e-9)
    assert np.allclose(m.Q, Q, rtol=1e-6)
    assert np.allclose(m.amp, amp, rtol=1e-7)
    assert np.allclose(np.angle(np.exp(1j * (m.phase - ph))), 0.0, atol=1e-7)


def test_esprit_noise_and_stride():
    dt, n = 1e-12, 6000
    f = np.array([14.95e9, 15.65e9])
    sigma = np.pi * f / np.array([500.0, 500.0])
    x = G.damped_cosines(n, dt, f, sigma, [1.0, 1.0], [0.0, 1.0], noise=1e-3)
    m = S.esprit(x, dt, 2, stride=3)
    assert np.allclose(m.f, f, rtol=2e-4)
    assert np.allclose(m.Q, 500.0, rtol=0.05)


def test_undamped_mode_has_infinite_or_huge_Q():
    dt, n = 5e-12, 400
    x = G.damped_cosines(n, dt, [10e9], [0.0], [1.0])
    m = S.esprit(x, dt, 1)
    assert abs(m.f[0] - 10e9) < 1e-3
    assert m.Q[0] > 1e9


def test_omega_pm_definition_and_invariants():
    for wp, d, g in [(15.2, 0.2, 0.335), (3.0, -0.7, 0.05), (1.0, 0.0, 0.2)]:
        lo, hi = S.omega_pm(wp, d, g)
        rlo, rhi = SO.omega_pm_oracle(wp, d, g)
        assert lo == pytest.approx(rlo, rel=1e-15) and hi == pytest.approx(rhi, rel=1e-15)
        assert lo + hi == pytest.approx(2 * wp + d, rel=1e-14)
        assert hi - lo >= 2 * g * (1 - 1e-15)
        if d == 0.0:
            assert hi - lo == pytest.approx(2 * g, rel=1e-15)


def test_omega_pm_reproduces_the_printed_hybrid_modes():
    h = GOLD["hybrid_modes"]
    lo, hi = S.omega_pm(h["fp_GHz"], h["delta_GHz"], h["g_mp_GHz"] / 2)
    assert lo == pytest.approx(h["f_lower_GHz"], rel=h["rel_tol"])
    assert hi == pytest.approx(h["f_upper_GHz"], rel=h["rel_tol"])


def test_kittel_printed_value_and_unit_systems():
    k = GOLD["kittel_main"]
    f = S.kittel_inplane_cgs(k["H0_Oe"], k["four_pi_Ms_G"])
    assert f / 1e9 == pytest.approx(k["f_GHz"], rel=k["rel_tol"])
    assert f == pytest.approx(SO.kittel_oracle(k["H0_Oe"], k["four_pi_Ms_G"]), rel=1e-15)
    # SI form with gamma/2pi = 2.8 MHz/Oe, 1 Oe = 1000/(4 pi) A/m
    oe = 1000.0 / (4 * np.pi)
    mu0_gamma = 2 * np.pi * 2.8e6 / oe
    fsi = S.kittel_inplane(k["H0_Oe"] * oe, k["four_pi_Ms_G"] * oe, mu0_gamma)
    assert fsi == pytest.approx(f, rel=1e-13)
    assert S.kittel_perpendicular(2e5, 1.4e5, mu0_gamma) == pytest.approx(mu0_gamma / (2 * np.pi) * 6e4, rel=1e-15)


def test_anticrossing_fit_recovers_parameters():
    H0 = np.linspace(1.3e5, 1.9e5, 41)
    fm = lambda h: S.kittel_inplane(h, 9.7e5, 2.23e5)
    fp, g = 15.2e9, 0.335e9
    lo, hi = S.omega_pm(fp, fm(H0) - fp, g)
    r = S.fit_anticrossing(H0, lo, hi, fm, fp0=14.8e9, g0=0.2e9)
    assert r.fp == pytest.approx(fp, rel=1e-9)
    assert r.g == pytest.approx(g, rel=1e-8)
    r2 = S.fit_anticrossing(H0, lo, hi, lambda h: 1.01 * fm(h), fp0=14.8e9, g0=0.2e9, fit_scale=True)
    assert r2.scale == pytest.approx(1 / 1.01, rel=1e-8)
    # a magnon branch 0.8 fm + 2 GHz: slope and offset recovered
    lo3, hi3 = S.omega_pm(fp, 0.8 * fm(H0) + 2e9 - fp, g)
    r3 = S.fit_anticrossing(H0, lo3, hi3, fm, fp0=14.8e9, g0=0.2e9, fit_scale=True, fit_offset=True)
    assert r3.scale == pytest.approx(0.8, rel=1e-7)
    assert r3.offset == pytest.approx(2e9, rel=1e-6)
    assert r3.g == pytest.approx(g, rel=1e-7) and r3.fp == pytest.approx(fp, rel=1e-9)
    d, q = S.mode_splitting(lo, hi)
    assert d >= 2 * g * (1 - 1e-12) and d == pytest.approx(2 * g, rel=2e-3)


def test_sweep_branches_from_synthetic_traces():
    dt, n = 5e-12, 600
    fp, g = 15.2e9, 0.335e9
    fms = np.linspace(14.2e9, 16.2e9, 9)
    lo, hi = S.omega_pm(fp, fms - fp, g)
    traces = [G.damped_cosines(n, dt, [a, b], [3e7, 3e7], [1.0, 0.8], [0.1, 0.7]) for a, b in zip(lo, hi)]
    br = S.sweep_branches(traces, dt, 2, fmin=10e9, fmax=20e9)
    assert np.allclose(br[:, 0], lo, rtol=1e-8)
    assert np.allclose(br[:, 1], hi, rtol=1e-8)


def test_sweep_branches_skips_close_pairs():
    """A strong mode split into a close pair (0.2 % apart) and a weaker
    distant mode: with a 2 % minimum separation the two branches are the
    strong mode and the distant one."""
    dt = 4e-15
    t = np.arange(12000) * dt
    x = (1.0 * np.cos(2 * np.pi * 41.8e9 * t) + 0.8 * np.cos(2 * np.pi * 41.9e9 * t + 0.3)
         + 0.05 * np.cos(2 * np.pi * 29.1e9 * t + 1.0))
    br = S.sweep_branches([x], dt, 2, fmin=1e9, min_separation=0.02, max_rows=512)[0]
    # the unresolved pair (a 0.005-cycle beat over the trace) costs ESPRIT
    # some accuracy; what is checked is which modes are taken
    assert br[0] == pytest.approx(29.1e9, rel=1e-3)
    assert br[1] == pytest.approx(41.8e9, rel=3e-3)
