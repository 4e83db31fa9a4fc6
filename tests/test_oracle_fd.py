"""CPU pins of the finite-difference helpers the adjoint tests rely on, and
of the spectral splitting functional.

* derivative(): Richardson-extrapolated central differences reproduce the
  derivatives of closed forms;
* trace_loss(): the weighted trace with a one-hot weight is the oracle's
  field-probe record at that step, and it is linear in the weights;
* without magnetic cells the bias never enters the fields, so its finite
  difference is exactly zero;
* band_centroid_splitting(): two pure tones on either side of the midpoint
  give their frequency difference.
"""
import math

import numpy as np
import pytest

from oracle import fd
from oracle import oracle as O
from synth import workloads as W


def test_derivative_of_closed_forms():
    assert fd.derivative(lambda d: math.exp(2.0 * d), 1e-3) == pytest.approx(2.0, rel=1e-10)
    assert fd.derivative(lambda d: math.sin(1.0 + d), 1e-3) == pytest.approx(math.cos(1.0), rel=1e-10)
    # a cubic: the h^2 term of the central difference cancels exactly
    assert fd.derivative(lambda d: (0.5 + d) ** 3, 0.1) == pytest.approx(0.75, rel=1e-13)


def small():
    w = W.random_case(21, nx=12, ny=10, nz=9, nsteps=20)
    w.H0 = (3e6, 0.0, 5e6)
    return w


def test_trace_loss_is_the_probe_record_dotted_with_the_weights():
    w = small()
    n, ijk = 20, (5, 4, 3)
    s = O.from_workload(w)
    pid = s.add_probe(O.PROBE_FIELD, field=1, ijk=ijk, cap=n)
    s.step(n)
    tr = np.asarray(s.read_probe(pid, 1), dtype=np.float64).ravel()
    assert tr.shape == (n,) and np.any(tr != 0.0)
    for i in (0, 7, n - 1):
        e = np.zeros(n)
        e[i] = 1.0
        assert fd.trace_loss(w, n, 1, ijk, e) == tr[i]
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal(n), rng.standard_normal(n)
    la, lb = fd.trace_loss(w, n, 1, ijk, a), fd.trace_loss(w, n, 1, ijk, b)
    assert fd.trace_loss(w, n, 1, ijk, a - 2.0 * b) == pytest.approx(la - 2.0 * lb, rel=1e-12, abs=1e-12 * abs(la))


def test_bias_gradient_vanishes_without_a_film():
    w = W.random_case(22, nx=12, ny=10, nz=9, nsteps=20, film=False)
    w.H0 = (1e6, 2e6, 3e6)
    wt = np.random.default_rng(4).standard_normal(20)
    assert fd.trace_loss(w, 20, 0, (6, 5, 4), wt) != 0.0
    for c in range(3):
        assert fd.grad_H0_of(lambda w2: fd.trace_loss(w2, 20, 0, (6, 5, 4), wt), w, c) == 0.0


@pytest.mark.parametrize("f1,f2", [(40.0, 60.0), (45.0, 55.0), (30.0, 72.0)])
def test_band_centroid_splitting_of_two_tones(f1, f2):
    torch = pytest.importorskip("torch")
    from paper_2510_22221_amd import grad as G
    dt, n = 1e-3, 4000
    t = np.arange(1, n + 1) * dt
    x = torch.tensor(np.sin(2 * np.pi * f1 * t) + np.sin(2 * np.pi * f2 * t + 0.3))
    s = G.band_centroid_splitting(x, dt, 0.5 * (f1 + f2), 25.0)
    assert float(s) == pytest.approx(f2 - f1, rel=1e-6)
