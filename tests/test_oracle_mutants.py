"""The pins can fail: plausible mistakes planted in copies of the C oracle
(built into a temporary directory, on the CPU) must each be caught by the
pin that guards that part of the scheme.  Nothing here touches the GPU path.
"""
import importlib.util
import os
import subprocess

import numpy as np
import pytest

import oracle.oracle as O
from tests import test_oracle_pins as P

SRC = os.path.join(os.path.dirname(O.__file__), "mpx_oracle.c")


def mutant(tmp_path, name, old, new):
    """A copy of the oracle's ctypes wrapper bound to a copy of the C source
    with `old` replaced by `new` (which must occur exactly once)."""
    src = open(SRC).read()
    assert src.count(old) == 1, old
    c = tmp_path / f"{name}.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-o", str(so), str(c), "-lm"])
    spec = importlib.util.spec_from_file_location(f"oracle_mutant_{name}", O.__file__)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.LIB_PATH = str(so)
    mod._lib = None
    return mod


@pytest.mark.parametrize("name,old,new", [
    # the H-type CPML recursion with the full step instead of the half step
    ("cpml_h_dt", "double b = exp(-sig * (0.5 * g->dt) / ORC_EPS0);", "double b = exp(-sig * g->dt / ORC_EPS0);"),
    # the H-type grading sampled at the E positions
    ("cpml_h_pos", "double x = p + 0.5 * half;", "double x = p;"),
])
def test_t12_catches_cpml_mistakes(tmp_path, t12_reference, name, old, new):
    M = mutant(tmp_path, name, old, new)
    a = P.t12_run(M, 50, 16, P.t12_probes(50, 16))
    b = t12_reference[16]
    worst = max(P.rel(a[p], b[p]) for p in range(3))
    assert worst > 1e-3, worst


t12_reference = P.t12_reference


@pytest.mark.parametrize("name,old,new", [
    ("edge_weight", "we += e2 / 4.0;", "we += e2 / 2.0;"),
    ("face_weight", "wh += h2 / 2.0;", "wh += h2;"),
])
def test_film_energy_pins_catch_weight_mistakes(tmp_path, name, old, new):
    M = mutant(tmp_path, name, old, new)
    # the uniform-field closed form, run against the mutant
    s, w = P._film_energy_sim((P.W.PERIODIC,) * 6, (2, 1, 3, 3, 2, 2))
    del s
    w2 = w
    s = M.from_workload(w2)
    s.add_probe(M.PROBE_FILM_ENERGY, film=0, cap=4)
    E, H = (1.3e3, -0.7e3, 2.1e3), (4.0, -9.0, 2.5)
    for c in range(3):
        s.set(c, np.full(s.get(c).shape, E[c]))
        s.set(3 + c, np.full(s.get(3 + c).shape, H[c]))
    s.step(1)
    dV = w.d[0] * w.d[1] * w.d[2]
    want = 12 * dV * (0.5 * P.EPS0 * P.FILM_EPS * sum(e * e for e in E) + 0.5 * P.MU0 * sum(h * h for h in H))
    assert abs(float(s.read_probe(0)[0]) / want - 1) > 1e-3
