"""The no-allocation energy entry point (mpx_energy_noalloc) gives the bits
of mpx_energy, through the C ABI, on two calls in a row (the second on a
smaller grid, so it reads less of the shared scratch than the first wrote),
in both precisions."""
import numpy as np
import pytest

from paper_2510_22221_amd import mpx
from synth import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("prec", [mpx.F64, mpx.F32])
def test_energy_noalloc_matches_energy(prec):
    big = W.c1(40)                                   # 32^3 with a film
    small = W.random_case(3, nx=13, ny=11, nz=9, nsteps=20)
    out = []
    for name, w, n in (("32^3 film box", big, 40), ("13x11x9 random box", small, 20)):
        say(f"energy_noalloc on {name}, prec={prec}")
        g = mpx.from_workload(w, precision=prec)
        g.step(n)
        g.sync()
        a = g.energy_noalloc()
        b = g.energy()
        c = g.energy_noalloc()
        say(f"  noalloc {a} energy {b}")
        assert a == b and c == b, (name, a, b, c)
        assert b[0] > 0 and np.isfinite(b).all()
        out.append(a)
        g.close()
    assert out[0] != out[1]
