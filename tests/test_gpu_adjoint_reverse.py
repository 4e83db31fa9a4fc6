"""The discrete adjoint (mpx_adjoint, mpx_adjoint_probe) against the FP64
reverse-mode reference (oracle/reverse.py: torch autograd over a separately
written float64 implementation of the step), element by element: the
gradient with respect to H0 and to eps_r and Ms of every cell of the grid.

Float64: within 1e-10 of the largest gradient of each group.  Float32 (the
forward and reverse passes in float32, the magnetisation and the gradient
sums in float64): within 1e-5 of the largest gradient of each group."""
import numpy as np
import pytest

from oracle.reverse import Reverse
from paper_2510_22221_amd import mpx
from tests.test_oracle_reverse import film_mask, small_case

pytestmark = pytest.mark.gpu
TOL = {mpx.F64: 1e-10, mpx.F32: 1e-5}


def say(msg):
    print(msg, flush=True)


def compare(res, ref, tol, what):
    for key in ("dH0", "deps", "dMs"):
        a, b = np.asarray(res[key]), np.asarray(ref[key])
        assert a.shape == b.shape, (what, key)
        scale = float(np.abs(b).max())
        err = float(np.abs(a - b).max())
        say(f"  {what} {key}: max |ref| {scale:.3e}, max |diff| / max |ref| {err / scale:.2e}")
        assert scale > 0, (what, key)
        assert err <= tol * scale, (what, key, err / scale)


@pytest.mark.parametrize("prec", [mpx.F64, mpx.F32])
@pytest.mark.parametrize("n,n0,cp,sched", [(40, 15, 0, 0), (41, 0, 6, 0), (33, 9, 5, 1)])
def test_adjoint_film_energy_matches_reverse_mode(prec, n, n0, cp, sched):
    """Every cell of the grid is a parameter (film cells too: the loss reads
    their eps_r itself), under the tape schedule (one or several checkpoint
    segments) and the plain one."""
    w = small_case(n)
    box = (0, 0, 0, w.nx, w.ny, w.nz)
    say(f"adjoint vs reverse mode: {n} steps, loss from {n0}, checkpoints {cp}, schedule {sched}, prec={prec}")
    g = mpx.from_workload(w, precision=prec)
    g.set_adjoint_schedule(sched)
    res = g.adjoint(n, n0, film=0, checkpoint_every=cp, eps_box=box, ms_box=box)
    g.close()
    ref = Reverse(w, box, box).gradients(n, loss="film_energy", loss_from=n0, film_cells=film_mask(w))
    assert abs(res["loss"] / ref["loss"] - 1) < (1e-12 if prec == mpx.F64 else 1e-4)
    compare(res, ref, TOL[prec], "film energy")


@pytest.mark.parametrize("prec", [mpx.F64, mpx.F32])
def test_adjoint_probe_matches_reverse_mode(prec):
    n = 37
    w = small_case(n, seed=23)
    box = (0, 0, 0, w.nx, w.ny, w.nz)
    wt = np.cos(0.21 * np.arange(n)) * np.exp(-np.arange(n) / 30.0)
    ijk = (3, 4, 2)
    say(f"adjoint_probe vs reverse mode: {n} steps, E_y at {ijk}, prec={prec}")
    g = mpx.from_workload(w, precision=prec)
    res = g.adjoint_probe(n, 1, ijk, wt, checkpoint_every=5, eps_box=box, ms_box=box)
    g.close()
    ref = Reverse(w, box, box).gradients(n, loss="trace", field=1, ijk=ijk, weights=wt)
    assert abs(res["loss"] - ref["loss"]) <= (1e-12 if prec == mpx.F64 else 1e-4) * abs(ref["loss"])
    compare(res, ref, TOL[prec], "trace")
