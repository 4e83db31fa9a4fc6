"""Pins of the FP64 reverse-mode reference (oracle/reverse.py): its forward
run reproduces the C oracle's loss (two implementations written separately,
one in C loops, one in torch array operations), and its autograd gradients
match central finite differences of the C oracle's loss."""
import numpy as np
import pytest

import oracle.oracle as O
from oracle import fd
from oracle.reverse import Reverse
from synth import workloads as W


@pytest.fixture(autouse=True, scope="module")
def _threads():
    O.build()
    O.set_threads(4)


def small_case(nsteps, seed=21):
    """A 7 x 6 x 6 PEC box: random dielectrics (one lossy), a PEC cell, a
    3 x 2 x 2 film of two magnetic materials, a tilted magnetisation under a
    strong oblique bias and a point current beside the film."""
    w = W.box(7, 6, 6, d=(1.1e-6, 0.9e-6, 1.0e-6), nsteps=nsteps)
    rng = np.random.default_rng(seed)
    w.materials = [W.VACUUM, (4.0, 0.0, 0, 0, 0, 0), W.PEC_METAL, (1.0, 0.0, 0, 1.4e5, 0.02, W.GAMMA),
                   (7.0, 3e3, 0, 0, 0, 0), (2.5, 0.0, 0, 0.9e5, 0.05, 1.9e11)]
    ids = rng.choice([0, 1, 4], size=(6, 6, 7), p=[0.5, 0.3, 0.2]).astype(np.uint8)
    ids[0, 0, 0] = 2
    ids[2:4, 2:4, 2:5] = 3
    ids[2, 2, 4] = 5
    w.ids = ids
    w.H0 = (3e6, -1e6, 5e6)
    w.m_dir = (0.3, 0.2, 1.0)
    w.sources = [W.Source(2, (5, 3, 2, 1, 1, 1), 4e10 * np.sin(0.45 * np.arange(nsteps) + 0.1))]
    return w


EPS_BOX = (1, 1, 1, 4, 3, 2)
MS_BOX = (2, 2, 2, 3, 2, 2)


def film_mask(w):
    return np.isin(w.ids, [3, 5])


def test_forward_loss_matches_c_oracle():
    n, n0 = 40, 15
    w = small_case(n)
    r = Reverse(w, EPS_BOX, MS_BOX)
    L = float(r.run(n, loss="film_energy", loss_from=n0, film_cells=film_mask(w)).detach())
    Lc = fd.loss(w, n, n0)
    assert Lc > 0
    assert abs(L / Lc - 1) < 1e-12, (L, Lc)
    wt = np.cos(0.3 * np.arange(n))
    L2 = float(Reverse(w).run(n, loss="trace", field=0, ijk=(3, 3, 2), weights=wt).detach())
    L2c = fd.trace_loss(w, n, 0, (3, 3, 2), wt)
    assert abs(L2 - L2c) <= 1e-12 * max(abs(L2c), 1e-300) and L2c != 0


def test_gradients_match_c_oracle_finite_differences():
    n, n0 = 40, 15
    w = small_case(n)
    g = Reverse(w, EPS_BOX, MS_BOX).gradients(n, loss="film_energy", loss_from=n0, film_cells=film_mask(w))
    tol = 2e-6
    for c in range(3):
        ref = fd.grad_H0(w, n, n0, c)
        assert abs(g["dH0"][c] - ref) <= tol * np.abs(g["dH0"]).max(), (c, g["dH0"][c], ref)
    # a cell inside the film, one under it and one beside the source
    for (i, j, k) in ((2, 2, 2), (3, 1, 1), (4, 3, 2)):
        a = g["deps"][k - EPS_BOX[2], j - EPS_BOX[1], i - EPS_BOX[0]]
        ref = fd.grad_eps(w, n, n0, (i, j, k))
        assert abs(a - ref) <= tol * np.abs(g["deps"]).max(), ((i, j, k), a, ref)
    for (i, j, k) in ((2, 2, 2), (4, 2, 2), (3, 3, 3)):
        a = g["dMs"][k - MS_BOX[2], j - MS_BOX[1], i - MS_BOX[0]]
        ref = fd.grad_Ms(w, n, n0, (i, j, k))
        assert abs(a - ref) <= tol * np.abs(g["dMs"]).max(), ((i, j, k), a, ref)
