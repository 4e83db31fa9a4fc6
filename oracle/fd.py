"""Two losses of a workload on the FP64 oracle and their central finite
differences (TEST INFRASTRUCTURE ONLY: the reference the adjoint gradients
are checked against; shares no code with the HIP library).

Film energy: L = dt * sum over steps n = loss_from+1 .. nsteps of W_f(n),
W_f the film EM energy the oracle's film-energy probe records at integer
time n.  Weighted trace: L = sum_i weights[i] * E_c(i, j, k) after step
i+1, the oracle's field probe record dotted with a weight sequence.
Parameters: the bias H0 (component w), eps_r of one cell, Ms of one cell
(each perturbed cell gets a material of its own).
"""
from __future__ import annotations

import copy

import numpy as np

from . import oracle as O


def loss(w, nsteps: int, loss_from: int, film: int = 0, threads=None) -> float:
    w = copy.copy(w)
    w.probes = []
    s = O.from_workload(w, threads=threads)
    pid = s.add_probe(O.PROBE_FILM_ENERGY, film=film, cap=nsteps)
    s.step(nsteps)
    tr = np.asarray(s.read_probe(pid, 1), dtype=np.float64).ravel()
    return float(w.dt * tr[loss_from:nsteps].sum())


def trace_loss(w, nsteps: int, field: int, ijk, weights, threads=None) -> float:
    w = copy.copy(w)
    w.probes = []
    s = O.from_workload(w, threads=threads)
    pid = s.add_probe(O.PROBE_FIELD, field=field, ijk=tuple(ijk), cap=nsteps)
    s.step(nsteps)
    tr = np.asarray(s.read_probe(pid, 1), dtype=np.float64).ravel()
    return float(np.dot(np.asarray(weights, dtype=np.float64), tr[:nsteps]))


def _with_cell_material(w, cell, **change):
    """A copy of w whose cell (i, j, k) has a material of its own: the cell's
    material with the given fields changed (eps_r, Ms)."""
    w2 = copy.copy(w)
    w2.ids = w.ids.copy()
    mats = list(w.materials)
    i, j, k = cell
    m = list(mats[int(w.ids[k, j, i])])
    if "eps_r" in change:
        m[0] = change["eps_r"]
    if "Ms" in change:
        m[3] = change["Ms"]
    mats.append(tuple(m))
    w2.materials = mats
    w2.ids[k, j, i] = len(mats) - 1
    return w2


def derivative(f, h: float) -> float:
    """f'(0) by Richardson extrapolation of central differences at steps h and
    h/2: (4 D(h/2) - D(h)) / 3, which cancels the h^2 error term.

    The step cannot be made arbitrarily small: the loss carries a rounding
    noise of some 1e-16..1e-15 of its value (every field value rounds
    differently once a parameter changes), and a central difference divides
    that by 2h.  Steps of 1e-3 of the parameter keep that noise near 1e-7 of
    the derivative on the small cases, and the extrapolation keeps the
    truncation error below it."""
    def central(s):
        return (f(s) - f(-s)) / (2 * s)
    return (4.0 * central(h / 2) - central(h)) / 3.0


def grad_H0(w, nsteps, loss_from, comp, rel=2e-3, film=0, threads=None) -> float:
    return grad_H0_of(lambda w2: loss(w2, nsteps, loss_from, film, threads), w, comp, rel)


def grad_eps(w, nsteps, loss_from, cell, rel=2e-3, film=0, threads=None) -> float:
    return grad_eps_of(lambda w2: loss(w2, nsteps, loss_from, film, threads), w, cell, rel)


def grad_Ms(w, nsteps, loss_from, cell, rel=2e-3, film=0, threads=None) -> float:
    return grad_Ms_of(lambda w2: loss(w2, nsteps, loss_from, film, threads), w, cell, rel)


# the same derivatives of any loss f(workload) -> float


def grad_H0_of(f, w, comp, rel=2e-3) -> float:
    h = rel * max(abs(v) for v in w.H0)

    def g(d):
        w2 = copy.copy(w)
        H0 = list(w.H0)
        H0[comp] += d
        w2.H0 = tuple(H0)
        return f(w2)
    return derivative(g, h)


def grad_eps_of(f, w, cell, rel=2e-3) -> float:
    i, j, k = cell
    e0 = w.materials[int(w.ids[k, j, i])][0]
    return derivative(lambda d: f(_with_cell_material(w, cell, eps_r=e0 + d)), rel * e0)


def grad_Ms_of(f, w, cell, rel=2e-3) -> float:
    i, j, k = cell
    m0 = w.materials[int(w.ids[k, j, i])][3]
    return derivative(lambda d: f(_with_cell_material(w, cell, Ms=m0 + d)), rel * m0)
