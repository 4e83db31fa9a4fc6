"""Full-size parity on the large single-GPU layout (1536 x 768 x 384 cells,
453 M cells) by light cones.

After T steps a value depends only on inputs within a bounded distance: one
cell per full step through the curl stencils, and a few more per step inside
a film (the transverse field averages and their curls).  So the oracle is run
on a box cropped around a sample point, with its own walls far enough away
that they cannot reach the compared core within T steps, and the core is
compared with the same region read back from the full-size GPU run.
"""
import os

import numpy as np
import pytest

import oracle.oracle as O
from paper_2510_22221_amd import mpx
from synth import workloads as W
from tests.parity import rel

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)
T = 10
REACH = 5            # cells per full step, upper bound inside films
R = REACH * T + 8    # half-width of the cropped oracle box
RC = 6               # half-width of the compared core


def say(msg):
    print(msg, flush=True)


def crop(w, center):
    lo = [c - R for c in center]
    n = [2 * R + 1] * 3
    ids = w.ids[lo[2]:lo[2] + n[2], lo[1]:lo[1] + n[1], lo[0]:lo[0] + n[0]].copy()
    sub = W.Workload(f"crop of {w.name} at {center}", n[0], n[1], n[2], w.d, w.dt, w.courant,
                     materials=w.materials, ids=ids, H0=w.H0, m_dir=w.m_dir, nsteps=w.nsteps)
    for s in w.sources:
        b = list(s.box)
        out = []
        for a in range(3):
            a0 = max(b[a], lo[a])
            a1 = min(b[a] + b[3 + a], lo[a] + n[a])
            out.append((a0 - lo[a], max(0, a1 - a0)))
        if all(m > 0 for _, m in out):
            sub.sources.append(W.Source(s.comp, (out[0][0], out[1][0], out[2][0], out[0][1], out[1][1], out[2][1]),
                                        s.table))
    return sub, lo


# film centre, film corner next to the layout's own source, a corner of the
# random-permittivity blocks, the edge of another film
CENTERS = [(192, 192, 194), (92, 172, 194), (900, 400, 150), (1000, 560, 196)]


@pytest.fixture(scope="module")
def c5():
    w = W.c5(T)
    # a point source at every sample centre so that its light cone carries
    # signal within T steps (all other inputs are the layout's own)
    tab = 3e11 * np.sin(0.9 * np.arange(T) + 0.3)
    for ctr in CENTERS:
        w.sources.append(W.Source(2, (ctr[0], ctr[1], ctr[2], 1, 1, 1), tab))
    return w


@pytest.mark.parametrize("prec", [mpx.F32, mpx.F64])
def test_c5_full_size_light_cone(c5, prec):
    w = c5
    # the compared points must be far from the PML (the crop has PEC walls)
    for ctr in CENTERS:
        for a, n in enumerate((w.nx, w.ny, w.nz)):
            assert R + 16 < ctr[a] < n - 16 - R
    say(f"C5 full size {w.nx}x{w.ny}x{w.nz}, {T} steps, prec={prec}: setup")
    g = mpx.from_workload(w, precision=prec)
    assert g.info()["films"] == 8
    g.step(T)
    g.sync()
    tol = 1e-11 if prec == mpx.F64 else 1e-4
    for ctr in CENTERS:
        sub, lo = crop(w, ctr)
        o = O.from_workload(sub, threads=THREADS)
        o.step(T)
        errs = {}
        for name, fields in (("E", (0, 1, 2)), ("H", (3, 4, 5)), ("dM", (9, 10, 11))):
            a, b = [], []
            for f in fields:
                box = [ctr[0] - RC, ctr[1] - RC, ctr[2] - RC, 2 * RC + 1, 2 * RC + 1, 2 * RC + 1]
                a.append(np.asarray(g.get_region(f, box), dtype=np.float64).ravel())
                full = o.get(f)
                sl = (Ellipsis, slice(R - RC, R + RC + 1), slice(R - RC, R + RC + 1), slice(R - RC, R + RC + 1))
                b.append(full[sl].ravel())
            a, b = np.concatenate(a), np.concatenate(b)
            errs[name] = rel(a, b) if np.linalg.norm(b) > 0 else float(np.linalg.norm(a))
            if name != "dM":
                assert np.linalg.norm(b) > 0, f"{name} core is all zero at {ctr}"
        say(f"  center {ctr}: {errs}")
        for k, v in errs.items():
            assert v <= tol, (ctr, k, v)
