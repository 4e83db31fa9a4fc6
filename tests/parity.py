"""Helpers for GPU-vs-oracle parity (test infrastructure).

Relative L2 is taken per group, as the parity metric is defined: {E}, {H}
and {M - M0} (M itself would hide errors behind the large M0), plus each
probe trace.
"""
import numpy as np

import oracle.oracle as O
from paper_2510_22221_amd import mpx
from synth import workloads as W

GROUPS = {"E": (0, 1, 2), "H": (3, 4, 5), "dM": (9, 10, 11)}


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


def group_errors(g, o):
    out = {}
    for name, fields in GROUPS.items():
        a = np.concatenate([np.asarray(g.get(f), dtype=np.float64).ravel() for f in fields])
        b = np.concatenate([o.get(f).ravel() for f in fields])
        out[name] = rel(a, b)
    return out


def probe_errors(g, o, w, f64=True):
    out = []
    for pid, p in enumerate(w.probes):
        nval = 3 if p.kind == "mean_m" else 1
        a = g.read_probe(pid, nval)
        b = o.read_probe(pid, nval)
        if p.kind == "mean_m":
            # The film average is ~Ms, so its relative L2 is dominated by the
            # offset; also bound the absolute difference, which is limited by
            # the summation order of the film sum (~1 ulp of Ms).
            if f64:
                scale = float(np.abs(b).max())
                assert float(np.abs(a - b).max()) <= 1e-14 * scale, "mean-M probe"
        out.append(rel(a, b))
    return out


def run_pair(w, nsteps, precision=mpx.F64, graph_steps=None, threads=None, chunks=1):
    o = O.from_workload(w, threads=threads)
    g = mpx.from_workload(w, precision=precision, graph_steps=graph_steps)
    per = nsteps // chunks
    done = 0
    for c in range(chunks):
        n = per if c < chunks - 1 else nsteps - done
        g.step(n)
        o.step(n)
        done += n
    g.sync()
    return g, o


def many_materials_case(nsteps):
    """150 lossy dielectrics and one PEC id on random cells: far more distinct
    triples of edge coefficients than free class ids, so the most frequent
    triples get compound classes (the table path) and the remaining mixed
    slots go through the mixed-slot kernel with their triple's entry of the
    extended table."""
    w = W.random_case(8, nx=40, ny=17, nz=13, bc=(W.PML,) * 6, npml=(3,) * 6, film=False, nsteps=nsteps)
    rng = np.random.default_rng(8)
    mats = [(float(rng.uniform(1.0, 12.0)), float(rng.uniform(0.0, 5e3)), 0, 0.0, 0.0, 0.0) for _ in range(150)]
    mats[7] = W.PEC_METAL
    w.materials = mats
    w.ids = rng.integers(0, 150, size=(w.nz, w.ny, w.nx)).astype(np.uint8)
    return w


def drive_film(w, nsteps, amp=2e11):
    """Adds two point currents just above the centre of the workload's
    topmost film layer (cells of material 3), so that the film's
    magnetisation moves within a short run; returns w."""
    k_top = int(np.nonzero((w.ids == 3).any(axis=(1, 2)))[0].max())
    ys, xs = np.nonzero(w.ids[k_top] == 3)
    ctr = (int(xs.mean()), int(ys.mean()), k_top + 1)
    tab = amp * np.sin(0.7 * np.arange(nsteps) + 0.2)
    w.sources.append(W.Source(0, (ctr[0], ctr[1], ctr[2], 1, 1, 1), tab))
    w.sources.append(W.Source(1, (ctr[0] + 3, ctr[1] - 2, ctr[2], 1, 1, 1), -0.6 * tab))
    return w
