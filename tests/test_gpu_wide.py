"""Grids at least 512 slots wide: the passes run on 256 x 1 tiles, and the
film's second half step shares one launch with the merged H/M pass.

A thin 520-wide box with a film, CPML slabs on the x faces and a source is
checked against the FP64 oracle in both precisions, and a batch holding it
(whose kernels launch the film and H/M work separately) must end bitwise
equal to stepping it alone.
"""
import os

import numpy as np
import pytest

import oracle.oracle as O
from paper_2510_22221_amd import mpx
from synth import workloads as W
from tests.parity import group_errors, rel, run_pair

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)
CALLS = (7, 12, 1, 5)


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _libs():
    O.build()
    mpx.load()


def wide_case(nsteps):
    w = W.random_case(41, nx=520, ny=12, nz=10, bc=(W.PML, W.PML, W.PEC, W.PEC, W.PEC, W.PEC),
                      npml=(2, 2, 0, 0, 0, 0), nsteps=nsteps)
    w.H0 = (3e6, 0.0, 5e6)
    w.probes = [W.Probe("field", 1, (260, 6, 5)), W.Probe("mean_m", film=0), W.Probe("film_energy", film=0)]
    return w


@pytest.mark.parametrize("prec,tol", [(mpx.F64, 1e-11), (mpx.F32, 1e-4)])
def test_wide_grid_matches_oracle(prec, tol):
    n = 30
    w = wide_case(n)
    say(f"520-wide box, film, x CPML, {n} steps prec={prec}")
    g, o = run_pair(w, n, prec, threads=THREADS, chunks=3)
    errs = group_errors(g, o)
    say(f"  groups {errs}")
    for k, v in errs.items():
        assert v <= tol, (k, v)
    # probes: the field trace and the film energy to the same relative L2;
    # the film-mean M in float64 to the summation-order bound of a mean of
    # n_sum terms of magnitude <= Ms (each partial order rounds differently):
    # n_sum 2^-53 max Ms, n_sum = 2 faces per family and cell, 3 families
    n_mag = int(sum(np.count_nonzero(w.ids == m) for m, mat in enumerate(w.materials) if mat[3] > 0))
    ms_max = max(mat[3] for mat in w.materials)
    for pid, p in enumerate(w.probes):
        nval = 3 if p.kind == "mean_m" else 1
        a, b = g.read_probe(pid, nval), o.read_probe(pid, nval)
        if p.kind == "mean_m" and prec == mpx.F64:
            bound = 6 * n_mag * 2.0 ** -53 * ms_max
            say(f"  mean M: max |diff| {float(np.abs(a - b).max()):.3e} (bound {bound:.3e})")
            assert float(np.abs(a - b).max()) <= bound
        else:
            e = rel(np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel())
            say(f"  {p.kind}: rel L2 {e:.2e}")
            assert e <= tol, p.kind


def state(sim, w):
    out = [sim.get(f).copy() for f in range(12)]
    for pid, p in enumerate(w.probes):
        out.append(sim.read_probe(pid, 3 if p.kind == "mean_m" else 1).copy())
    return out


@pytest.mark.parametrize("prec", [mpx.F64, mpx.F32])
def test_wide_member_of_a_batch_bitwise(prec):
    n = sum(CALLS) + 2
    ws = [wide_case(n), W.c3_instance(64, 40, 32, 1.05, n)]
    ref = []
    for w in ws:
        s = mpx.from_workload(w, precision=prec, graph_steps=4)
        for c in CALLS:
            s.step(c)
        s.sync()
        ref.append(state(s, w))
        s.close()
    sims = [mpx.from_workload(w, precision=prec) for w in ws]
    b = mpx.Batch(sims)
    b.set_graph_steps(4)
    for c in CALLS:
        b.step(c)
    b.sync()
    for q, (s, w) in enumerate(zip(sims, ws)):
        for k, (a, r) in enumerate(zip(state(s, w), ref[q])):
            assert np.array_equal(a, r), (q, k)
    b.close()
    for s in sims:
        s.close()


def test_narrow_tile_schedule_bitwise_equal_wide_tiles():
    """Schedule 6 (the separate passes on 64 x 4 tiles, the film's second
    half step as its own launch) gives the 520-wide box the bits of the
    256 x 1 tiles in both precisions."""
    w = wide_case(26)
    for prec in (mpx.F64, mpx.F32):
        say(f"64 x 4 tiles on the 520-wide box, prec={prec}")
        ref = mpx.from_workload(w, precision=prec)
        ref.step(13)
        ref.step(13)
        g = mpx.from_workload(w, precision=prec, fused=6)
        g.step(13)
        g.step(13)
        for f in range(12):
            assert np.array_equal(g.get(f), ref.get(f)), (prec, f)
        for pid, p in enumerate(w.probes):
            nv = 3 if p.kind == "mean_m" else 1
            assert np.array_equal(g.read_probe(pid, nv), ref.read_probe(pid, nv)), (prec, pid)


def test_probes_in_the_h_pass_launch_bitwise():
    """E-point and mean-M probes, strided ones among them, ride in the merged
    H/M launch on wide grids (its probe block reads the step counter and
    advances it). One H-point probe more sends every probe back to the probe
    launch. Both runs must give the same fields, traces and step counter in
    both precisions."""
    w = wide_case(40)
    w.probes = []
    for prec in (mpx.F64, mpx.F32):
        runs = []
        for with_h in (False, True):
            say(f"520-wide box, E and mean-M probes{' + an H probe' if with_h else ''}, prec={prec}")
            s = mpx.from_workload(w, precision=prec, graph_steps=4)
            spec = [(mpx.PROBE_FIELD, 1, (260, 6, 5), 1), (mpx.PROBE_MEAN_M, 0, None, 1),
                    (mpx.PROBE_FIELD, 2, (100, 5, 4), 3), (mpx.PROBE_MEAN_M, 0, None, 4)]
            pids = []
            for kind, fld, ijk, every in spec:
                if kind == mpx.PROBE_MEAN_M:
                    pids.append((s.add_probe(kind, film=0, cap=64, every=every), 3))
                else:
                    pids.append((s.add_probe(kind, field=fld, ijk=ijk, cap=64, every=every), 1))
            if with_h:
                s.add_probe(mpx.PROBE_FIELD, field=4, ijk=(259, 6, 5), cap=64)
            for c in CALLS:
                s.step(c)
            s.sync()
            runs.append(([s.get(f).copy() for f in range(12)],
                         [s.read_probe(pid, nv).copy() for pid, nv in pids], s.info()["step"]))
            s.close()
        (fa, pa, sa), (fb, pb, sb) = runs
        assert sa == sb == sum(CALLS), (sa, sb)
        for f in range(12):
            assert np.array_equal(fa[f], fb[f]), (prec, f)
        for q, (a, b) in enumerate(zip(pa, pb)):
            assert a.shape == b.shape and a.size > 0, (prec, q, a.shape, b.shape)
            assert np.array_equal(a, b), (prec, q)
        assert np.any(pa[1] != 0.0), "mean M never sampled"
