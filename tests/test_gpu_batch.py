"""Batched stepping of a bias sweep (several simulations per launch).

Each member of a batch must end bitwise equal to the same simulation stepped
alone with the same tile variant and z-chunk: the batched kernels run the
single-instance bodies on a work list, so not one rounding may differ.  The
members differ in grid size, bias and boundary conditions, one has no film
(its step counter advances by the tick kernel), and the batch is stepped in
several calls (odd and even step counts, through captured graphs and direct
launches).  The members of one batch are also compared with the FP64
oracle directly (two resonator instances of the sweep with their films
driven, and a member with overflowing coefficient classes).
"""
import numpy as np
import pytest

import oracle.oracle as O
from paper_2510_22221_amd import mpx
from synth import workloads as W
from tests.parity import drive_film, group_errors, many_materials_case, probe_errors

pytestmark = pytest.mark.gpu
CALLS = (7, 12, 1, 5)


def say(msg):
    print(msg, flush=True)


def members(nsteps):
    ws = [W.c3_instance(80, 64, 48, 0.9, nsteps),
          W.c3_instance(64, 80, 40, 1.15, nsteps),
          W.random_case(5, nx=37, ny=21, nz=19, bc=(W.PML,) * 6, npml=(4,) * 6, film=False, nsteps=nsteps),
          W.random_case(6, nx=29, ny=17, nz=23, bc=(W.PERIODIC, W.PERIODIC, W.PEC, W.PEC, W.PML, W.PML),
                        npml=(0, 0, 0, 0, 4, 4), nsteps=nsteps)]
    return ws


def state(sim, w):
    out = [sim.get(f).copy() for f in range(12)]
    for pid, p in enumerate(w.probes):
        out.append(sim.read_probe(pid, 3 if p.kind == "mean_m" else 1).copy())
    out.append(np.array([sim.info()["step"]]))
    return out


@pytest.mark.parametrize("prec,variant,kchunk", [(mpx.F64, 0, 16), (mpx.F32, 0, 16), (mpx.F64, 1, 16),
                                                 (mpx.F32, 1, 16), (mpx.F64, 2, 5), (mpx.F32, 3, 7)])
def test_batch_bitwise_equals_single(prec, variant, kchunk):
    nsteps = sum(CALLS) + 2
    ws = members(nsteps)
    say(f"batch of {len(ws)}, prec={prec}, variant={variant}, kchunk={kchunk}: single runs")
    ref = []
    for w in ws:
        s = mpx.from_workload(w, precision=prec, fused=variant, kchunk=kchunk, graph_steps=4)
        for n in CALLS:
            s.step(n)
        s.sync()
        ref.append(state(s, w))
        s.close()
    say("  batched run")
    sims = [mpx.from_workload(w, precision=prec) for w in ws]
    b = mpx.Batch(sims)
    b.set_schedule(variant, kchunk)
    b.set_graph_steps(4)
    for n in CALLS:
        b.step(n)
    b.sync()
    for q, (s, w) in enumerate(zip(sims, ws)):
        got = state(s, w)
        for k, (a, r) in enumerate(zip(got, ref[q])):
            assert a.shape == r.shape, (q, k)
            assert np.array_equal(a, r), (q, k, float(np.max(np.abs(a.astype(np.float64) - r))))
    b.close()
    for s in sims:
        s.close()


def test_batch_members_step_alone_between_calls():
    """A member stepped on its own between batch calls (changing its buffer
    parity) continues correctly in the batch."""
    ws = members(40)[:2]
    ref = []
    for w in ws:
        s = mpx.from_workload(w, precision=mpx.F64)
        s.step(6)
        s.step(3)
        s.step(6)
        s.sync()
        ref.append(state(s, w))
    sims = [mpx.from_workload(w, precision=mpx.F64) for w in ws]
    b = mpx.Batch(sims)
    b.set_graph_steps(4)
    b.step(6)
    sims[0].step(3)
    sims[1].step(3)
    b.step(6)
    b.sync()
    for q, (s, w) in enumerate(zip(sims, ws)):
        for k, (a, r) in enumerate(zip(state(s, w), ref[q])):
            assert np.array_equal(a, r), (q, k)


def test_batch_rejects_bad_members():
    w = W.random_case(7, nsteps=4)
    a = mpx.from_workload(w, precision=mpx.F64)
    c = mpx.from_workload(w, precision=mpx.F32)
    with pytest.raises(mpx.MpxError):
        mpx.Batch([a, c])
    with pytest.raises(mpx.MpxError):
        mpx.Batch([a, a])
    with pytest.raises(mpx.MpxError):
        mpx.Batch([])


@pytest.mark.parametrize("prec", [mpx.F64, mpx.F32])
def test_batch_member_with_mixed_slots(prec):
    """A member whose mixed slots overflow the class table (150 materials:
    its slots take the extended table inside the E pass) beside one without
    any: the batch gives the single-run bits."""
    nsteps = sum(CALLS) + 2
    ws = [many_materials_case(nsteps), W.c3_instance(64, 48, 40, 1.0, nsteps)]
    ref = []
    for w in ws:
        s = mpx.from_workload(w, precision=prec, graph_steps=4)
        for n in CALLS:
            s.step(n)
        s.sync()
        ref.append(state(s, w))
        s.close()
    sims = [mpx.from_workload(w, precision=prec) for w in ws]
    b = mpx.Batch(sims)
    b.set_graph_steps(4)
    for n in CALLS:
        b.step(n)
    b.sync()
    for q, (s, w) in enumerate(zip(sims, ws)):
        for k, (a, r) in enumerate(zip(state(s, w), ref[q])):
            assert np.array_equal(a, r), (q, k)
    b.close()
    for s in sims:
        s.close()


@pytest.mark.parametrize("prec,tol", [(mpx.F64, 1e-11), (mpx.F32, 1e-4)])
def test_batch_members_match_oracle(prec, tol):
    """Two instances of the bias sweep (uneven sizes, biases 0.9 and 1.15 of
    the anti-crossing field, films driven by a point current so that M moves)
    and the 150-material member, stepped as one batch in several calls: each
    member against the FP64 oracle, element by element (E, H, M - M0 and
    the probes)."""
    nsteps = sum(CALLS) + 8
    ws = [drive_film(W.c3_instance(80, 64, 48, 0.9, nsteps), nsteps),
          drive_film(W.c3_instance(64, 80, 40, 1.15, nsteps), nsteps),
          many_materials_case(nsteps)]
    say(f"batch of {len(ws)} against the oracle, prec={prec}")
    sims = [mpx.from_workload(w, precision=prec) for w in ws]
    b = mpx.Batch(sims)
    b.set_graph_steps(4)
    done = 0
    for n in CALLS + (8,):
        b.step(n)
        done += n
    b.sync()
    for q, (s, w) in enumerate(zip(sims, ws)):
        o = O.from_workload(w, threads=16)
        o.step(done)
        if q < 2:
            dm = np.concatenate([o.get(f).ravel() for f in (9, 10, 11)])
            assert np.abs(dm).max() > 1e-3, q
        errs = group_errors(s, o)
        perr = probe_errors(s, o, w, f64=tol < 1e-9)
        say(f"  member {q}: {errs} probes max {max(perr) if perr else 0:.2e}")
        for k, v in errs.items():
            assert v <= tol, (q, k, v)
        for v in perr:
            assert v <= tol, q
    b.close()
    for s in sims:
        s.close()


@pytest.mark.parametrize("prec", [mpx.F64, mpx.F32])
def test_every_tuning_candidate_gives_the_same_bits(prec):
    """The autotuner may pick any of its candidates (the separate passes or
    a fused variant with a z-chunk): each gives the batch the same bits, so
    the choice changes speed only."""
    from paper_2510_22221_amd import tune
    nsteps = 2 * 11 + 2
    ws = members(nsteps)[:3]
    ref = None
    for v, kc in tune.candidates(max(w.nz for w in ws)):
        say(f"tuning candidate variant {v} z-chunk {kc}, prec={prec}")
        sims = [mpx.from_workload(w, precision=prec) for w in ws]
        b = mpx.Batch(sims)
        b.set_schedule(v, kc)
        b.set_graph_steps(4)
        b.step(11)
        b.step(11)
        b.sync()
        got = [state(s, w) for s, w in zip(sims, ws)]
        b.close()
        for s in sims:
            s.close()
        if ref is None:
            ref = got
            continue
        for q in range(len(ws)):
            for k, (a, r) in enumerate(zip(got[q], ref[q])):
                assert np.array_equal(a, r), (v, kc, q, k)
