"""The grid-energy probe and probe strides.

* The EM-energy probe records, after each step, the discrete energy W_EM the
  FP64 oracle computes at that integer time (the oracle stepped one step at
  a time), and the value mpx_energy returns at the end of a call.
* A probe with stride s holds exactly every s-th sample of the same probe at
  stride 1 (all kinds, ring-buffer wrap, calls of odd lengths through graphs
  and direct launches, batched members).
"""
import numpy as np
import pytest

import oracle.oracle as O
from paper_2510_22221_amd import mpx
from synth import workloads as W

pytestmark = pytest.mark.gpu
CALLS = (7, 12, 1, 17)


def say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("prec,tol", [(mpx.F64, 1e-12), (mpx.F32, 1e-4)])
def test_em_energy_probe_matches_oracle(prec, tol):
    w = W.c1(60)
    n = 60
    say(f"EM energy probe, C1 {n} steps prec={prec}")
    g = mpx.from_workload(w, precision=prec)
    pid = g.add_probe(mpx.PROBE_EM_ENERGY, cap=n)
    g.step(n)
    tr = g.read_probe(pid, 1).ravel()
    o = O.from_workload(w)
    ref = []
    for _ in range(n):
        o.step(1)
        ref.append(o.energy()[0])
    ref = np.array(ref)
    assert tr.shape == (n,)
    err = np.max(np.abs(tr - ref)) / np.max(np.abs(ref))
    say(f"  max |probe - oracle| / max W = {err:.2e}")
    assert err <= tol


def test_em_energy_probe_equals_mpx_energy():
    w = W.c1(40)
    g = mpx.from_workload(w, precision=mpx.F64)
    pid = g.add_probe(mpx.PROBE_EM_ENERGY, cap=64)
    done = 0
    for n in (5, 13, 1):
        g.step(n)
        done += n
        tr = g.read_probe(pid, 1).ravel()
        assert tr.shape == (done,)
        assert tr[-1] == pytest.approx(g.energy()[0], rel=1e-13)


def test_em_energy_probe_periodic_box():
    """Periodic x and y (the energy sums wrap), PEC z, random media and a
    film: the probe after each step against the oracle's energy, and
    mpx_energy at the end."""
    n = 30
    w = W.random_case(34, nx=20, ny=16, nz=12, bc=(W.PERIODIC, W.PERIODIC, W.PERIODIC, W.PERIODIC, W.PEC, W.PEC),
                      nsteps=n)
    w.probes = []
    g = mpx.from_workload(w, precision=mpx.F64)
    pid = g.add_probe(mpx.PROBE_EM_ENERGY, cap=n, every=2)
    g.step(n)
    tr = g.read_probe(pid, 1).ravel()
    o = O.from_workload(w)
    ref = []
    for _ in range(n // 2):
        o.step(2)
        ref.append(o.energy()[0])
    ref = np.array(ref)
    assert tr.shape == ref.shape
    err = np.max(np.abs(tr - ref)) / np.max(np.abs(ref))
    say(f"periodic box: max |probe - oracle| / max W = {err:.2e}")
    assert err <= 1e-12
    assert g.energy()[0] == pytest.approx(o.energy()[0], rel=1e-12)


def stride_case(nsteps):
    w = W.random_case(31, nx=24, ny=18, nz=16, bc=(W.PEC,) * 6, npml=(0,) * 6, nsteps=nsteps)
    w.H0 = (3e6, 0.0, 5e6)
    w.probes = []
    return w


def add_all(s, every, cap):
    return [s.add_probe(mpx.PROBE_FIELD, field=1, ijk=(9, 7, 6), cap=cap, every=every),
            s.add_probe(mpx.PROBE_FIELD, field=5, ijk=(10, 8, 7), cap=cap, every=every),
            s.add_probe(mpx.PROBE_MEAN_M, film=0, cap=cap, every=every),
            s.add_probe(mpx.PROBE_FILM_ENERGY, film=0, cap=cap, every=every),
            s.add_probe(mpx.PROBE_EM_ENERGY, cap=cap, every=every)]


NVAL = (1, 1, 3, 1, 1)


@pytest.mark.parametrize("prec", [mpx.F64, mpx.F32])
def test_probe_stride_subsamples_bitwise(prec):
    n = sum(CALLS)
    w = stride_case(n)
    say(f"probe strides prec={prec}")
    s = mpx.from_workload(w, precision=prec, graph_steps=4)
    ref = add_all(s, 1, n)
    st3 = add_all(s, 3, n)
    st5 = add_all(s, 5, 2)  # wraps: the last two samples stay
    for c in CALLS:
        s.step(c)
    for q in range(5):
        r = s.read_probe(ref[q], NVAL[q]).reshape(n, NVAL[q])
        assert np.any(r != 0.0), q
        a = s.read_probe(st3[q], NVAL[q]).reshape(-1, NVAL[q])
        assert np.array_equal(a, r[2::3]), q
        b = s.read_probe(st5[q], NVAL[q]).reshape(-1, NVAL[q])
        assert np.array_equal(b, r[4::5][-2:]), q
    s.close()


def test_probe_stride_in_a_batch():
    n = sum(CALLS)
    ws = [stride_case(n), W.random_case(32, nx=20, ny=22, nz=14,
                                        bc=(W.PERIODIC, W.PERIODIC, W.PEC, W.PEC, W.PEC, W.PEC),
                                        npml=(0,) * 6, nsteps=n)]
    ws[1].probes = []
    ref = []
    for w in ws:
        s = mpx.from_workload(w, precision=mpx.F64, graph_steps=4)
        ids = add_all(s, 4, n)
        for c in CALLS:
            s.step(c)
        ref.append([s.read_probe(i, NVAL[q]) for q, i in enumerate(ids)])
        s.close()
    sims = [mpx.from_workload(w, precision=mpx.F64) for w in ws]
    ids = [add_all(s, 4, n) for s in sims]
    b = mpx.Batch(sims)
    b.set_graph_steps(4)
    for c in CALLS:
        b.step(c)
    b.sync()
    for m, s in enumerate(sims):
        for q, i in enumerate(ids[m]):
            got = s.read_probe(i, NVAL[q])
            assert got.shape[0] == n // 4, (m, q)
            assert np.array_equal(got, ref[m][q]), (m, q)
    b.close()
    for s in sims:
        s.close()


def test_probe_arguments():
    w = W.random_case(33, nx=16, ny=12, nz=10, bc=(W.PML,) * 6, npml=(3,) * 6, film=False, nsteps=4)
    s = mpx.from_workload(w, precision=mpx.F64)
    with pytest.raises(mpx.MpxError) as e:
        s.add_probe(mpx.PROBE_EM_ENERGY)
    assert e.value.code == 5
    with pytest.raises(mpx.MpxError) as e:
        s.add_probe(mpx.PROBE_FIELD, field=0, ijk=(3, 3, 3), every=-1)
    assert e.value.code == 1
    with pytest.raises(mpx.MpxError) as e:
        s.add_probe(4)
    assert e.value.code == 1
    s.close()
