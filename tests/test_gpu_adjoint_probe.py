"""Gradients of a weighted probe trace by the discrete adjoint
(mpx_adjoint_probe), and of spectral functionals of the trace through the
torch wrapper.

L = sum_i w_i E_c(site) after step i+1.  Small cases: the loss and its
central finite differences come from the FP64 CPU oracle; the adjoint
gradients must agree within 1e-5 relative.  The resonator at full size
(128 x 64 x 64, 400 steps): a spectral functional of the trace (the
band-centroid splitting) through probe_functional against Richardson
central differences of the GPU forward run.
"""
import numpy as np
import pytest

from oracle import fd
from paper_2510_22221_amd import mpx
from synth import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(msg):
    print(msg, flush=True)


def small_case(pml: bool):
    w = W.random_case(11, nx=20, ny=16, nz=14, nsteps=60,
                      bc=(W.PML, W.PML, W.PEC, W.PEC, W.PML, W.PML) if pml else (W.PEC,) * 6,
                      npml=(2, 2, 0, 0, 2, 2) if pml else (0,) * 6)
    w.H0 = (3e6, 0.0, 5e6)
    return w


def film_geometry(w):
    cells = list(zip(*[a.tolist() for a in np.nonzero(w.ids == 3)]))  # (k, j, i)
    kf, jf, i_f = cells[len(cells) // 2]
    kz0 = min(c[0] for c in cells)
    return kf, jf, i_f, kz0


def close(a, b, scale, tol=TOL):
    return abs(a - b) <= tol * scale


@pytest.mark.parametrize("pml,field", [(False, 0), (True, 1), (True, 2)])
def test_trace_adjoint_matches_oracle_finite_differences(pml, field):
    w = small_case(pml)
    n, K = 60, 7
    kf, jf, i_f, kz0 = film_geometry(w)
    ijk = (i_f, jf, kz0 - 1)
    wt = np.random.default_rng(100 + field).standard_normal(n)
    eps_box = (i_f - 1, jf - 1, kz0 - 3, 3, 2, 2)
    ms_box = (i_f, jf, kf, 2, 1, 1)
    say(f"trace adjoint pml={pml} field={field} at {ijk}: GPU")
    g = mpx.from_workload(w, precision=mpx.F64)
    res = g.adjoint_probe(n, field, ijk, wt, checkpoint_every=K, eps_box=eps_box, ms_box=ms_box)
    g.close()

    def lossf(w2):
        return fd.trace_loss(w2, n, field, ijk, wt)

    L = lossf(w)
    say(f"  loss GPU {res['loss']:.15e} oracle {L:.15e}")
    assert res["loss"] == pytest.approx(L, rel=1e-11)
    gh = [fd.grad_H0_of(lossf, w, c) for c in range(3)]
    say(f"  dL/dH0 adjoint {res['dH0']} fd {gh}")
    sc = max(abs(v) for v in gh)
    assert sc > 0
    for c in range(3):
        assert close(res["dH0"][c], gh[c], sc), (c, res["dH0"][c], gh[c])
    ge = []
    for (di, dj, dk) in ((0, 0, 0), (1, 1, 1), (2, 0, 1)):
        cell = (eps_box[0] + di, eps_box[1] + dj, eps_box[2] + dk)
        if w.materials[int(w.ids[cell[2], cell[1], cell[0]])][2]:
            continue  # a PEC cell has no eps
        ge.append((res["deps"][dk, dj, di], fd.grad_eps_of(lossf, w, cell)))
    say(f"  dL/deps (adjoint, fd) {ge}")
    sc = max(abs(b) for _, b in ge)
    assert sc > 0
    for a, b in ge:
        assert close(a, b, sc), (a, b)
    gm = [(res["dMs"][0, 0, di], fd.grad_Ms_of(lossf, w, (ms_box[0] + di, ms_box[1], ms_box[2]))) for di in range(2)]
    say(f"  dL/dMs (adjoint, fd) {gm}")
    sc = max(abs(b) for _, b in gm)
    assert sc > 0
    for a, b in gm:
        assert close(a, b, sc), (a, b)


def test_trace_adjoint_periodic_box():
    """Periodic x, PEC y, CPML z, a film: the weighted E_z trace at an edge
    one cell from the periodic seam; dL/dH0 and dL/deps_r of cells that
    straddle the seam against the oracle's differences."""
    w = W.random_case(6, nx=29, ny=17, nz=23, bc=(W.PERIODIC, W.PERIODIC, W.PEC, W.PEC, W.PML, W.PML),
                      npml=(0, 0, 0, 0, 4, 4), nsteps=40)
    w.H0 = (2e6, 1e6, 4e6)
    n, K = 40, 6
    kf, jf, i_f, kz0 = film_geometry(w)
    ijk = (1, jf, kz0 - 1)
    wt = np.random.default_rng(13).standard_normal(n)
    eb = (27, jf - 1, kz0 - 3, 2, 2, 2)  # x cells 27, 28: the seam is at 0
    g = mpx.from_workload(w, precision=mpx.F64)
    res = g.adjoint_probe(n, 2, ijk, wt, checkpoint_every=K, eps_box=eb)
    g.close()

    def lossf(w2):
        return fd.trace_loss(w2, n, 2, ijk, wt)

    assert res["loss"] == pytest.approx(lossf(w), rel=1e-11)
    gh = [fd.grad_H0_of(lossf, w, c) for c in range(3)]
    say(f"periodic: dL/dH0 adjoint {res['dH0']} fd {gh}")
    sc = max(abs(v) for v in gh)
    assert sc > 0
    for c in range(3):
        assert close(res["dH0"][c], gh[c], sc), (c, res["dH0"][c], gh[c])
    ge = []
    for (di, dj, dk) in ((1, 0, 0), (0, 1, 1), (1, 1, 0)):
        cell = (eb[0] + di, eb[1] + dj, eb[2] + dk)
        if w.materials[int(w.ids[cell[2], cell[1], cell[0]])][2]:
            continue
        ge.append((res["deps"][dk, dj, di], fd.grad_eps_of(lossf, w, cell)))
    say(f"periodic: dL/deps (adjoint, fd) {ge}")
    sc = max(abs(b) for _, b in ge)
    assert sc > 0
    for a, b in ge:
        assert close(a, b, sc), (a, b)


def test_trace_adjoint_without_films():
    """No magnetic cell: the bias enters nothing, so dL/dH0 is exactly zero,
    and dL/deps_r still matches the oracle's differences."""
    w = W.random_case(12, nx=18, ny=14, nz=12, nsteps=40, film=False)
    n, K, ijk = 40, 6, (9, 7, 6)
    wt = np.random.default_rng(12).standard_normal(n)
    eb = (7, 5, 4, 3, 2, 2)
    g = mpx.from_workload(w, precision=mpx.F64)
    res = g.adjoint_probe(n, 1, ijk, wt, checkpoint_every=K, eps_box=eb)
    g.close()

    def lossf(w2):
        return fd.trace_loss(w2, n, 1, ijk, wt)

    assert res["loss"] == pytest.approx(lossf(w), rel=1e-11)
    assert np.all(res["dH0"] == 0.0)
    ge = []
    for (di, dj, dk) in ((0, 0, 0), (2, 1, 1), (1, 0, 1)):
        cell = (eb[0] + di, eb[1] + dj, eb[2] + dk)
        if w.materials[int(w.ids[cell[2], cell[1], cell[0]])][2]:
            continue
        ge.append((res["deps"][dk, dj, di], fd.grad_eps_of(lossf, w, cell)))
    say(f"no film: dL/deps (adjoint, fd) {ge}")
    sc = max(abs(b) for _, b in ge)
    assert sc > 0
    for a, b in ge:
        assert close(a, b, sc), (a, b)


def run(w, prec, n, field, ijk, wt, K, eps_box, ms_box, graphs=True):
    g = mpx.from_workload(w, precision=prec, graph_steps=None if graphs else 0)
    res = g.adjoint_probe(n, field, ijk, wt, checkpoint_every=K, eps_box=eps_box, ms_box=ms_box)
    g.close()
    return res


def test_trace_adjoint_is_linear_in_the_weights_and_graph_free():
    """Gradients of w1 + 3 w2 equal those of w1 plus 3 times those of w2 (up
    to rounding), and the graph-replayed segments equal direct launches
    bitwise."""
    w = small_case(True)
    n, K = 50, 6
    kf, jf, i_f, kz0 = film_geometry(w)
    ijk, eb, mb = (i_f + 1, jf, kz0 - 1), (i_f - 1, jf - 1, kz0 - 3, 3, 2, 2), (i_f - 1, jf, kf, 3, 1, 1)
    rng = np.random.default_rng(7)
    w1, w2 = rng.standard_normal(n), rng.standard_normal(n)
    say("trace adjoint linearity")
    r1 = run(w, mpx.F64, n, 0, ijk, w1, K, eb, mb)
    r2 = run(w, mpx.F64, n, 0, ijk, w2, K, eb, mb)
    r3 = run(w, mpx.F64, n, 0, ijk, w1 + 3.0 * w2, K, eb, mb)
    for key in ("dH0", "deps", "dMs"):
        a, b = r3[key], r1[key] + 3.0 * r2[key]
        sc = np.max(np.abs(b))
        assert sc > 0, key
        assert np.max(np.abs(a - b)) <= 1e-10 * sc, key
    say("trace adjoint without graphs")
    r4 = run(w, mpx.F64, n, 0, ijk, w1, K, eb, mb, graphs=False)
    for key in ("dH0", "deps", "dMs"):
        assert np.array_equal(r1[key], r4[key]), key
    assert r1["loss"] == r4["loss"]


def test_trace_adjoint_kept_tapes_match_recompute():
    """The weighted-trace loss with segments that keep their forward tapes
    (all of them, or a cap that keeps only some) against every segment
    recomputed from its checkpoint: float64 bitwise."""
    w = small_case(True)
    n, K = 48, 5
    kf, jf, i_f, kz0 = film_geometry(w)
    ijk, eb, mb = (i_f, jf + 1, kz0 - 1), (i_f - 2, jf - 1, kz0 - 3, 4, 2, 2), (i_f - 1, jf, kf, 3, 1, 1)
    wt = np.random.default_rng(21).standard_normal(n)
    out = {}
    for cap in (0, -1, 2 ** 16, 2 ** 18, 2 ** 20):
        say(f"trace adjoint, kept-tape cap {cap}")
        g = mpx.from_workload(w, precision=mpx.F64)
        g.set_adjoint_memory(cap)
        out[cap] = g.adjoint_probe(n, 1, ijk, wt, checkpoint_every=K, eps_box=eb, ms_box=mb)
        out[cap]["E1"] = g.get(1)
        g.close()
    ref = out[0]
    for cap, r in out.items():
        assert r["loss"] == ref["loss"], cap
        assert np.array_equal(r["E1"], ref["E1"]), cap
        for key in ("dH0", "deps", "dMs"):
            assert np.array_equal(r[key], ref[key]), (cap, key)


def test_trace_adjoint_float32_tracks_float64():
    w = small_case(True)
    n, K = 60, 8
    kf, jf, i_f, kz0 = film_geometry(w)
    ijk, eb, mb = (i_f, jf, kz0 - 1), (i_f - 1, jf - 1, kz0 - 3, 3, 2, 2), (i_f - 1, jf, kf, 3, 1, 1)
    wt = np.random.default_rng(9).standard_normal(n)
    r64 = run(w, mpx.F64, n, 2, ijk, wt, K, eb, mb)
    r32 = run(w, mpx.F32, n, 2, ijk, wt, K, eb, mb)
    say(f"f32 {r32['dH0']} f64 {r64['dH0']}")
    for key in ("dH0", "deps", "dMs"):
        sc = np.max(np.abs(r64[key]))
        assert np.max(np.abs(r32[key] - r64[key])) <= 1e-3 * sc, key


def test_trace_adjoint_rejects_bad_arguments():
    w = small_case(False)
    g = mpx.from_workload(w, precision=mpx.F64)
    wt = np.ones(10)
    z = (0, 0, 0, 0, 0, 0)
    with pytest.raises(mpx.MpxError) as e:
        g.adjoint_probe(10, 3, (1, 1, 1), wt)
    assert e.value.code == 1
    with pytest.raises(mpx.MpxError) as e:
        g.adjoint_probe(10, 0, (w.nx, 1, 1), wt)
    assert e.value.code == 1
    bad = wt.copy()
    bad[4] = np.nan
    with pytest.raises(mpx.MpxError) as e:
        g.adjoint_probe(10, 0, (1, 1, 1), bad)
    assert e.value.code == 1
    with pytest.raises(ValueError):
        g.adjoint_probe(10, 0, (1, 1, 1), np.ones(9))
    g.set_adjoint_schedule(1)
    with pytest.raises(mpx.MpxError) as e:
        g.adjoint_probe(10, 0, (1, 1, 1), wt, eps_box=z, ms_box=z)
    assert e.value.code == 5
    assert g.info()["step"] == 0  # nothing ran
    g.close()


def c4_param_workload(n, h0, eps_patch, f):
    """The resonator with its eps_r patch at eps_patch (one material) and the
    film's top layer at Ms f (a material of its own, same film)."""
    w = W.c4(n)
    w.m_dir = (0.25, 0.0, 1.0)
    w.H0 = tuple(h0)
    mats = list(w.materials)
    m3 = mats[3]
    mats[4] = (float(eps_patch),) + tuple(mats[4][1:])
    mats.append((m3[0], m3[1], m3[2], m3[3] * f, m3[4], m3[5]))
    ids = w.ids.copy()
    ft = w.film_top
    ids[ft[2], ft[1]:ft[1] + ft[4], ft[0]:ft[0] + ft[3]] = len(mats) - 1
    w.materials = mats
    w.ids = ids
    return w


def test_probe_functional_splitting_resonator():
    """probe_functional over the 128 x 64 x 64 resonator, 400 steps, E_x
    just above the film centre: the band-centroid splitting of the trace,
    d/dH0_z, d/df (top-layer Ms fraction) and d/deps_r of the patch against
    Richardson central differences of the GPU forward run (float64)."""
    import torch
    from paper_2510_22221_amd import grad as G

    n = 400
    w0 = W.c4(n)
    ms_top = w0.materials[3][3]
    h0 = (0.0, 0.0, w0.H0[2])
    ft = w0.film_top
    ijk = (ft[0] + ft[3] // 2, ft[1] + ft[4] // 2, ft[2] + 1)
    dt = w0.dt
    f_mid, half = 3.0 / (n * dt), 3.0 / (n * dt)

    def fn(tr):
        return G.band_centroid_splitting(tr, dt, f_mid, half)

    def make_sim(h, e, f):
        return mpx.from_workload(c4_param_workload(n, h, float(e), f), precision=mpx.F64)

    spec = G.ProbeTraceSpec(make_sim, n, 0, ijk, eps_box=w0.patch_box, top_box=ft, ms_top=ms_top)
    H0 = torch.tensor(h0, dtype=torch.float64, requires_grad=True)
    eps = torch.tensor(11.7, dtype=torch.float64, requires_grad=True)
    f = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    say("probe functional C4: trace, forward + adjoint")
    F = G.probe_functional(H0, eps, f, spec, fn)
    F.backward()

    def gpu_F(h, e, fv):
        d = torch.float64
        tr = G.record_trace(spec, torch.tensor(h, dtype=d), torch.tensor(e, dtype=d), torch.tensor(fv, dtype=d))
        return float(fn(torch.tensor(tr, dtype=d)))

    assert F.item() == gpu_F(h0, 11.7, 1.0)
    gz = fd.derivative(lambda d: gpu_F((0.0, 0.0, h0[2] + d), 11.7, 1.0), 2e-4 * h0[2])
    gf = fd.derivative(lambda d: gpu_F(h0, 11.7, 1.0 + d), 2e-3)
    ge = fd.derivative(lambda d: gpu_F(h0, 11.7 + d, 1.0), 2e-3 * 11.7)
    say(f"  F {F.item():.9e}")
    say(f"  dF/dH0z {H0.grad[2].item():.9e} fd {gz:.9e}")
    say(f"  dF/df   {f.grad.item():.9e} fd {gf:.9e}")
    say(f"  dF/deps {eps.grad.item():.9e} fd {ge:.9e}")
    assert close(H0.grad[2].item(), gz, abs(gz))
    assert close(f.grad.item(), gf, abs(gf))
    assert close(eps.grad.item(), ge, abs(ge), tol=1e-4)


@pytest.mark.parametrize("prec", [mpx.F64, mpx.F32])
def test_trace_adjoint_merged_pass_bitwise(prec):
    """The weighted-trace adjoint with the merged reverse pass equals the
    one with a pass per half step (schedule 2), bitwise."""
    w = small_case(True)
    n, K = 44, 6
    kf, jf, i_f, kz0 = film_geometry(w)
    ijk, eb, mb = (i_f, jf, kz0 - 1), (i_f - 2, jf - 1, kz0 - 3, 4, 2, 2), (i_f - 1, jf, kf, 3, 1, 1)
    wt = np.random.default_rng(33).standard_normal(n)
    out = []
    for sched in (0, 2):
        g = mpx.from_workload(w, precision=prec)
        g.set_adjoint_schedule(sched)
        out.append(g.adjoint_probe(n, 2, ijk, wt, checkpoint_every=K, eps_box=eb, ms_box=mb))
        g.close()
    a, b = out
    assert a["loss"] == b["loss"]
    for key in ("dH0", "deps", "dMs"):
        assert np.array_equal(a[key], b[key]), key
