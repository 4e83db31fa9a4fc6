#!/usr/bin/env python3
"""Throughput of the coupled Yee + LLG step on one MI355X.

One bench "step" is one full time step of the hot path over the workload
(H/M half step, E step with CPML and source, H/M half step, probes), so a
run of K steps advances the simulation K time steps.  The headline workload
is the large single-GPU layout: 1536 x 768 x 384 cells (453 M), eight PEC
strips each carrying a 200 x 40 x 4-cell film, random eps_r blocks, PML 16 on
every face (synthetic, seeded), in float32.

Prints one JSON line: Gcell-updates/s of the headline workload, the roofline
of its dominant kernel (per-launch durations from HIP events on the
library's stream), the 512 x 256 x 128 single resonator in float32 and
float64 ("secondary"), the batched bias sweep against sequential runs, the
anti-crossing analysed from a sweep's own traces, the adjoint's cost against
the forward run on the 128 x 64 x 64 resonator, and the float64 CPU oracle
timed on a bounded sample of the headline workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gcell-updates/s (Yee+LLG) & % HBM roofline; batched vs single; adjoint/fwd time"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(w, esz):
    """Bytes each stencil kernel must move per launch (one full step).
    Fused pass: read E(3), H(3) and the uint8 id, write E(3), H(3); per slab
    cell and slab axis, read + write the two E-type and the two H-type CPML
    psi.  Two-pass schedule: the E pass reads E, H, id and writes E (+ the
    E-type psi), the H pass reads E, H and writes H (+ the H-type psi)."""
    ncell = w.nx * w.ny * w.nz
    n = (w.nx, w.ny, w.nz)
    slab = 0
    for a in range(3):
        thick = w.npml[2 * a] * (w.bc[2 * a] == 1) + w.npml[2 * a + 1] * (w.bc[2 * a + 1] == 1)
        slab += thick * ncell // n[a]
    return {"fused": ncell * (12 * esz + 1) + slab * 8 * esz,
            "e_pass": ncell * (9 * esz + 1) + slab * 4 * esz,
            "h_pass": ncell * 9 * esz + slab * 4 * esz,
            "ncell": ncell, "slab_cells": slab}


def kernel_source_hash():
    """Hash of the sources the separate passes' kernels are built from
    (passes.hip and the headers it includes), with comments removed and
    every run of white space made one space (an edited comment, a reformatted
    line or a change to another kernel file leaves the measured kernels, and
    this hash, as they were)."""
    import re

    h = hashlib.sha256()
    for f in ("passes.hip", "stencil.h", "film.h", "device_common.h", "mpx_internal.h"):
        with open(os.path.join(ROOT, "paper_2510_22221_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, dtype, wkey):
    """HBM bytes per launch of a kernel on workload `wkey` (c2, c5) from the
    committed rocprofv3 PMC summaries, if they were taken on the current
    kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        data = json.load(open(p))
        ent = data.get(f"{wkey}:{kernel}:{dtype}")
        if ent and ent.get("source_hash") == kernel_source_hash():
            return ent["bytes_per_launch"]
    except Exception:
        return None
    return None


def run_gpu(w, precision, steps, warmup, timing_steps=12, schedule=0):
    """Steps `w` on the GPU: `warmup` untimed steps, one untimed call that
    captures the HIP graph of the step batch the timed call replays, then
    `steps` steps timed by the host clock between two device synchronisations
    (graph replays, no per-step events), then a separate short pass of
    `timing_steps` steps with every kernel group bracketed by HIP events on
    the library's stream (direct launches) for the per-launch durations."""
    import torch
    from paper_2510_22221_amd import mpx

    stream = torch.cuda.current_stream()
    t0 = time.time()
    sim = mpx.from_workload(w, precision=precision, stream=stream, fused=schedule)
    # an even batch the timed call replays at least once
    G = max(2, min(64, (steps - 1) // 2 * 2))
    sim.set_graph_steps(G)
    sim.step(1)
    sim.sync()
    log(f"  setup {time.time() - t0:.1f} s, graph batch {G} steps")
    if warmup > 1:
        sim.step(warmup - 1)
    sim.step(G + 1)  # captures the graph for the parity the timed call starts at
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    sim.sync()
    wall = time.perf_counter() - t0
    sim.set_timing(1)
    sim.step(timing_steps)
    sim.sync()
    kt = sim.kernel_time()
    sim.set_timing(0)
    return sim, wall, kt


def schedule_name(sched):
    if sched == 0:
        return "separate E and H/M passes (256 x 1 tiles on grids at least 512 wide)"
    if sched == 6:
        return "separate E and H/M passes on 64 x 4 tiles"
    return f"fused pass, variant {sched}"


def roofline_for(w, esz, kt, dtype_name, schedule=0, wkey="c5"):
    fused = 1 <= schedule <= 5
    ab = algorithmic_bytes(w, esz)
    if fused:
        name, ms, nl = "fused", kt[0][0], kt[0][1]
    else:
        # the dominant of the two stencil kernels
        q = 0 if kt[0][0] >= kt[1][0] else 1
        name, ms, nl = ("e_pass", "h_pass")[q], kt[q][0], kt[q][1]
    achieved = ab[name] / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    out = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": traffic_from_profiles(name, dtype_name, wkey),
           "algorithmic_bytes_per_launch": ab[name], "avg_launch_ms": round(ms, 5), "launches_timed": nl,
           "film_half1_ms_per_step": round(kt[2][0], 5)}
    if not fused:
        # the H/M pass group also holds the film's second half step (on
        # 256 x 1 tiles in the same launch, with the probes when all of them
        # read only E or a film's mean M)
        out["other_stencil_kernel"] = {"kernel": ("h_pass", "e_pass")[0 if name == "e_pass" else 1],
                                       "avg_launch_ms": round(kt[1 if name == "e_pass" else 0][0], 5)}
    return out


def batched_sweep(steps, n_inst, tune_steps=20):
    """The bias sweep: n_inst resonator + film instances of uneven size,
    float32, stepped one after another (each with its own captured graphs),
    then as one batch (one launch per pass over all instances) with the
    default schedule, and as one batch with the schedule the autotuner picks
    for it (every candidate timed on scratch copies of the same instances).
    All runs give the single runs' bits (checked in the GPU tests); returns
    the throughput of each."""
    from paper_2510_22221_amd import mpx, tune
    from synth import workloads as W

    ws = W.c3(nsteps=3 * steps + 60, n=n_inst)
    cells = sum(w.ncells for w in ws)
    t0 = time.time()
    sims = [mpx.from_workload(w, precision=mpx.F32) for w in ws]
    log(f"  {n_inst} instances, {cells} cells, setup {time.time() - t0:.1f} s")
    for s in sims:
        s.step(4)
    for s in sims:
        s.sync()
    t0 = time.perf_counter()
    for s in sims:
        s.step(steps)
        s.sync()
    seq = time.perf_counter() - t0

    def timed_batch(variant, kchunk):
        b = mpx.Batch(sims)
        b.set_schedule(variant, kchunk)
        b.step(4)
        b.sync()
        t0 = time.perf_counter()
        b.step(steps)
        b.sync()
        el = time.perf_counter() - t0
        b.close()
        return el

    bat = timed_batch(0, 0)
    t0 = time.time()
    v, kc, _ = tune.tune_batch(ws, precision=mpx.F32, steps=tune_steps, cache=None)
    log(f"  autotuner: variant {v}, z-chunk {kc} ({time.time() - t0:.1f} s)")
    tuned = timed_batch(v, kc)
    for s in sims:
        s.close()
    rate = lambda el: round(cells * steps / el / 1e9, 3)
    return {"instances": n_inst, "cells": cells, "steps": steps, "dtype": "f32",
            "sequential_Gcell_s": rate(seq),
            "batched_Gcell_s": rate(bat),
            "batched_over_sequential": round(seq / bat, 3),
            "schedule": "separate E and H/M passes (64 x 4 tiles)",
            "tuned": {"variant": v, "kchunk": kc,
                      "schedule": ("separate E and H/M passes" if v == 0 else f"fused pass, variant {v}"),
                      "batched_Gcell_s": rate(tuned), "batched_over_sequential": round(seq / tuned, 3)}}


def anticrossing(steps, n_inst, drive_factor=3000.0):
    """The bias sweep's own traces through the spectral analysis: n_inst
    copies of one 96 x 64 x 64 resonator + film whose bias runs over
    0.7-1.3 of the field that tunes the film to the resonator, stepped as
    one float32 batch; per instance the two strongest modes of the film's
    mean M_x (ESPRIT on the trace after the drive pulse), then a fit of the
    hybrid-mode law (eq. omega_pm) with the magnon branch proportional to
    mu0 |gamma| H0 / 2 pi: the photon frequency, the coupling g and the
    minimum splitting (the magnon branch fitted with a slope and an offset on
    that law).  The drive-power variant: the instance nearest the
    crossing with its source `drive_factor` times stronger."""
    import numpy as np
    from paper_2510_22221_amd import mpx, spectral as S
    from synth import workloads as W

    hs = np.linspace(0.7, 1.3, n_inst)
    ws = [W.c3_instance(96, 64, 64, float(h), steps) for h in hs]
    for w in ws:
        w.probes = [W.Probe("mean_m", film=0)]
    dt = ws[0].dt
    sims = [mpx.from_workload(w, precision=mpx.F32) for w in ws]
    b = mpx.Batch(sims)
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    run_s = time.perf_counter() - t0
    b.close()
    skip = steps // 5

    def two_modes(sim):
        mx = sim.read_probe(0, 3)[skip:, 0]
        return S.sweep_branches([mx], dt, 2, stride=8, fmin=1e9, min_separation=0.02, max_rows=512)[0]

    br = np.array([two_modes(s) for s in sims])
    for s in sims:
        s.close()
    H0 = np.array([w.H0[2] for w in ws])
    lo, hi = br[:, 0], br[:, 1]
    fit = S.fit_anticrossing(H0, lo, hi, lambda h: S.kittel_perpendicular(h, 0.0), fp0=float(np.median(hi[:2])),
                             g0=0.25 * float(np.min(hi - lo)), fit_scale=True, fit_offset=True)
    split, q = S.mode_splitting(lo, hi)
    out = {"instances": n_inst, "grid": "96x64x64", "steps": steps, "dtype": "f32", "batched_run_s": round(run_s, 2),
           "H0_over_tuned": [round(float(h), 4) for h in hs],
           "lower_GHz": [round(float(v) / 1e9, 4) for v in lo], "upper_GHz": [round(float(v) / 1e9, 4) for v in hi],
           "fit": {"f_photon_GHz": round(fit.fp / 1e9, 4), "g_GHz": round(fit.g / 1e9, 4),
                   "magnon_branch": f"{fit.scale:.5f} x mu0|gamma|H0/2pi + {fit.offset / 1e9:.4f} GHz",
                   "residual_rms_GHz": round(fit.residual_rms / 1e9, 4)},
           "min_splitting_GHz": round(split / 1e9, 4), "min_at_H0_over_tuned": round(float(hs[q]), 4)}
    # the drive-power variant at the instance nearest the crossing
    qc = int(np.argmin(np.abs(hs - 1.0)))
    drv = {}
    for name, w in (("x1", ws[qc]), (f"x{drive_factor:g}", W.scaled_drive(ws[qc], drive_factor))):
        s = mpx.from_workload(w, precision=mpx.F32)
        s.step(steps)
        s.sync()
        f = two_modes(s)
        drv[name] = {"lower_GHz": round(float(f[0]) / 1e9, 4), "upper_GHz": round(float(f[1]) / 1e9, 4),
                     "max_abs_dMx_over_Ms": round(float(np.abs(s.read_probe(0, 3)[:, 0]).max()) / 1.4e5, 6)}
        s.close()
    out["drive_power"] = {"H0_over_tuned": round(float(hs[qc]), 4), **drv}
    return out


def adjoint_cost(steps, window, graphs=True):
    """The adjoint of the 128 x 64 x 64 resonator + film + eps_r patch
    workload: loss = film EM energy summed over the last `window` of `steps`
    time steps, gradients w.r.t. H0, eps_r of each of the 32 x 16 x 4 patch
    cells and Ms of the film's top layer (the thickness fraction), sqrt(N)
    checkpoints; its wall time against the forward run of the same steps."""
    from paper_2510_22221_amd import mpx
    from synth import workloads as W

    w = W.c4(steps + 10)
    out = {"workload": f"resonator + film + eps_r patch, {w.nx}x{w.ny}x{w.nz} cells, d=(40,2,2) um, PML 8",
           "steps": steps, "loss_window": window, "eps_cells": int(w.patch_box[3] * w.patch_box[4] * w.patch_box[5]),
           "schedule": "tape (segments keep their forward tapes as memory allows), fused field passes"}
    gs = None if graphs else 0
    for name, prec in (("f32", mpx.F32), ("f64", mpx.F64)):
        s = mpx.from_workload(w, precision=prec, graph_steps=gs)
        s.step(50)
        s.sync()
        s.close()
        s = mpx.from_workload(w, precision=prec, graph_steps=gs)
        t0 = time.perf_counter()
        s.step(steps)
        s.sync()
        fwd = time.perf_counter() - t0
        s.close()
        t_adj = {}
        for mem in (-1, 0):
            # -1: tapes kept as memory allows (the default); 0: every segment
            # recomputed from its checkpoint
            s = mpx.from_workload(w, precision=prec, graph_steps=gs)
            s.set_adjoint_memory(mem)
            t0 = time.perf_counter()
            r = s.adjoint(steps, steps - window, eps_box=w.patch_box, ms_box=w.film_top)
            t_adj[mem] = time.perf_counter() - t0
            s.close()
            if mem == -1:
                res = r
        adj = t_adj[-1]
        out[name] = {"forward_s": round(fwd, 4), "adjoint_s": round(adj, 4), "adjoint_over_forward": round(adj / fwd, 3),
                     "loss": res["loss"], "dL_dH0z": float(res["dH0"][2]),
                     "recompute_every_segment": {"adjoint_s": round(t_adj[0], 4),
                                                 "adjoint_over_forward": round(t_adj[0] / fwd, 3)}}
        log(f"  adjoint {name}: forward {fwd:.3f} s, adjoint {adj:.3f} s, ratio {adj / fwd:.2f} "
            f"(every segment recomputed: {t_adj[0]:.3f} s, {t_adj[0] / fwd:.2f})")
    return out


def adjoint_cost_c2(steps, graphs=True):
    """The adjoint on the 512 x 256 x 128 resonator: loss = film EM energy
    over the last quarter of `steps`, gradients w.r.t. H0 and eps_r of a
    32 x 16 x 4 patch in the substrate under the film centre; wall time
    against the forward run of the same steps (float32 and float64)."""
    import numpy as np
    from paper_2510_22221_amd import mpx
    from synth import workloads as W

    w = W.c2(steps + 10)
    w.probes = [W.Probe("film_energy", film=0)]
    kf = int(np.nonzero((w.ids == 3).any(axis=(1, 2)))[0].min())
    ys, xs = np.nonzero(w.ids[kf] == 3)
    eps_box = (int(xs.mean()) - 16, int(ys.mean()) - 8, kf - 8, 32, 16, 4)
    window = steps // 4
    out = {"workload": f"single CPW resonator + film, {w.nx}x{w.ny}x{w.nz} cells, PML 10", "steps": steps,
           "loss_window": window, "eps_cells": 32 * 16 * 4,
           "schedule": "tape (segments keep their forward tapes as memory allows), fused field passes"}
    gs = None if graphs else 0
    for name, prec in (("f32", mpx.F32), ("f64", mpx.F64)):
        s = mpx.from_workload(w, precision=prec, graph_steps=gs)
        s.step(20)
        s.sync()
        s.close()
        s = mpx.from_workload(w, precision=prec, graph_steps=gs)
        t0 = time.perf_counter()
        s.step(steps)
        s.sync()
        fwd = time.perf_counter() - t0
        s.close()
        s = mpx.from_workload(w, precision=prec, graph_steps=gs)
        t0 = time.perf_counter()
        r = s.adjoint(steps, steps - window, eps_box=eps_box, ms_box=(0, 0, 0, 0, 0, 0))
        adj = time.perf_counter() - t0
        s.close()
        out[name] = {"forward_s": round(fwd, 4), "adjoint_s": round(adj, 4), "adjoint_over_forward": round(adj / fwd, 3),
                     "loss": r["loss"], "dL_dH0z": float(r["dH0"][2])}
        log(f"  adjoint 512x256x128 {name}: forward {fwd:.3f} s, adjoint {adj:.3f} s, ratio {adj / fwd:.2f}")
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_oracle(O, w, seconds):
    """Steps the oracle one step at a time until `seconds` have passed;
    returns (steps, elapsed), setup excluded."""
    s = O.from_workload(w)
    s.step(1)  # first touch of every array
    n, t0 = 0, time.perf_counter()
    while True:
        s.step(1)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= seconds:
            return n, dt


def cpu_baseline(w_full, seconds=10.0):
    """The float64 CPU oracle on a bounded sample of the headline workload:
    a 384 x 384 x 192 crop of the 1536 x 768 x 384 layout around its first
    resonator (its film, strip, source, PML 16 and random eps_r blocks), timed
    with all the host threads it may use and with one thread."""
    import oracle.oracle as O
    from synth import workloads as W

    O.build()
    w = W.crop(w_full, (0, 0, 96), (384, 384, 192))
    O.set_threads(min(os.cpu_count() or 1, 64))
    threads = O.get_threads()
    n, dt = _time_oracle(O, w, seconds)
    log(f"  oracle {threads} threads: {n} steps in {dt:.1f} s")
    O.set_threads(1)
    n1, dt1 = _time_oracle(O, w, seconds)
    log(f"  oracle 1 thread: {n1} steps in {dt1:.1f} s")
    O.set_threads(threads)
    sample = (f"{w.nx}x{w.ny}x{w.nz} crop (origin 0,0,96) of the {w_full.nx}x{w_full.ny}x{w_full.nz} layout, "
              f"float64, setup excluded")
    return {"value": round(w.ncells * n / dt / 1e9, 5), "unit": "Gcell-updates/s", "cores": threads,
            "kind": "oracle", "sample": f"{sample}: {n} steps in {dt:.1f} s",
            "single_core": {"value": round(w.ncells * n1 / dt1 / 1e9, 5), "cores": 1,
                            "sample": f"{sample}: {n1} steps in {dt1:.1f} s"},
            "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count()}


def stencil_line(w, precision, dtype_name, esz, steps, warmup, sched, wkey):
    from paper_2510_22221_amd import mpx
    sim, wall, kt = run_gpu(w, precision, steps, warmup, schedule=sched)
    sim.close()
    return {"dtype": dtype_name, "value": round(w.ncells * steps / wall / 1e9, 3), "unit": "Gcell-updates/s",
            "steps": steps, "ms_per_step": round(wall / steps * 1e3, 5),
            "roofline": roofline_for(w, esz, kt, dtype_name, sched, wkey)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--c2-steps", type=int, default=4000, help="steps of the 512x256x128 lines (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--schedule", type=int, default=0,
                    help="0: separate E and H/M passes (default); 1-5: fused pass variants; 6: separate passes on "
                         "64 x 4 tiles")
    ap.add_argument("--sweep-steps", type=int, default=1000, help="steps of the batched bias sweep (0: skip)")
    ap.add_argument("--sweep-instances", type=int, default=64)
    ap.add_argument("--anticrossing-steps", type=int, default=100000,
                    help="steps of the sweep analysed for the anti-crossing (0: skip)")
    ap.add_argument("--adjoint-steps", type=int, default=20000, help="steps of the adjoint cost run (0: skip)")
    ap.add_argument("--adjoint-c2-steps", type=int, default=2000,
                    help="steps of the adjoint cost run on the 512x256x128 resonator (0: skip)")
    ap.add_argument("--adjoint-window", type=int, default=5000)
    ap.add_argument("--adjoint-no-graphs", action="store_true",
                    help="launch the adjoint's kernels directly (for kernel traces)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path would shard by "
              "z-slabs across GPUs; only the one-GPU path is built)", file=sys.stderr)
        sys.exit(2)
    from synth import workloads as W
    from paper_2510_22221_amd import mpx

    sched = args.schedule
    w = W.c5(args.steps + args.warmup + 160)
    log(f"workload {w.name}: {w.ncells} cells, FP32 {args.steps} steps (+{args.warmup} warmup)")
    sim, wall, kt = run_gpu(w, mpx.F32, args.steps, args.warmup, schedule=sched)
    sim.close()
    del sim
    value = w.ncells * args.steps / wall / 1e9
    roof = roofline_for(w, 4, kt, "f32", sched, "c5")
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"large single-GPU multi-resonator layout, {w.nx}x{w.ny}x{w.nz} cells, "
                               f"d=2 um, 8 PEC strips each with a 200x40x4 film, random eps_r in [1,12] per "
                               f"32^3 block, PML 16, source + 8 mean-M probes, one time step per bench step",
                   "cells": w.ncells, "precision": "f32 fields, f64 magnetisation",
                   "schedule": schedule_name(sched),
                   "timing": "host clock around graph replays; kernel durations from a separate "
                             "event-timed pass of 12 steps",
                   "parallelism": "single GPU"},
        "roofline": roof,
    }
    sec = []
    if args.c2_steps > 0:
        w2 = W.c2(args.c2_steps + args.warmup + 160)
        log(f"workload {w2.name}: FP32 {args.c2_steps} steps")
        ent = stencil_line(w2, mpx.F32, "f32", 4, args.c2_steps, args.warmup, sched, "c2")
        ent["workload"] = f"single CPW resonator + film, {w2.nx}x{w2.ny}x{w2.nz} cells, PML 10"
        sec.append(ent)
        if not args.no_f64:
            log(f"workload {w2.name}: FP64 {args.c2_steps} steps")
            ent = stencil_line(w2, mpx.F64, "f64", 8, args.c2_steps, args.warmup, sched, "c2")
            ent["workload"] = f"single CPW resonator + film, {w2.nx}x{w2.ny}x{w2.nz} cells, PML 10"
            sec.append(ent)
    if sec:
        out["secondary"] = sec
    if args.sweep_steps > 0:
        log(f"batched bias sweep: {args.sweep_instances} instances, {args.sweep_steps} steps")
        out["batched_sweep"] = batched_sweep(args.sweep_steps, args.sweep_instances)
    if args.anticrossing_steps > 0:
        log(f"anti-crossing: 12 instances, {args.anticrossing_steps} steps")
        out["anticrossing"] = anticrossing(args.anticrossing_steps, 12)
    if args.adjoint_steps > 0:
        log(f"adjoint: {args.adjoint_steps} steps, loss over the last {args.adjoint_window}")
        out["adjoint"] = adjoint_cost(args.adjoint_steps, min(args.adjoint_window, args.adjoint_steps),
                                      graphs=not args.adjoint_no_graphs)
    if args.adjoint_c2_steps > 0:
        log(f"adjoint on the 512x256x128 resonator: {args.adjoint_c2_steps} steps")
        out["adjoint_512x256x128"] = adjoint_cost_c2(args.adjoint_c2_steps, graphs=not args.adjoint_no_graphs)
    if not args.no_cpu:
        log(f"CPU oracle baseline: about {args.cpu_seconds} s per thread setting")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
