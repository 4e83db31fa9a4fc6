#!/usr/bin/env python3
"""Throughput of the coupled Yee + LLG step on one MI355X.

One bench "step" is one full time step of the hot path over the workload
(H/M half step, E step with CPML and source, H/M half step, probes), so a
run of K steps advances the simulation K time steps.  The workload is the
single on-chip resonator: 512 x 256 x 128 cells, silicon substrate, PEC CPW
strips, a 400 x 60 x 4-cell film, PML 10 on every face (synthetic, seeded).

Prints one JSON line: Gcell-updates/s in float32 (float64 in "secondary"),
the roofline of the dominant kernel measured with HIP events on the
library's stream over the timed region, the batched bias sweep against
sequential runs, the adjoint's cost against the forward run on the
128 x 64 x 64 resonator, and the float64 CPU oracle timed on a bounded
sample of the same workload.
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
    h = hashlib.sha256()
    for f in ("kernels.hip", "passes.hip", "fused.hip", "sweep.hip", "stencil.h", "film.h", "device_common.h",
              "mpx_internal.h"):
        with open(os.path.join(ROOT, "paper_2510_22221_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, dtype):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, if they
    were taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        data = json.load(open(p))
        ent = data.get(f"{kernel}:{dtype}")
        if ent and ent.get("source_hash") == kernel_source_hash():
            return ent["bytes_per_launch"]
    except Exception:
        return None
    return None


def run_gpu(w, precision, steps, warmup, every, schedule=0):
    import torch
    from paper_2510_22221_amd import mpx

    stream = torch.cuda.current_stream()
    t0 = time.time()
    sim = mpx.from_workload(w, precision=precision, stream=stream, fused=schedule)
    sim.step(1)
    sim.sync()
    log(f"  setup {time.time() - t0:.1f} s")
    if warmup > 1:
        sim.step(warmup - 1)
    sim.sync()
    torch.cuda.synchronize()
    sim.set_timing(every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    sim.sync()
    wall = time.perf_counter() - t0
    kt = sim.kernel_time()
    sim.set_timing(0)
    return sim, wall, kt


def roofline_for(w, esz, kt, dtype_name, schedule=0):
    fused = schedule != 0
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
           "traffic": traffic_from_profiles(name, dtype_name),
           "algorithmic_bytes_per_launch": ab[name], "avg_launch_ms": round(ms, 5), "launches_timed": nl,
           "film_half1_and_probe_ms_per_step": round(kt[2][0], 5)}
    if not fused:
        # the H/M pass group also holds the film's second half step (on
        # 256 x 1 tiles in the same launch)
        out["other_stencil_kernel"] = {"kernel": ("h_pass", "e_pass")[0 if name == "e_pass" else 1],
                                       "avg_launch_ms": round(kt[1 if name == "e_pass" else 0][0], 5)}
    return out


def batched_sweep(steps, n_inst, variant=None, kchunk=None):
    """The bias sweep: n_inst resonator + film instances of uneven size,
    float32, stepped one after another (each with its own captured graphs)
    and then as one batch (one launch per pass over all instances).
    Both runs start from the same state and the batch's results are bitwise
    those of the single runs (checked in the GPU tests); returns the
    throughput of both."""
    from paper_2510_22221_amd import mpx
    from synth import workloads as W

    ws = W.c3(nsteps=2 * steps + 40, n=n_inst)
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
    b = mpx.Batch(sims)
    if variant:
        b.set_schedule(variant, kchunk or 0)
    b.step(4)
    b.sync()
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    bat = time.perf_counter() - t0
    b.close()
    for s in sims:
        s.close()
    return {"instances": n_inst, "cells": cells, "steps": steps, "dtype": "f32",
            "sequential_Gcell_s": round(cells * steps / seq / 1e9, 3),
            "batched_Gcell_s": round(cells * steps / bat / 1e9, 3),
            "batched_over_sequential": round(seq / bat, 3),
            "schedule": ("separate E and H/M passes" if not variant else f"fused pass, variant {variant}")}


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
           "schedule": "tape, fused field passes"}
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
        s = mpx.from_workload(w, precision=prec, graph_steps=gs)
        t0 = time.perf_counter()
        r = s.adjoint(steps, steps - window, eps_box=w.patch_box, ms_box=w.film_top)
        adj = time.perf_counter() - t0
        s.close()
        out[name] = {"forward_s": round(fwd, 4), "adjoint_s": round(adj, 4), "adjoint_over_forward": round(adj / fwd, 3),
                     "loss": r["loss"], "dL_dH0z": float(r["dH0"][2])}
        log(f"  adjoint {name}: forward {fwd:.3f} s, adjoint {adj:.3f} s, ratio {adj / fwd:.2f}")
    return out


def cpu_baseline(w, nsteps):
    import oracle.oracle as O
    O.build()
    O.set_threads(min(os.cpu_count() or 1, 64))
    threads = O.get_threads()
    t0 = time.time()
    s = O.from_workload(w)
    log(f"  oracle setup {time.time() - t0:.1f} s, {threads} threads")
    t0 = time.perf_counter()
    s.step(nsteps)
    dt = time.perf_counter() - t0
    return {"value": round(w.ncells * nsteps / dt / 1e9, 5), "unit": "Gcell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{w.nx}x{w.ny}x{w.nz} resonator, {nsteps} of its time steps, float64, setup excluded, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--f64-steps", type=int, default=4000)
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--timing-every", type=int, default=0, help="event-time every n-th step (0: auto)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--ny", type=int, default=256)
    ap.add_argument("--nz", type=int, default=128)
    ap.add_argument("--schedule", type=int, default=0,
                    help="0: separate E and H/M passes (default); 1-5: fused pass variants")
    ap.add_argument("--sweep-steps", type=int, default=1000, help="steps of the batched bias sweep (0: skip)")
    ap.add_argument("--sweep-instances", type=int, default=64)
    ap.add_argument("--adjoint-steps", type=int, default=20000, help="steps of the adjoint cost run (0: skip)")
    ap.add_argument("--adjoint-window", type=int, default=5000)
    ap.add_argument("--adjoint-no-graphs", action="store_true",
                    help="launch the adjoint's kernels directly (for kernel traces)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path shards by z-slabs "
              "across GPUs by design; only the one-GPU path is implemented)", file=sys.stderr)
        sys.exit(2)
    from synth import workloads as W
    from paper_2510_22221_amd import mpx

    w = W.c2(max(args.steps, args.f64_steps) + args.warmup + 2, nx=args.nx, ny=args.ny, nz=args.nz)
    every = args.timing_every or max(1, args.steps // 2000)
    log(f"workload {w.name}: {w.ncells} cells, FP32 {args.steps} steps (+{args.warmup} warmup)")
    sched = args.schedule
    sim, wall, kt = run_gpu(w, mpx.F32, args.steps, args.warmup, every, sched)
    del sim
    value = w.ncells * args.steps / wall / 1e9
    roof = roofline_for(w, 4, kt, "f32", sched)
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
        "config": {"workload": f"single on-chip CPW resonator + film, {w.nx}x{w.ny}x{w.nz} cells, "
                               f"d=(45,2,2) um, PML 10, source + probes, one time step per bench step",
                   "cells": w.ncells, "precision": "f32 fields, f64 magnetisation",
                   "schedule": ("separate E and H/M passes" if sched == 0 else f"fused pass, variant {sched}"),
                   "parallelism": "single GPU"},
        "roofline": roof,
    }
    if not args.no_f64:
        log(f"FP64 {args.f64_steps} steps")
        sim, wall64, kt64 = run_gpu(w, mpx.F64, args.f64_steps, args.warmup, max(1, args.f64_steps // 2000), sched)
        del sim
        out["secondary"] = [{"dtype": "f64", "value": round(w.ncells * args.f64_steps / wall64 / 1e9, 3),
                             "unit": "Gcell-updates/s", "steps": args.f64_steps,
                             "ms_per_step": round(wall64 / args.f64_steps * 1e3, 5),
                             "roofline": roofline_for(w, 8, kt64, "f64", sched)}]
    if args.sweep_steps > 0:
        log(f"batched bias sweep: {args.sweep_instances} instances, {args.sweep_steps} steps")
        out["batched_sweep"] = batched_sweep(args.sweep_steps, args.sweep_instances)
    if args.adjoint_steps > 0:
        log(f"adjoint: {args.adjoint_steps} steps, loss over the last {args.adjoint_window}")
        out["adjoint"] = adjoint_cost(args.adjoint_steps, min(args.adjoint_window, args.adjoint_steps),
                                      graphs=not args.adjoint_no_graphs)
    if not args.no_cpu:
        log(f"CPU oracle baseline: {args.cpu_steps} steps")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
