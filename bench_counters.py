#!/usr/bin/env python3
"""HBM traffic of the stencil kernels from rocprofv3 PMC counters.

Two steps (the counters need rocprofv3 as the outer process):

  1. run, once per counter (one counter block per run):
       rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir_fetch> -o pmc -- \
           python3 bench_counters.py --run [--workload c2|c5] [--dtype f32|f64] [--steps N]
       rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir_write> -o pmc -- \
           python3 bench_counters.py --run [--workload c2|c5] [--dtype f32|f64] [--steps N]
     The program runs N time steps of the workload (c2: the 512 x 256 x 128
     resonator, c5: the 1536 x 768 x 384 multi-resonator layout; schedule
     --fused, default 0: the separate E and H/M passes) and, after them, a
     plain elementwise kernel (b = a * 2 over 1 GiB of
     float32: reads 1 GiB, writes 1 GiB) whose true traffic is known.

  2. parse:
       python3 bench_counters.py --parse <dir_fetch> <dir_write> [--workload c2|c5] [--dtype f32]
     FETCH_SIZE and WRITE_SIZE are in KiB per dispatch.  Each is scaled by
     (known bytes / what the same counter reads for the calibration kernel), and
     the per-launch HBM bytes of each stencil kernel found are written to
     profiles/traffic.json together with a hash of the kernel source, so that
     bench.py reports them only for the kernel version that was measured.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

COPY_BYTES = 1 << 30


def workload(name: str, nsteps: int):
    from synth import workloads as W
    return W.c5(nsteps) if name == "c5" else W.c2(nsteps)


def run(dtype: str, steps: int, wname: str, fused: int = 0):
    import torch
    from paper_2510_22221_amd import mpx

    w = workload(wname, steps + 4)
    prec = mpx.F32 if dtype == "f32" else mpx.F64
    stream = torch.cuda.current_stream()
    sim = mpx.from_workload(w, precision=prec, stream=stream, graph_steps=0, fused=fused)
    sim.step(steps)
    sim.sync()
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.mul(a, 2.0, out=b)
    torch.cuda.synchronize()
    print(f"ran {steps} steps ({dtype}) and 3 elementwise passes over {COPY_BYTES} bytes", flush=True)


def read_counters(d):
    """{kernel name: [values per dispatch]} from a rocprofv3 csv directory."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection*.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection csv under {d}")
    out = {}
    for f in files:
        with open(f) as fh:
            for row in csv.DictReader(fh):
                name = row.get("Kernel_Name") or row.get("Kernel-Name") or ""
                val = float(row.get("Counter_Value") or row.get("Counter-Value") or 0.0)
                out.setdefault(name, []).append(val)
    return out


def pick(counters, key):
    vals = [v for k, vs in counters.items() if key(k) for v in vs]
    if not vals:
        raise SystemExit("kernel not found in counters")
    return sum(vals) / len(vals), len(vals)


# kernels whose traffic is recorded: the bench's roofline key and a
# predicate on the rocprofv3 kernel name (the merged H/M pass runs as
# k_hbulk_film, which also holds the film's second half step, on 256 x 1
# tiles, else as k_hbulk<T, 2, ...>)
KERNELS = {"e_pass": lambda k: "k_epass<" in k and "batch" not in k,
           "h_pass": lambda k: (re.search(r"k_hbulk<\w+, 2[,>]", k) is not None or "k_hbulk_film<" in k)
           and "batch" not in k,
           "fused": lambda k: ("k_sweep<" in k or "k_fused<" in k) and "batch" not in k}


def parse(dfetch, dwrite, dtype, wname):
    import bench

    cf, cw = read_counters(dfetch), read_counters(dwrite)
    # calibration: b = a * 2 over 1 GiB reads 1 GiB and writes 1 GiB
    cal = {}
    for label, c in (("FETCH_SIZE", cf), ("WRITE_SIZE", cw)):
        kib, n = pick(c, lambda k: "elementwise" in k and "Mul" in k)
        cal[label] = {"calibration_kib_per_dispatch": kib, "calibration_dispatches": n,
                      "scale": (COPY_BYTES / 1024.0) / kib}
    w = workload(wname, 10)
    esz = 4 if dtype == "f32" else 8
    alg = bench.algorithmic_bytes(w, esz)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    for name, pred in KERNELS.items():
        if not any(pred(k) for k in cf):
            continue
        res = {}
        for label, c in (("FETCH_SIZE", cf), ("WRITE_SIZE", cw)):
            kib, n = pick(c, pred)
            res[label] = {"kib_per_dispatch": kib, "dispatches": n, "scale": cal[label]["scale"],
                          "bytes_per_launch": kib * 1024.0 * cal[label]["scale"]}
        total = res["FETCH_SIZE"]["bytes_per_launch"] + res["WRITE_SIZE"]["bytes_per_launch"]
        data[f"{wname}:{name}:{dtype}"] = {"workload": w.name, "source_hash": bench.kernel_source_hash(), "bytes_per_launch": round(total),
                                   "algorithmic_bytes_per_launch": alg[name],
                                   "ratio_to_algorithmic": round(total / alg[name], 4),
                                   "counters": res, "calibration": cal}
        print(name, json.dumps(data[f"{wname}:{name}:{dtype}"], indent=1))
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--run", action="store_true")
    ap.add_argument("--parse", nargs=2, metavar=("DIR_FETCH", "DIR_WRITE"))
    ap.add_argument("--dtype", default="f32", choices=("f32", "f64"))
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--workload", default="c5", choices=("c2", "c5"))
    ap.add_argument("--fused", type=int, default=0, help="0: separate E and H/M passes; 1-5: fused variants")
    args = ap.parse_args()
    if args.run:
        run(args.dtype, args.steps, args.workload, args.fused)
    elif args.parse:
        parse(args.parse[0], args.parse[1], args.dtype, args.workload)
    else:
        ap.error("--run or --parse")


if __name__ == "__main__":
    main()
