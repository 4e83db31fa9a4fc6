#!/usr/bin/env python3
"""HBM traffic of the stencil kernels from rocprofv3 PMC counters.

Two steps (the counters need rocprofv3 as the outer process):

  1. run, once per counter (one counter block per run):
       rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir_fetch> -o pmc -- \
           python3 bench_counters.py --run [--dtype f32|f64] [--steps N]
       rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir_write> -o pmc -- \
           python3 bench_counters.py --run [--dtype f32|f64] [--steps N]
     The program runs N time steps of the resonator workload (fused pass)
     and, after them, a plain elementwise kernel (b = a * 2 over 1 GiB of
     float32: reads 1 GiB, writes 1 GiB) whose true traffic is known.

  2. parse:
       python3 bench_counters.py --parse <dir_fetch> <dir_write> [--dtype f32]
     FETCH_SIZE and WRITE_SIZE are in KiB per dispatch.  Each is scaled by
     (known bytes / what the same counter reads for the calibration kernel), and
     the per-launch HBM bytes of the fused pass are written to
     profiles/traffic.json together with a hash of the kernel source, so that
     bench.py reports them only for the kernel version that was measured.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

COPY_BYTES = 1 << 30
KERNEL = "k_sweep"


def run(dtype: str, steps: int, nx: int, ny: int, nz: int, fused: int = 1):
    import torch
    from paper_2510_22221_amd import mpx
    from synth import workloads as W

    w = W.c2(steps + 4, nx=nx, ny=ny, nz=nz)
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


def parse(dfetch, dwrite, dtype):
    import bench

    from synth import workloads as W

    res = {}
    for label, d in (("FETCH_SIZE", dfetch), ("WRITE_SIZE", dwrite)):
        c = read_counters(d)
        fused, nf = pick(c, lambda k: KERNEL in k)
        copy, nc = pick(c, lambda k: "elementwise" in k and "Mul" in k)
        scale = (COPY_BYTES / 1024.0) / copy   # counter reads KiB
        res[label] = {"fused_kib_per_dispatch": fused, "dispatches": nf, "copy_kib_per_dispatch": copy,
                      "copy_dispatches": nc, "scale": scale, "bytes_per_launch": fused * 1024.0 * scale}
    w = W.c2(10)
    esz = 4 if dtype == "f32" else 8
    alg = bench.algorithmic_bytes(w, esz)["fused"]
    total = res["FETCH_SIZE"]["bytes_per_launch"] + res["WRITE_SIZE"]["bytes_per_launch"]
    path = os.path.join(ROOT, "profiles", "traffic.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    data[f"fused:{dtype}"] = {"source_hash": bench.kernel_source_hash(), "bytes_per_launch": round(total),
                              "algorithmic_bytes_per_launch": alg, "ratio_to_algorithmic": round(total / alg, 4),
                              "counters": res}
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    print(json.dumps(data[f"fused:{dtype}"], indent=1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--run", action="store_true")
    ap.add_argument("--parse", nargs=2, metavar=("DIR_FETCH", "DIR_WRITE"))
    ap.add_argument("--dtype", default="f32", choices=("f32", "f64"))
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--ny", type=int, default=256)
    ap.add_argument("--nz", type=int, default=128)
    ap.add_argument("--fused", type=int, default=1, help="0: separate E and H passes; 1-4: fused tile variant")
    args = ap.parse_args()
    if args.run:
        run(args.dtype, args.steps, args.nx, args.ny, args.nz, args.fused)
    elif args.parse:
        parse(args.parse[0], args.parse[1], args.dtype)
    else:
        ap.error("--run or --parse")


if __name__ == "__main__":
    main()
