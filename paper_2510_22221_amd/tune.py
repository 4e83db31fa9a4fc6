"""Schedule autotuner for the fused step pass.

A step runs as two separate passes (schedule 0, or 6 for 64 x 4 tiles on
grids that schedule 0 runs on 256 x 1 tiles) or as one fused pass in one of
five tile variants with a z-chunk length; which is fastest depends on
the grid shape, the share of CPML and film tiles, and the precision.  ``tune`` builds scratch
simulations of the caller's workload (the caller's own handles are never
stepped), times every candidate with captured graphs, and caches the winner
in a JSON file keyed by grid, boundary and precision.  All candidates give
bitwise identical results, so the choice only affects speed.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

from . import mpx

VARIANTS = (0, 1, 2, 3, 4, 5)
KCHUNKS = (8, 16, 32)
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def candidates(nz: int, single: bool = False) -> List[Tuple[int, int]]:
    """(schedule, z-chunk) pairs: the separate passes (schedule 0; for a
    single handle also on 64 x 4 tiles on wide grids, schedule 6), and the
    fused variants 1-5 at each z-chunk."""
    out = [(0, 16)]  # the separate passes have no z-chunk
    if single:
        out.append((6, 16))
    for v in VARIANTS[1:]:
        for kc in KCHUNKS:
            if kc <= max(8, nz):
                out.append((v, kc))
    return out


def key(w, precision, batch: int = 1) -> str:
    pr = "f64" if precision == mpx.F64 else "f32"
    bc = "".join(str(b) for b in w.bc)
    pml = ",".join(str(v) for v in w.npml)
    ms = np.array([m[3] for m in w.materials], dtype=np.float64)
    nmag = int((ms[w.ids] > 0).sum())
    return f"{w.nx}x{w.ny}x{w.nz}:{pr}:bc{bc}:pml{pml}:magcells{nmag}:batch{batch}"


def _load(path: str) -> Dict:
    if path and os.path.exists(path):
        try:
            with open(path) as fh:
                return json.load(fh)
        except (OSError, ValueError):
            return {}
    return {}


def _store(path: str, data: Dict) -> None:
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_sims(step, sync, steps: int, repeats: int) -> float:
    step(4)
    sync()
    best = float("inf")
    for _ in range(repeats):
        t0 = time.perf_counter()
        step(steps)
        sync()
        best = min(best, time.perf_counter() - t0)
    return best / steps


def tune(w, precision=mpx.F32, steps: int = 40, repeats: int = 2, cache: Optional[str] = DEFAULT_CACHE,
         device: int = 0, force: bool = False, cands: Optional[Sequence[Tuple[int, int]]] = None):
    """(variant, kchunk, seconds per step) for workload ``w``; cached."""
    k = key(w, precision)
    data = _load(cache) if cache else {}
    if not force and k in data:
        e = data[k]
        return e["variant"], e["kchunk"], e["s_per_step"]
    s = mpx.from_workload(w, precision=precision, device=device, graph_steps=16)
    timings = {}
    try:
        for v, kc in (cands or candidates(w.nz, single=True)):
            s.set_schedule(v, kc)
            timings[(v, kc)] = _time_sims(s.step, s.sync, steps, repeats)
    finally:
        s.close()
    (v, kc), t = min(timings.items(), key=lambda it: it[1])
    if cache:
        data = _load(cache)
        data[k] = {"variant": v, "kchunk": kc, "s_per_step": t,
                   "all": {f"{a}:{b}": round(x, 9) for (a, b), x in sorted(timings.items())}}
        _store(cache, data)
    return v, kc, t


def tune_batch(ws: Iterable, precision=mpx.F32, steps: int = 20, repeats: int = 2,
               cache: Optional[str] = DEFAULT_CACHE, device: int = 0, force: bool = False,
               cands: Optional[Sequence[Tuple[int, int]]] = None):
    """(variant, kchunk, seconds per step) of a batch of workloads; cached
    under the key of its first member and the member count."""
    ws = list(ws)
    k = key(ws[0], precision, batch=len(ws)) + f":cells{sum(w.ncells for w in ws)}"
    data = _load(cache) if cache else {}
    if not force and k in data:
        e = data[k]
        return e["variant"], e["kchunk"], e["s_per_step"]
    sims = [mpx.from_workload(w, precision=precision, device=device) for w in ws]
    b = mpx.Batch(sims)
    b.set_graph_steps(16)
    timings = {}
    try:
        for v, kc in (cands or candidates(max(w.nz for w in ws))):
            b.set_schedule(v, kc)
            timings[(v, kc)] = _time_sims(b.step, b.sync, steps, repeats)
    finally:
        b.close()
        for s in sims:
            s.close()
    (v, kc), t = min(timings.items(), key=lambda it: it[1])
    if cache:
        data = _load(cache)
        data[k] = {"variant": v, "kchunk": kc, "s_per_step": t,
                   "all": {f"{a}:{b_}": round(x, 9) for (a, b_), x in sorted(timings.items())}}
        _store(cache, data)
    return v, kc, t
