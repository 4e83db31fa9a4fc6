"""ctypes wrapper around the FP64 CPU oracle (``oracle/mpx_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The oracle shares no code
with the HIP library and is never a fallback for it.

The wrapped scheme is arXiv:2510.22221, Methods, "Numerical Model": Ampere
(eq. Ampere and the semi-implicit E update), Faraday with B = mu0 (H + M)
(eq. iterate_H) and the trapezoidal Gilbert LLG (eqs. llg_tra4-llg_tra6),
on a Yee grid.  Arrays use numpy order [k, j, i] (x fastest in memory).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "mpx_oracle.c")

PEC, PML, PERIODIC = 0, 1, 2
PROBE_FIELD, PROBE_MEAN_M, PROBE_FILM_ENERGY = 0, 1, 2
EX, EY, EZ, HX, HY, HZ, MXF, MYF, MZF, DMXF, DMYF, DMZF = range(12)

C0 = 299792458.0
MU0 = 4e-7 * math.pi
EPS0 = 1.0 / (MU0 * C0 * C0)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off, OpenMP)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11",
             "-Wall", "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("dt", C.c_double),
                ("bc", C.c_int32 * 6), ("npml", C.c_int32 * 6),
                ("pml_order", C.c_double), ("pml_sigma_factor", C.c_double)]


class _Mat(C.Structure):
    _fields_ = [("eps_r", C.c_double), ("sigma", C.c_double), ("is_pec", C.c_int32),
                ("Ms", C.c_double), ("alpha", C.c_double), ("gamma_abs", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(_Grid)]
        L.orc_destroy.argtypes = [P]
        L.orc_set_materials.argtypes = [P, C.POINTER(_Mat), C.c_int, C.c_void_p]
        L.orc_set_bias.argtypes = [P, C.c_double, C.c_double, C.c_double]
        L.orc_init_magnetization.argtypes = [P, C.c_double, C.c_double, C.c_double]
        L.orc_add_source.argtypes = [P, C.c_int] + [C.c_int] * 6 + [C.c_void_p, C.c_int64]
        L.orc_add_probe.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64]
        L.orc_step.argtypes = [P, C.c_int64, C.c_int, C.c_double, C.c_int]
        L.orc_last_iterations.argtypes = [P]
        L.orc_field_dims.restype = C.c_int64
        L.orc_field_dims.argtypes = [P, C.c_int, C.POINTER(C.c_int32)]
        L.orc_get_field.argtypes = [P, C.c_int, C.c_void_p]
        L.orc_set_field.argtypes = [P, C.c_int, C.c_void_p]
        L.orc_read_probe.restype = C.c_int64
        L.orc_read_probe.argtypes = [P, C.c_int, C.c_void_p, C.c_int64]
        L.orc_energy.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_n_films.argtypes = [P]
        L.orc_film_box.argtypes = [P, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.orc_step_count.restype = C.c_int64
        L.orc_step_count.argtypes = [P]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        _lib = L
    return _lib


def courant_dt(courant: float, dx: float, dy: float, dz: float) -> float:
    """Yee stability limit scaled by the Courant number (Results, setup:
    a CFL factor of 0.9 gives the printed time step)."""
    return courant / (C0 * math.sqrt(1.0 / dx ** 2 + 1.0 / dy ** 2 + 1.0 / dz ** 2))


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_load().orc_get_threads())


class OracleSim:
    """One oracle instance.  ``bc`` is six of PEC/PML/PERIODIC for
    -x,+x,-y,+y,-z,+z; ``npml`` the PML thickness in cells per face."""

    def __init__(self, nx, ny, nz, d, dt, bc=(PEC,) * 6, npml=(0,) * 6, pml_order=3.0, pml_factor=0.8):
        L = _load()
        g = _Grid()
        g.nx, g.ny, g.nz = int(nx), int(ny), int(nz)
        g.dx, g.dy, g.dz = (float(v) for v in d)
        g.dt = float(dt)
        for a in range(6):
            g.bc[a] = int(bc[a])
            g.npml[a] = int(npml[a])
        g.pml_order = float(pml_order)
        g.pml_sigma_factor = float(pml_factor)
        self._p = L.orc_create(C.byref(g))
        if not self._p:
            raise ValueError("oracle rejected the grid")
        self._L = L
        self.shape = (int(nz), int(ny), int(nx))
        self.dt = float(dt)
        self.d = tuple(float(v) for v in d)

    def __del__(self):
        p = getattr(self, "_p", None)
        if p:
            self._L.orc_destroy(p)
            self._p = None

    def set_materials(self, table, ids):
        n = len(table)
        mats = (_Mat * n)()
        for q, m in enumerate(table):
            mats[q].eps_r, mats[q].sigma, mats[q].is_pec = float(m[0]), float(m[1]), int(m[2])
            mats[q].Ms, mats[q].alpha, mats[q].gamma_abs = float(m[3]), float(m[4]), float(m[5])
        ids = np.ascontiguousarray(ids, dtype=np.uint8)
        if ids.shape != self.shape:
            raise ValueError("ids must have shape (nz, ny, nx)")
        rc = self._L.orc_set_materials(self._p, mats, n, ids.ctypes.data)
        if rc != 0:
            raise ValueError(f"oracle rejected the materials (code {rc})")

    def set_bias(self, h0):
        self._L.orc_set_bias(self._p, *(float(v) for v in h0))

    def init_magnetization(self, u):
        rc = self._L.orc_init_magnetization(self._p, *(float(v) for v in u))
        if rc != 0:
            raise ValueError("init_magnetization failed")

    def add_source(self, comp, box, table):
        t = np.ascontiguousarray(table, dtype=np.float64)
        sid = self._L.orc_add_source(self._p, int(comp), *(int(b) for b in box), t.ctypes.data, t.size)
        if sid < 0:
            raise ValueError("add_source failed")
        return sid

    def add_probe(self, kind, field=0, ijk=(0, 0, 0), film=0, cap=1 << 16):
        pid = self._L.orc_add_probe(self._p, int(kind), int(field), *(int(v) for v in ijk), int(film), int(cap))
        if pid < 0:
            raise ValueError("add_probe failed")
        return pid

    def step(self, n, literal=False, tol=1e-6, rmax=50):
        rc = self._L.orc_step(self._p, int(n), 1 if literal else 0, float(tol), int(rmax))
        if rc == 3:
            raise RuntimeError("literal LLG iteration did not converge")
        if rc != 0:
            raise RuntimeError(f"oracle step failed ({rc})")

    @property
    def last_iterations(self):
        return int(self._L.orc_last_iterations(self._p))

    @property
    def step_count(self):
        return int(self._L.orc_step_count(self._p))

    def dims(self, field):
        d = (C.c_int32 * 4)()
        self._L.orc_field_dims(self._p, int(field), d)
        return tuple(int(v) for v in d)

    def get(self, field):
        nx, ny, nz, nc = self.dims(field)
        out = np.empty((nc, nz, ny, nx), dtype=np.float64)
        self._L.orc_get_field(self._p, int(field), out.ctypes.data)
        return out[0] if nc == 1 else out

    def set(self, field, arr):
        nx, ny, nz, nc = self.dims(field)
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(-1)
        if a.size != nx * ny * nz * nc:
            raise ValueError("wrong field size")
        self._L.orc_set_field(self._p, int(field), a.ctypes.data)

    def read_probe(self, pid, nval=None):
        cap = 1 << 24
        buf = np.empty(cap * 3, dtype=np.float64)
        n = self._L.orc_read_probe(self._p, int(pid), buf.ctypes.data, cap)
        if n < 0:
            raise ValueError("probe read failed")
        out = buf[: n * (nval or 1)] if nval else buf[:n]
        return out.reshape(n, nval) if nval and nval > 1 else out

    def energy(self):
        a, b = C.c_double(), C.c_double()
        self._L.orc_energy(self._p, C.byref(a), C.byref(b))
        return a.value, b.value

    def films(self):
        out = []
        for f in range(self._L.orc_n_films(self._p)):
            box = (C.c_int32 * 6)()
            nc = C.c_int64()
            self._L.orc_film_box(self._p, f, box, C.byref(nc))
            out.append((tuple(int(v) for v in box), int(nc.value)))
        return out


def from_workload(w, threads=None):
    """Build an oracle instance from a ``synth.workloads.Workload``."""
    if threads:
        set_threads(threads)
    s = OracleSim(w.nx, w.ny, w.nz, w.d, w.dt, w.bc, w.npml, w.pml_order, w.pml_factor)
    s.set_materials(w.materials, w.ids)
    s.set_bias(w.H0)
    s.init_magnetization(w.m_dir)
    for f, arr in (w.init_fields or {}).items():
        s.set(f, arr)
    for src in w.sources:
        s.add_source(src.comp, src.box, src.table)
    for p in w.probes:
        kind = {"field": PROBE_FIELD, "mean_m": PROBE_MEAN_M, "film_energy": PROBE_FILM_ENERGY}[p.kind]
        s.add_probe(kind, p.field, p.ijk, p.film, cap=max(1, p.cap or w.nsteps))
    return s
