"""ctypes binding of libmpx (include/mpx.h): argument marshalling only.

Every step of the coupled Yee + LLG update runs in the HIP kernels of
``libmpx.so``; this module converts Python/numpy/torch arguments to the C ABI
and back.  There is no fallback: if the shared library is missing or was not
built for this tree, loading raises.

PyTorch is optional plumbing: a torch stream can be handed to the library
(``stream=torch.cuda.current_stream()``) and fields can be read into, or
written from, CUDA tensors.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpx.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mpx.h")

F64, F32 = 0, 1
PEC, PML, PERIODIC = 0, 1, 2
EX, EY, EZ, HX, HY, HZ, MXF, MYF, MZF, DMXF, DMYF, DMZF = range(12)
PROBE_FIELD, PROBE_MEAN_M, PROBE_FILM_ENERGY, PROBE_EM_ENERGY = 0, 1, 2, 3
ABI_VERSION = 4

STATUS = {0: "MPX_OK", 1: "MPX_E_INVALID", 2: "MPX_E_STATE", 3: "MPX_E_NOMEM", 4: "MPX_E_DEVICE",
          5: "MPX_E_UNSUPPORTED", 6: "MPX_E_RANGE", 7: "MPX_E_NONFINITE"}

# every function the header declares (checked by the CPU test suite)
EXPORTS = ["mpx_abi_version", "mpx_create", "mpx_destroy", "mpx_query_field", "mpx_set_materials",
           "mpx_set_bias", "mpx_init_magnetization", "mpx_add_source", "mpx_add_probe", "mpx_step",
           "mpx_synchronize", "mpx_read_field", "mpx_read_field_region", "mpx_write_field", "mpx_field_storage", "mpx_read_probe", "mpx_energy", "mpx_energy_noalloc", "mpx_info",
           "mpx_film_box", "mpx_set_graph_steps", "mpx_set_schedule", "mpx_set_timing", "mpx_kernel_time",
           "mpx_last_error", "mpx_adjoint", "mpx_adjoint_probe", "mpx_set_adjoint_schedule", "mpx_set_adjoint_memory", "mpx_batch_create", "mpx_batch_destroy", "mpx_batch_set_schedule",
           "mpx_batch_set_graph_steps", "mpx_batch_step", "mpx_batch_synchronize", "mpx_batch_last_error"]


class MpxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("courant", C.c_double), ("dt", C.c_double),
                ("bc", C.c_int32 * 6), ("pml_cells", C.c_int32 * 6),
                ("pml_order", C.c_double), ("pml_sigma_factor", C.c_double)]


class Material(C.Structure):
    _fields_ = [("eps_r", C.c_double), ("sigma", C.c_double), ("is_pec", C.c_int32),
                ("Ms", C.c_double), ("alpha", C.c_double), ("gamma_abs", C.c_double)]


class SourceDesc(C.Structure):
    _fields_ = [("component", C.c_int32), ("i0", C.c_int32), ("j0", C.c_int32), ("k0", C.c_int32),
                ("ni", C.c_int32), ("nj", C.c_int32), ("nk", C.c_int32),
                ("table", C.c_void_p), ("n_table", C.c_int64)]


class ProbeDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("field", C.c_int32), ("i", C.c_int32), ("j", C.c_int32),
                ("k", C.c_int32), ("film", C.c_int32), ("every", C.c_int32), ("capacity", C.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libmpx.so; raises if it is absent (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libmpx.so not found at {path}: build it with paper_2510_22221_amd/build.py "
                           "(or __graft_entry__.build()); there is no CPU fallback")
    L = C.CDLL(path)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "mpx_abi_version": (C.c_uint32, []),
        "mpx_create": (I32, [C.POINTER(GridDesc), I32, I32, P, C.POINTER(P)]),
        "mpx_destroy": (I32, [P]),
        "mpx_query_field": (I32, [P, I32, C.POINTER(I64), C.POINTER(I64)]),
        "mpx_set_materials": (I32, [P, C.POINTER(Material), I32, P]),
        "mpx_set_bias": (I32, [P, D, D, D]),
        "mpx_init_magnetization": (I32, [P, D, D, D]),
        "mpx_add_source": (I32, [P, C.POINTER(SourceDesc), C.POINTER(I32)]),
        "mpx_add_probe": (I32, [P, C.POINTER(ProbeDesc), C.POINTER(I32)]),
        "mpx_step": (I32, [P, I64]),
        "mpx_synchronize": (I32, [P]),
        "mpx_read_field": (I32, [P, I32, P, I64, I32]),
        "mpx_read_field_region": (I32, [P, I32, C.POINTER(I32), P, I64, I32]),
        "mpx_write_field": (I32, [P, I32, P, I64, I32]),
        "mpx_field_storage": (I32, [P, I32, C.POINTER(P), C.POINTER(I64), C.POINTER(I64)]),
        "mpx_read_probe": (I32, [P, I32, P, I64, C.POINTER(I64)]),
        "mpx_energy": (I32, [P, C.POINTER(D), C.POINTER(D)]),
        "mpx_energy_noalloc": (I32, [P, C.POINTER(D), C.POINTER(D)]),
        "mpx_info": (I32, [P, C.POINTER(I64), C.POINTER(D), C.POINTER(D), C.POINTER(I32)]),
        "mpx_film_box": (I32, [P, I32, C.POINTER(I32), C.POINTER(I64)]),
        "mpx_set_graph_steps": (I32, [P, I32]),
        "mpx_set_schedule": (I32, [P, I32, I32]),
        "mpx_set_timing": (I32, [P, I32]),
        "mpx_kernel_time": (I32, [P, C.POINTER(D), C.POINTER(I64)]),
        "mpx_last_error": (C.c_char_p, [P]),
        "mpx_adjoint": (I32, [P, I64, I64, I32, I32, C.POINTER(I32), C.POINTER(I32), C.POINTER(D), C.POINTER(D),
                              P, P]),
        "mpx_adjoint_probe": (I32, [P, I64, I32, C.POINTER(I32), P, I32, C.POINTER(I32), C.POINTER(I32),
                                    C.POINTER(D), C.POINTER(D), P, P]),
        "mpx_set_adjoint_schedule": (I32, [P, I32]),
        "mpx_set_adjoint_memory": (I32, [P, C.c_int64]),
        "mpx_batch_create": (I32, [C.POINTER(P), I32, C.POINTER(P)]),
        "mpx_batch_destroy": (I32, [P]),
        "mpx_batch_set_schedule": (I32, [P, I32, I32]),
        "mpx_batch_set_graph_steps": (I32, [P, I32]),
        "mpx_batch_step": (I32, [P, I64]),
        "mpx_batch_synchronize": (I32, [P]),
        "mpx_batch_last_error": (C.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    if L.mpx_abi_version() != ABI_VERSION:
        raise RuntimeError("libmpx ABI version mismatch")
    _lib = L
    return L


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


class Sim:
    """One coupled Yee + LLG simulation on one GPU."""

    def __init__(self, nx, ny, nz, d, dt=0.0, courant=0.9, bc=(PEC,) * 6, npml=(0,) * 6, pml_order=3.0,
                 pml_factor=0.8, precision=F64, device=0, stream=None):
        self._L = load()
        g = GridDesc()
        g.nx, g.ny, g.nz = int(nx), int(ny), int(nz)
        g.dx, g.dy, g.dz = (float(v) for v in d)
        g.courant = float(courant)
        g.dt = float(dt)
        for a in range(6):
            g.bc[a] = int(bc[a])
            g.pml_cells[a] = int(npml[a])
        g.pml_order = float(pml_order)
        g.pml_sigma_factor = float(pml_factor)
        h = C.c_void_p()
        rc = self._L.mpx_create(C.byref(g), int(precision), int(device), _stream_ptr(stream), C.byref(h))
        if rc != 0:
            raise MpxError(rc, "mpx_create")
        self._h = h
        self.precision = precision
        self.shape = (int(nz), int(ny), int(nx))
        self.device = int(device)
        self.dtype = np.float64 if precision == F64 else np.float32

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.mpx_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ck(self, rc, what):
        if rc != 0:
            raise MpxError(rc, f"{what}: {self._L.mpx_last_error(self._h).decode()}")

    # ---- setup -------------------------------------------------------------
    def set_materials(self, table, ids):
        n = len(table)
        mats = (Material * n)()
        for q, m in enumerate(table):
            mats[q].eps_r, mats[q].sigma, mats[q].is_pec = float(m[0]), float(m[1]), int(m[2])
            mats[q].Ms, mats[q].alpha, mats[q].gamma_abs = float(m[3]), float(m[4]), float(m[5])
        ids = np.ascontiguousarray(ids, dtype=np.uint8)
        if ids.shape != self.shape:
            raise ValueError("ids must have shape (nz, ny, nx)")
        self._ck(self._L.mpx_set_materials(self._h, mats, n, ids.ctypes.data), "set_materials")

    def set_bias(self, h0):
        self._ck(self._L.mpx_set_bias(self._h, *(float(v) for v in h0)), "set_bias")

    def init_magnetization(self, u):
        self._ck(self._L.mpx_init_magnetization(self._h, *(float(v) for v in u)), "init_magnetization")

    def add_source(self, comp, box, table):
        t = np.ascontiguousarray(table, dtype=np.float64)
        sd = SourceDesc(int(comp), *(int(b) for b in box), t.ctypes.data, t.size)
        sid = C.c_int32()
        self._ck(self._L.mpx_add_source(self._h, C.byref(sd), C.byref(sid)), "add_source")
        return sid.value

    def add_probe(self, kind, field=0, ijk=(0, 0, 0), film=0, cap=1 << 16, every=1):
        """A probe sampled after every `every`-th step (see mpx_probe_desc)."""
        pd = ProbeDesc(int(kind), int(field), *(int(v) for v in ijk), int(film), int(every), int(cap))
        pid = C.c_int32()
        self._ck(self._L.mpx_add_probe(self._h, C.byref(pd), C.byref(pid)), "add_probe")
        return pid.value

    def set_graph_steps(self, n):
        self._ck(self._L.mpx_set_graph_steps(self._h, int(n)), "set_graph_steps")

    def set_timing(self, every):
        """0: off; n > 0: event-time every n-th step (launched directly; the
        steps between replay a captured graph)."""
        self._ck(self._L.mpx_set_timing(self._h, int(every)), "set_timing")

    # ---- stepping ------------------------------------------------------------
    def step(self, n):
        self._ck(self._L.mpx_step(self._h, int(n)), "step")

    def sync(self):
        self._ck(self._L.mpx_synchronize(self._h), "synchronize")

    def set_schedule(self, fused=True, kchunk=0):
        """fused: False/0 = separate E and H passes (the default); True/1 =
        register-blocked fused sweep; 2..5 = LDS-staged fused tile variants;
        6 = the separate passes on 64 x 4 tiles on wide grids too."""
        v = int(fused) if not isinstance(fused, bool) else (1 if fused else 0)
        self._ck(self._L.mpx_set_schedule(self._h, v, int(kchunk)), "set_schedule")

    def kernel_time(self):
        """[(avg ms per launch, launches)] of: the main stencil kernel, the
        second stencil kernel (two-pass schedule only), film + probe kernels."""
        ms = (C.c_double * 3)()
        n = (C.c_int64 * 3)()
        self._ck(self._L.mpx_kernel_time(self._h, ms, n), "kernel_time")
        return [(ms[q], n[q]) for q in range(3)]

    # ---- fields ------------------------------------------------------------------
    def dims(self, field):
        d = (C.c_int64 * 4)()
        nb = C.c_int64()
        self._ck(self._L.mpx_query_field(self._h, int(field), d, C.byref(nb)), "query_field")
        return tuple(int(v) for v in d), int(nb.value)

    def get(self, field, out=None):
        (nx, ny, nz, nc), nb = self.dims(field)
        dt = np.float64 if field >= 6 else self.dtype
        if out is not None and hasattr(out, "data_ptr"):  # torch CUDA tensor
            if out.numel() * out.element_size() < nb:
                raise ValueError("output tensor too small")
            self._ck(self._L.mpx_read_field(self._h, int(field), C.c_void_p(out.data_ptr()), nb, 1), "read_field")
            return out
        arr = np.empty((nc, nz, ny, nx), dtype=dt)
        self._ck(self._L.mpx_read_field(self._h, int(field), arr.ctypes.data, nb, 0), "read_field")
        return arr[0] if nc == 1 else arr

    def storage(self, field):
        """A torch tensor [nz, ny, nx] viewing the library's own storage of
        E or H component `field` (0..5), without a copy: writes through it
        change the simulation (order them with the handle's stream and keep
        PEC edges at zero)."""
        import torch
        ptr = C.c_void_p()
        st = (C.c_int64 * 3)()
        nb = C.c_int64()
        self._ck(self._L.mpx_field_storage(self._h, int(field), C.byref(ptr), st, C.byref(nb)), "field_storage")
        esz = np.dtype(self.dtype).itemsize
        shape = self.shape
        typestr = "<f8" if esz == 8 else "<f4"

        class _View:
            __cuda_array_interface__ = {"shape": shape, "typestr": typestr, "data": (ptr.value, False),
                                        "strides": (st[2] * esz, st[1] * esz, esz), "version": 3}
        return torch.as_tensor(_View(), device=f"cuda:{self.device}")

    def get_region(self, field, box):
        """Sub-box (i0, j0, k0, ni, nj, nk) of a field, numpy [k, j, i] (or
        [3, k, j, i] for the M fields)."""
        (_, _, _, nc), _ = self.dims(field)
        dt = np.float64 if field >= 6 else self.dtype
        b = (C.c_int32 * 6)(*(int(v) for v in box))
        arr = np.empty((nc, box[5], box[4], box[3]), dtype=dt)
        self._ck(self._L.mpx_read_field_region(self._h, int(field), b, arr.ctypes.data, arr.nbytes, 0),
                 "read_field_region")
        return arr[0] if nc == 1 else arr

    def set(self, field, arr):
        (nx, ny, nz, nc), nb = self.dims(field)
        if hasattr(arr, "data_ptr"):
            self._ck(self._L.mpx_write_field(self._h, int(field), C.c_void_p(arr.data_ptr()), nb, 1), "write_field")
            return
        dt = np.float64 if field >= 6 else self.dtype
        a = np.ascontiguousarray(arr, dtype=dt).reshape(-1)
        if a.size * a.itemsize != nb:
            raise ValueError("wrong field size")
        self._ck(self._L.mpx_write_field(self._h, int(field), a.ctypes.data, nb, 0), "write_field")

    def read_probe(self, pid, nval=1):
        n = C.c_int64()
        rc = self._L.mpx_read_probe(self._h, int(pid), None, 0, C.byref(n))
        if rc not in (0, 6):
            self._ck(rc, "read_probe")
        buf = np.empty(max(1, n.value) * nval, dtype=np.float64)
        self._ck(self._L.mpx_read_probe(self._h, int(pid), buf.ctypes.data, n.value, C.byref(n)), "read_probe")
        out = buf[: n.value * nval]
        return out.reshape(n.value, nval) if nval > 1 else out

    def energy(self):
        a, b = C.c_double(), C.c_double()
        self._ck(self._L.mpx_energy(self._h, C.byref(a), C.byref(b)), "energy")
        return a.value, b.value

    def energy_noalloc(self):
        """energy() through the entry point that allocates no device memory."""
        a, b = C.c_double(), C.c_double()
        self._ck(self._L.mpx_energy_noalloc(self._h, C.byref(a), C.byref(b)), "energy_noalloc")
        return a.value, b.value

    def info(self):
        st, t, dt, nf = C.c_int64(), C.c_double(), C.c_double(), C.c_int32()
        self._ck(self._L.mpx_info(self._h, C.byref(st), C.byref(t), C.byref(dt), C.byref(nf)), "info")
        return {"step": st.value, "time": t.value, "dt": dt.value, "films": nf.value}

    def adjoint(self, nsteps, loss_from, film=0, checkpoint_every=0, eps_box=(0, 0, 0, 0, 0, 0),
                ms_box=(0, 0, 0, 0, 0, 0)):
        """Run nsteps forward and return the film-energy loss with its
        gradients by the discrete adjoint: {"loss", "dH0" (3,), "deps"
        [nk, nj, ni] over eps_box, "dMs" [nk, nj, ni] over ms_box}."""
        eb = (C.c_int32 * 6)(*(int(v) for v in eps_box))
        mb = (C.c_int32 * 6)(*(int(v) for v in ms_box))
        loss = C.c_double()
        dh0 = (C.c_double * 3)()
        deps = np.zeros((eps_box[5], eps_box[4], eps_box[3]), dtype=np.float64)
        dms = np.zeros((ms_box[5], ms_box[4], ms_box[3]), dtype=np.float64)
        self._ck(self._L.mpx_adjoint(self._h, int(nsteps), int(loss_from), int(film), int(checkpoint_every), eb, mb,
                                     C.byref(loss), dh0, deps.ctypes.data if deps.size else None,
                                     dms.ctypes.data if dms.size else None), "adjoint")
        return {"loss": loss.value, "dH0": np.array(dh0[:]), "deps": deps, "dMs": dms}

    def adjoint_probe(self, nsteps, field, ijk, weights, checkpoint_every=0, eps_box=(0, 0, 0, 0, 0, 0),
                      ms_box=(0, 0, 0, 0, 0, 0)):
        """Run nsteps forward and return L = sum_i weights[i] E_field(ijk)
        after step i+1 with its gradients (same keys as adjoint)."""
        w = np.ascontiguousarray(weights, dtype=np.float64)
        if w.shape != (int(nsteps),):
            raise ValueError(f"weights must have shape ({int(nsteps)},), got {w.shape}")
        eb = (C.c_int32 * 6)(*(int(v) for v in eps_box))
        mb = (C.c_int32 * 6)(*(int(v) for v in ms_box))
        at = (C.c_int32 * 3)(*(int(v) for v in ijk))
        loss = C.c_double()
        dh0 = (C.c_double * 3)()
        deps = np.zeros((eps_box[5], eps_box[4], eps_box[3]), dtype=np.float64)
        dms = np.zeros((ms_box[5], ms_box[4], ms_box[3]), dtype=np.float64)
        self._ck(self._L.mpx_adjoint_probe(self._h, int(nsteps), int(field), at, w.ctypes.data,
                                           int(checkpoint_every), eb, mb, C.byref(loss), dh0,
                                           deps.ctypes.data if deps.size else None,
                                           dms.ctypes.data if dms.size else None), "adjoint_probe")
        return {"loss": loss.value, "dH0": np.array(dh0[:]), "deps": deps, "dMs": dms}

    def set_adjoint_schedule(self, schedule: int):
        """0: tape schedule (default; the two half-step transposes around an
        integer time in one pass where the films allow); 1: plain
        recompute-per-step schedule; 2: tape schedule with every half-step
        transpose in a pass of its own (same results as 0)."""
        self._ck(self._L.mpx_set_adjoint_schedule(self._h, int(schedule)), "set_adjoint_schedule")

    def set_adjoint_memory(self, max_bytes: int):
        """Device memory the tape schedule may keep forward tapes in: -1 (default)
        three quarters of the free memory, 0 none (every segment recomputed),
        > 0 a cap in bytes."""
        self._ck(self._L.mpx_set_adjoint_memory(self._h, int(max_bytes)), "set_adjoint_memory")

    def films(self):
        out = []
        for f in range(self.info()["films"]):
            box = (C.c_int32 * 6)()
            nc = C.c_int64()
            self._ck(self._L.mpx_film_box(self._h, f, box, C.byref(nc)), "film_box")
            out.append((tuple(int(v) for v in box), int(nc.value)))
        return out


class Batch:
    """Several simulations of one precision stepped together: one fused
    stencil launch per time step covers every member's tiles.  Members keep
    their own fields, probes and step counters; each ends bitwise equal to
    stepping it alone.  The members must stay alive and unconfigured while
    the batch exists."""

    def __init__(self, sims):
        self._L = load()
        self.sims = list(sims)
        arr = (C.c_void_p * len(self.sims))(*(s._h.value for s in self.sims))
        h = C.c_void_p()
        rc = self._L.mpx_batch_create(arr, len(self.sims), C.byref(h))
        if rc != 0:
            raise MpxError(rc, "mpx_batch_create")
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.mpx_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ck(self, rc, what):
        if rc != 0:
            raise MpxError(rc, f"{what}: {self._L.mpx_batch_last_error(self._h).decode()}")

    def set_schedule(self, variant=0, kchunk=0):
        """0: separate passes; 1..5: fused variants (as for Sim)."""
        self._ck(self._L.mpx_batch_set_schedule(self._h, int(variant), int(kchunk)), "batch_set_schedule")

    def set_graph_steps(self, n):
        self._ck(self._L.mpx_batch_set_graph_steps(self._h, int(n)), "batch_set_graph_steps")

    def step(self, n):
        self._ck(self._L.mpx_batch_step(self._h, int(n)), "batch_step")

    def sync(self):
        self._ck(self._L.mpx_batch_synchronize(self._h), "batch_synchronize")


def from_workload(w, precision=F64, device=0, stream=None, graph_steps=None, fused=None, kchunk=0):
    """Build a Sim from a ``synth.workloads.Workload`` (same inputs the
    oracle takes)."""
    s = Sim(w.nx, w.ny, w.nz, w.d, dt=w.dt, courant=w.courant, bc=w.bc, npml=w.npml, pml_order=w.pml_order,
            pml_factor=w.pml_factor, precision=precision, device=device, stream=stream)
    s.set_materials(w.materials, w.ids)
    s.set_bias(w.H0)
    s.init_magnetization(w.m_dir)
    for f, arr in (w.init_fields or {}).items():
        s.set(f, arr)
    for src in w.sources:
        s.add_source(src.comp, src.box, src.table)
    for p in w.probes:
        kind = {"field": PROBE_FIELD, "mean_m": PROBE_MEAN_M, "film_energy": PROBE_FILM_ENERGY,
                "em_energy": PROBE_EM_ENERGY}[p.kind]
        s.add_probe(kind, p.field, p.ijk, p.film, cap=max(1, p.cap or w.nsteps))
    if graph_steps is not None:
        s.set_graph_steps(graph_steps)
    if fused is not None or kchunk:
        s.set_schedule(True if fused is None else fused, kchunk)
    return s
