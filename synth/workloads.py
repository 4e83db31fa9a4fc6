"""Seeded synthetic workloads shared by the oracle and the HIP library.

This module only *describes* inputs: grid sizes and spacings, the time step
chosen for a configuration, material tables and per-cell id maps, source
waveform tables, probe lists and (for physics tests) initial fields.  It
holds none of the time-stepping arithmetic, and neither side of a parity
test imports the other -- both read their inputs from here.

The paper's own runs (arXiv:2510.22221, Results, "Magnon-Photon Hybrid Quantum
Circuit Modeling Setup": a CPW resonator on silicon with a permalloy stripe,
PML on all faces, a modulated Gaussian voltage pulse) used data that is not
public; the configurations below are synthetic stand-ins with the same
structure (substrate + conductor strips + thin magnetic film + PML + pulse).
Every random draw uses numpy ``default_rng`` with the stated seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

SEED = 22221
C0 = 299792458.0
PEC, PML, PERIODIC = 0, 1, 2
EX, EY, EZ, HX, HY, HZ = range(6)

# material table rows: (eps_r, sigma [S/m], is_pec, Ms [A/m], alpha, |gamma| [rad/(s T)])
VACUUM = (1.0, 0.0, 0, 0.0, 0.0, 0.0)
SILICON = (11.7, 0.0, 0, 0.0, 0.0, 0.0)
PEC_METAL = (1.0, 0.0, 1, 0.0, 0.0, 0.0)
GAMMA = 1.76e11
FILM = (1.0, 0.0, 0, 1.4e5, 1e-4, GAMMA)
BASE_TABLE = [VACUUM, SILICON, PEC_METAL, FILM]


@dataclass
class Source:
    comp: int                      # 0..2 = Jx..Jz, on E_comp edges
    box: Tuple[int, int, int, int, int, int]  # i0, j0, k0, ni, nj, nk (E_comp index space)
    table: np.ndarray              # J(t_{n+1/2}) for n = 0.., float64


@dataclass
class Probe:
    kind: str                      # "field" | "mean_m" | "film_energy" | "em_energy"
    field: int = 0                 # 0..5 = Ex..Hz for kind "field"
    ijk: Tuple[int, int, int] = (0, 0, 0)
    film: int = 0
    cap: int = 0                   # 0 -> nsteps


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    d: Tuple[float, float, float]
    dt: float
    courant: float
    bc: Tuple[int, ...] = (PEC,) * 6
    npml: Tuple[int, ...] = (0,) * 6
    pml_order: float = 3.0
    pml_factor: float = 0.8
    materials: List[tuple] = field(default_factory=lambda: list(BASE_TABLE))
    ids: Optional[np.ndarray] = None           # uint8 [nz, ny, nx]
    H0: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    m_dir: Tuple[float, float, float] = (0.0, 0.0, 1.0)
    sources: List[Source] = field(default_factory=list)
    probes: List[Probe] = field(default_factory=list)
    nsteps: int = 0
    init_fields: Dict[int, np.ndarray] = field(default_factory=dict)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz


def config_dt(courant: float, d) -> float:
    """Time step of a configuration: the Courant number times the 3-D Yee
    limit, as the paper states its step (CFL factor 0.9)."""
    dx, dy, dz = d
    return courant / (C0 * math.sqrt(1.0 / dx ** 2 + 1.0 / dy ** 2 + 1.0 / dz ** 2))


def gaussian_pulse(n: int, dt: float, amp: float, f0: float, tp: float, t0: float) -> np.ndarray:
    """Modulated Gaussian excitation of the paper's setup section,
    amp * exp(-(t - t0)^2 / (2 tp^2)) * cos(2 pi f0 t), sampled at the
    half-integer times t_{n+1/2} = (n + 1/2) dt.  Host libm, float64."""
    t = (np.arange(n, dtype=np.float64) + 0.5) * dt
    return amp * np.exp(-((t - t0) ** 2) / (2.0 * tp * tp)) * np.cos(2.0 * math.pi * f0 * t)


def _empty_ids(nx, ny, nz) -> np.ndarray:
    return np.zeros((nz, ny, nx), dtype=np.uint8)


# --------------------------------------------------------------------------
# C1: plain 32^3 PEC box with a small perpendicular film and a point pulse
# --------------------------------------------------------------------------

def c1(nsteps: int = 2000) -> Workload:
    d = (1e-6, 1e-6, 1e-6)
    dt = config_dt(0.9, d)
    ids = _empty_ids(32, 32, 32)
    ids[15:17, 12:20, 12:20] = 3
    # the pulse is centred above the box's lowest cavity mode (c/(2L) sqrt(2)
    # = 6.6 THz for L = 32 um), so it excites cavity modes that stay in the
    # box; a pulse below cutoff is evanescent and leaves a field ~1e-3 of its
    # transient peak, which float32 storage of the peak cannot resolve to 1e-4
    f0 = 10e12
    table = gaussian_pulse(nsteps, dt, 1e12, f0, 1.0 / f0, 3.0 / f0)
    # E at the source cell, on the dipole's equatorial axis and above it; the
    # x and y components on the equatorial axis vanish by symmetry (their
    # traces are ~1e-2 of Ez there) and are not recorded
    probes = [Probe("field", comp, (8, 16, 16)) for comp in (EX, EY, EZ)]
    probes.append(Probe("field", EZ, (24, 16, 16)))
    probes += [Probe("field", comp, (16, 16, 24)) for comp in (EX, EY, EZ)]
    probes.append(Probe("mean_m", film=0))
    probes.append(Probe("film_energy", film=0))
    return Workload("C1 32^3 PEC box, 8x8x2 film, FP64", 32, 32, 32, d, dt, 0.9,
                    ids=ids, H0=(0.0, 0.0, 8e4), m_dir=(0.0, 0.0, 1.0),
                    sources=[Source(2, (8, 16, 16, 1, 1, 1), table)], probes=probes, nsteps=nsteps)


# --------------------------------------------------------------------------
# C2: single on-chip CPW resonator with a film, PML on all faces
# --------------------------------------------------------------------------

def c2(nsteps: int = 50000, nx: int = 512, ny: int = 256, nz: int = 128) -> Workload:
    """512x256x128 cells, d = (45, 2, 2) um, PML 10 on every face.
    Silicon (eps_r 11.7) below k = 40, a one-cell PEC layer at k = 40 patterned
    into a centre strip (60 cells wide) with 30-cell gaps to grounds that run
    into the y-PML; the strip is cut by 4-cell gap capacitors into a half-wave
    resonator tuned to the film's perpendicular FMR estimate; a 400x60x4 film
    sits on the strip at k = 41..44; H0 along z; a pulse on the gap edges at
    the feed end."""
    d = (45e-6, 2e-6, 2e-6)
    dt = config_dt(0.9, d)
    npml = 10
    ids = _empty_ids(nx, ny, nz)
    ksub, kmet = 40 * nz // 128, 40 * nz // 128
    ids[:ksub, :, :] = 1
    yc = ny // 2
    sw, gw = 60 * ny // 256, 30 * ny // 256
    s0, s1 = yc - sw // 2, yc - sw // 2 + sw
    # grounds from the y-PML up to the gaps
    ids[kmet, : s0 - gw, :] = 2
    ids[kmet, s1 + gw:, :] = 2
    # resonator length from the perpendicular Kittel estimate without static
    # demagnetisation, f = mu0 |gamma| H0 / (2 pi), eps_eff = 6.35
    H0 = 8e4
    f_k = 4e-7 * math.pi * GAMMA * H0 / (2.0 * math.pi)
    lres = int(round(C0 / (2.0 * f_k * d[0] * math.sqrt(6.35))))
    lres = min(lres, nx - 2 * npml - 20)
    x0 = (nx - lres) // 2
    gap = 4
    ids[kmet, s0:s1, : x0 - gap] = 2             # feed (into the -x PML)
    ids[kmet, s0:s1, x0:x0 + lres] = 2           # resonator
    ids[kmet, s0:s1, x0 + lres + gap:] = 2       # output feed (into the +x PML)
    fl = min(400 * nx // 512, lres - 8)
    fx0 = x0 + (lres - fl) // 2
    ids[kmet + 1:kmet + 5, s0:s1, fx0:fx0 + fl] = 3
    tp = 1.0 / f_k
    table = gaussian_pulse(nsteps, dt, 1e6, f_k, tp, 3.0 * tp)
    xi = npml + 1
    srcs = [Source(1, (xi, s0 - gw, kmet, 2, gw, 2), table),
            Source(1, (xi, s1, kmet, 2, gw, 2), -table)]
    probes = [Probe("field", EY, (x0 + 2, s0 - gw // 2, kmet + 1)),
              Probe("field", EY, (x0 + lres - 3, s0 - gw // 2, kmet + 1)),
              Probe("mean_m", film=0)]
    return Workload(f"C2 {nx}x{ny}x{nz} CPW resonator + film, PML {npml}", nx, ny, nz, d, dt, 0.9,
                    bc=(PML,) * 6, npml=(npml,) * 6, ids=ids, H0=(0.0, 0.0, H0),
                    m_dir=(0.0, 0.0, 1.0), sources=srcs, probes=probes, nsteps=nsteps)


# --------------------------------------------------------------------------
# C5: large single-GPU multi-resonator layout
# --------------------------------------------------------------------------

def c5(nsteps: int = 10000, nx: int = 1536, ny: int = 768, nz: int = 384, seed: int = SEED) -> Workload:
    """1536x768x384 cells, d = 2 um, PML 16.  eps_r drawn per 32^3 block from
    U[1, 12] and quantised to 1/16 (ids 4+), eight PEC strips 200x24 cells in a
    4x2 layout, each carrying a 200x40x4 film above it."""
    d = (2e-6, 2e-6, 2e-6)
    dt = config_dt(0.9, d)
    npml = 16
    rng = np.random.default_rng(seed)
    bz, by, bx = -(-nz // 32), -(-ny // 32), -(-nx // 32)
    q = np.round(rng.uniform(1.0, 12.0, size=(bz, by, bx)) * 16.0) / 16.0
    levels = np.unique(q)
    table = list(BASE_TABLE) + [(float(v), 0.0, 0, 0.0, 0.0, 0.0) for v in levels]
    lut = {float(v): 4 + n for n, v in enumerate(levels)}
    blk = np.vectorize(lambda v: lut[float(v)])(q).astype(np.uint8)
    ids = np.repeat(np.repeat(np.repeat(blk, 32, 0), 32, 1), 32, 2)[:nz, :ny, :nx].copy()
    kmet = nz // 2
    for r in range(8):
        cx = nx * (2 * (r % 4) + 1) // 8
        cy = ny * (2 * (r // 4) + 1) // 4
        sx0 = cx - 100
        ids[kmet, cy - 12:cy + 12, sx0:sx0 + 200] = 2
        ids[kmet + 1:kmet + 5, cy - 20:cy + 20, sx0:sx0 + 200] = 3
    tp = 1.0 / 3e9
    tab = gaussian_pulse(nsteps, dt, 1e6, 3e9, tp, 3 * tp)
    srcs = [Source(0, (nx // 8 - 100, ny // 4 - 20, kmet + 1, 200, 1, 1), tab)]
    probes = [Probe("mean_m", film=f) for f in range(8)]
    return Workload(f"C5 {nx}x{ny}x{nz} multi-resonator, 8 films, PML {npml}", nx, ny, nz, d, dt, 0.9,
                    bc=(PML,) * 6, npml=(npml,) * 6, materials=table, ids=ids, H0=(0.0, 0.0, 8e4),
                    m_dir=(0.0, 0.0, 1.0), sources=srcs, probes=probes, nsteps=nsteps)


# --------------------------------------------------------------------------
# small physics / parity cases
# --------------------------------------------------------------------------

def box(nx, ny, nz, d=(1e-6, 1e-6, 1e-6), courant=0.9, bc=(PEC,) * 6, npml=(0,) * 6, nsteps=0,
        name="box") -> Workload:
    """Empty vacuum box; tests fill in materials, sources and fields."""
    return Workload(name, nx, ny, nz, tuple(d), config_dt(courant, d), courant, bc=tuple(bc),
                    npml=tuple(npml), ids=_empty_ids(nx, ny, nz), nsteps=nsteps)


def random_case(seed: int, nx=13, ny=11, nz=9, bc=(PEC,) * 6, npml=(0,) * 6, film=True,
                sigma=True, nsteps=20) -> Workload:
    """Random dielectric/conductor/PEC cells, a film box, random initial E and
    H, a source -- the fixture for element-by-element single-step parity."""
    rng = np.random.default_rng(seed)
    w = box(nx, ny, nz, d=(1e-6 * (1 + rng.uniform()), 1e-6 * (1 + rng.uniform()), 1e-6), bc=bc, npml=npml,
            nsteps=nsteps, name=f"random seed {seed}")
    table = [VACUUM, (4.0, 0.0, 0, 0.0, 0.0, 0.0), PEC_METAL,
             (1.0, 0.0, 0, 1.4e5, 0.01, GAMMA),
             (7.0, 2e3 if sigma else 0.0, 0, 0.0, 0.0, 0.0),
             (2.5, 0.0, 0, 0.9e5, 0.003, 1.9e11)]
    w.materials = table
    ids = rng.choice([0, 1, 4], size=(nz, ny, nx), p=[0.6, 0.25, 0.15]).astype(np.uint8)
    # a few PEC cells away from the film
    ids[rng.integers(0, nz, 6), rng.integers(0, ny, 6), rng.integers(0, 3, 6)] = 2
    if film:
        fz0 = nz // 2 - 1
        ids[fz0:fz0 + 2, 3:ny - 3, 4:nx - 3] = 3
        ids[fz0, 4:6, 6:8] = 5
    w.ids = ids
    w.H0 = (2e4, -1e4, 6e4)
    w.m_dir = (0.3, 0.1, 1.0)
    w.sources = [Source(1, (2, 2, 2, 2, 3, 1), 1e9 * np.sin(np.arange(max(nsteps, 1)) * 0.3))]
    return w


# --------------------------------------------------------------------------
# C3: batched bias sweep, 64 resonator + film instances of uneven size
# --------------------------------------------------------------------------

def c3_instance(nx: int, ny: int, nz: int, h_scale: float, nsteps: int) -> Workload:
    """C2's stack scaled to (nx, ny, nz): silicon in the lower 40 % of nz, a
    one-cell PEC layer with a centre strip 12 cells wide (gaps of 8 cells to
    grounds that run into the y-PML), the strip a half-wave resonator of
    0.75 nx cells between 2-cell gap capacitors, a 0.6 nx x 12 x 4 film on it,
    PML 8 on every face, d = (20, 2, 2) um.  H0 along z is h_scale times the
    field whose perpendicular resonance (mu0 |gamma| H0 / 2 pi, no static
    demagnetisation) matches the resonator's half-wave estimate."""
    d = (20e-6, 2e-6, 2e-6)
    dt = config_dt(0.9, d)
    npml = 8
    ids = _empty_ids(nx, ny, nz)
    kmet = int(0.4 * nz)
    ids[:kmet] = 1
    yc = ny // 2
    sw, gw = 12, 8
    s0, s1 = yc - sw // 2, yc + sw // 2
    ids[kmet, : s0 - gw, :] = 2
    ids[kmet, s1 + gw:, :] = 2
    lres = int(0.75 * nx)
    x0 = (nx - lres) // 2
    ids[kmet, s0:s1, : x0 - 2] = 2
    ids[kmet, s0:s1, x0:x0 + lres] = 2
    ids[kmet, s0:s1, x0 + lres + 2:] = 2
    fl = int(0.6 * nx)
    fx0 = x0 + (lres - fl) // 2
    ids[kmet + 1:kmet + 5, s0:s1, fx0:fx0 + fl] = 3
    f_p = C0 / (2.0 * lres * d[0] * math.sqrt(6.35))
    H_ac = 2.0 * math.pi * f_p / (4e-7 * math.pi * GAMMA)
    tp = 1.0 / f_p
    table = gaussian_pulse(nsteps, dt, 1e6, f_p, tp, 3.0 * tp)
    srcs = [Source(1, (npml + 1, s0 - gw, kmet, 2, gw, 2), table),
            Source(1, (npml + 1, s1, kmet, 2, gw, 2), -table)]
    probes = [Probe("mean_m", film=0), Probe("field", EY, (x0 + 2, s0 - gw // 2, kmet + 1))]
    return Workload(f"C3 instance {nx}x{ny}x{nz}, H0 = {h_scale:.3f} H_ac", nx, ny, nz, d, dt, 0.9,
                    bc=(PML,) * 6, npml=(npml,) * 6, ids=ids, H0=(0.0, 0.0, h_scale * H_ac),
                    m_dir=(0.0, 0.0, 1.0), sources=srcs, probes=probes, nsteps=nsteps)


def c3(nsteps: int = 20000, n: int = 64, seed: int = SEED) -> List[Workload]:
    """The bias sweep: nx = 64 + 16 U{0..8}, ny = 64 + 16 U{0..2}, nz = 64
    from the seed; H0_i = H_ac (0.8 + 0.4 i/(n-1))."""
    rng = np.random.default_rng(seed)
    nxs = 64 + 16 * rng.integers(0, 9, size=n)
    nys = 64 + 16 * rng.integers(0, 3, size=n)
    return [c3_instance(int(nxs[i]), int(nys[i]), 64, 0.8 + 0.4 * i / max(1, n - 1), nsteps) for i in range(n)]


def scaled_drive(w: Workload, factor: float) -> Workload:
    """The drive-power variant of a workload: every source table multiplied
    by `factor` (the excitation-intensity sweep of the paper's nonlinear
    spectra); all other inputs shared."""
    import copy

    out = copy.copy(w)
    out.sources = [Source(s.comp, s.box, np.asarray(s.table) * factor) for s in w.sources]
    out.probes = list(w.probes)
    out.name = f"{w.name}, drive x{factor:g}"
    return out


# --------------------------------------------------------------------------
# C4: the adjoint workload (film-energy loss, gradients w.r.t. H0, eps_r of a
# substrate patch and the film's top-layer Ms)
# --------------------------------------------------------------------------

def c4_instance(nx: int = 128, ny: int = 64, nz: int = 64, nsteps: int = 20000, npml: int = 8) -> Workload:
    """C2's stack at (nx, ny, nz), d = (40, 2, 2) um: silicon below k = 20 nz/64,
    a PEC layer at that height with a 12-cell centre strip (gaps of 8 cells to
    grounds), the strip a half-wave resonator of 0.75 nx cells, a film of
    0.5 nx x 12 x 4 cells on it, and an eps_r patch of 0.25 nx x 16 x 4 cells
    in the substrate under the film centre (its own material id, eps_r 11.7,
    so that its cells can be perturbed one by one).  H0 along z at the
    resonator's perpendicular-FMR estimate; a pulse on the feed gaps."""
    d = (40e-6, 2e-6, 2e-6)
    dt = config_dt(0.9, d)
    ids = _empty_ids(nx, ny, nz)
    kmet = 20 * nz // 64
    ids[:kmet] = 1
    yc = ny // 2
    sw, gw = 12, 8
    s0, s1 = yc - sw // 2, yc + sw // 2
    ids[kmet, : s0 - gw, :] = 2
    ids[kmet, s1 + gw:, :] = 2
    lres = int(0.75 * nx)
    x0 = (nx - lres) // 2
    ids[kmet, s0:s1, : x0 - 2] = 2
    ids[kmet, s0:s1, x0:x0 + lres] = 2
    ids[kmet, s0:s1, x0 + lres + 2:] = 2
    fl = nx // 2
    fx0 = (nx - fl) // 2
    ids[kmet + 1:kmet + 5, s0:s1, fx0:fx0 + fl] = 3
    pw, ph = nx // 4, 16
    px0, py0 = (nx - pw) // 2, yc - ph // 2
    ids[kmet - 4:kmet, py0:py0 + ph, px0:px0 + pw] = 4
    mats = [VACUUM, (11.7, 0.0, 0, 0.0, 0.0, 0.0), PEC_METAL, (1.0, 0.0, 0, 1.4e5, 1e-4, GAMMA),
            (11.7, 0.0, 0, 0.0, 0.0, 0.0)]
    f_p = C0 / (2.0 * lres * d[0] * math.sqrt(6.35))
    H_ac = 2.0 * math.pi * f_p / (4e-7 * math.pi * GAMMA)
    tp = 1.0 / f_p
    table = gaussian_pulse(nsteps, dt, 1e6, f_p, tp, 3.0 * tp)
    srcs = [Source(1, (npml + 1, s0 - gw, kmet, 2, gw, 2), table),
            Source(1, (npml + 1, s1, kmet, 2, gw, 2), -table)]
    w = Workload(f"C4 {nx}x{ny}x{nz} resonator + film, eps patch", nx, ny, nz, d, dt, 0.9,
                 bc=(PML,) * 6, npml=(npml,) * 6, ids=ids, H0=(0.0, 0.0, H_ac),
                 m_dir=(0.0, 0.0, 1.0), sources=srcs, probes=[Probe("film_energy", film=0)], nsteps=nsteps)
    w.materials = mats
    w.patch_box = (px0, py0, kmet - 4, pw, ph, 4)
    w.film_top = (fx0, s0, kmet + 4, fl, sw, 1)
    return w


def c4(nsteps: int = 20000) -> Workload:
    return c4_instance(128, 64, 64, nsteps)


def crop(w: Workload, lo: Tuple[int, int, int], size: Tuple[int, int, int], name: str = "") -> Workload:
    """A sub-box of a workload's grid (x, y, z origin `lo`, cell counts
    `size`) with the same materials, boundaries and PML depth; sources that
    lie wholly inside move with it, probes are dropped.  A bounded sample of a
    large configuration for timing the oracle on the host."""
    (i0, j0, k0), (nx, ny, nz) = lo, size
    ids = None if w.ids is None else w.ids[k0:k0 + nz, j0:j0 + ny, i0:i0 + nx].copy()
    srcs = []
    for s in w.sources:
        a, b, c, ni, nj, nk = s.box
        if a >= i0 and b >= j0 and c >= k0 and a + ni <= i0 + nx and b + nj <= j0 + ny and c + nk <= k0 + nz:
            srcs.append(Source(s.comp, (a - i0, b - j0, c - k0, ni, nj, nk), s.table))
    return Workload(name or f"{w.name} [crop {nx}x{ny}x{nz} at {lo}]", nx, ny, nz, w.d, w.dt, w.courant,
                    bc=w.bc, npml=w.npml, pml_order=w.pml_order, pml_factor=w.pml_factor,
                    materials=list(w.materials), ids=ids, H0=w.H0, m_dir=w.m_dir, sources=srcs, probes=[],
                    nsteps=w.nsteps)
