"""The C-ABI library loads and exports every function include/mpx.h
declares; structure layouts of the binding match the header.  No compute
calls (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2510_22221_amd import mpx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "mpx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpx_[a-z_]+)\s*\(", text)))


def test_header_declarations_match_binding():
    assert declared() == sorted(mpx.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(mpx.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name


def test_abi_version():
    assert mpx.load().mpx_abi_version() == mpx.ABI_VERSION


def test_struct_layouts():
    # natural C layouts of the header structs on x86-64
    assert ctypes.sizeof(mpx.GridDesc) == 3 * 4 + 4 + 5 * 8 + 12 * 4 + 2 * 8
    assert ctypes.sizeof(mpx.Material) == 8 * 2 + 8 + 8 * 3
    assert ctypes.sizeof(mpx.SourceDesc) == 7 * 4 + 4 + 8 + 8
    assert ctypes.sizeof(mpx.ProbeDesc) == 7 * 4 + 4 + 8
    assert mpx.ProbeDesc.capacity.offset == 32


def test_create_rejects_bad_grid_without_touching_the_device():
    g = mpx.GridDesc()
    g.nx = 0
    h = ctypes.c_void_p()
    assert mpx.load().mpx_create(ctypes.byref(g), 0, 0, None, ctypes.byref(h)) == 1
    assert not h.value


def test_missing_library_fails_loudly(tmp_path):
    saved = mpx._lib
    mpx._lib = None
    try:
        with pytest.raises(RuntimeError, match="no CPU fallback"):
            mpx.load(str(tmp_path / "absent.so"))
    finally:
        mpx._lib = saved


def _grid(dt, courant=0.9, d=(1e-6, 2e-6, 1.5e-6)):
    g = mpx.GridDesc()
    g.nx, g.ny, g.nz = 8, 8, 8
    g.dx, g.dy, g.dz = d
    g.courant = courant
    g.dt = dt
    for a in range(6):
        g.bc[a] = 0
    return g


@pytest.mark.parametrize("factor", [1.0 + 1e-9, 1.5, float("inf")])
def test_create_rejects_dt_above_the_courant_limit_without_touching_the_device(factor):
    """An explicit dt above the 3-D Yee limit is refused before any device
    call (the library's own limit, compared with the oracle's formula)."""
    from oracle import oracle as O
    d = (1e-6, 2e-6, 1.5e-6)
    lim = O.courant_dt(1.0, *d)
    h = ctypes.c_void_p()
    g = _grid(lim * factor, d=d)
    assert mpx.load().mpx_create(ctypes.byref(g), 0, 0, None, ctypes.byref(h)) == 1
    assert not h.value


@pytest.mark.parametrize("courant", [0.0, -0.5, 1.01])
def test_create_rejects_courant_outside_the_unit_interval(courant):
    h = ctypes.c_void_p()
    g = _grid(0.0, courant=courant)
    assert mpx.load().mpx_create(ctypes.byref(g), 0, 0, None, ctypes.byref(h)) == 1
    assert not h.value
