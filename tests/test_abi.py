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
