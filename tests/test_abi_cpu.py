"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the header declares, and rejects invalid arguments before any
device call."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2607_20650_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "lbm.h")).read()
    return sorted(set(re.findall(r"\b(lbm3?_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(lbm.LIB_PATH):
        pytest.skip("library not built")
    lib = lbm.load_library()
    names = _declared_symbols()
    assert "lbm_create" in names and "lbm_step" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(lbm.EXPORTED) <= set(names)


def _create(**over):
    lib = lbm.load_library()
    grid = lbm.Grid(over.get("nx", 16), over.get("ny", 8), over.get("scheme", 1), over.get("layout", 0),
                    over.get("precision", 0), over.get("tile_x", 0), over.get("tile_y", 0))
    bc = lbm.BC(over.get("x_axis", 0), over.get("y_axis", 0), (ctypes.c_double * 2)(0, 0),
                (ctypes.c_double * 2)(*over.get("g", (0, 0))), over.get("rho0", 1.0), (ctypes.c_double * 2)(0, 0),
                over.get("bounce", 0))
    flags = over["flags"] if "flags" in over else np.zeros((grid.ny if grid.ny > 0 else 1, max(grid.nx, 1)), np.uint8)
    out = ctypes.c_void_p(1234)
    st = lib.lbm_create(ctypes.byref(grid), flags.ctypes.data_as(ctypes.c_void_p), over.get("tau", 0.8),
                        ctypes.byref(bc), None, ctypes.byref(out))
    return st, out, lib.lbm_last_error(None).decode()


@pytest.mark.parametrize("over,needle", [
    ({"tau": 0.5}, "tau"),
    ({"tau": float("nan")}, "tau"),
    ({"nx": 0}, "nx"),
    ({"scheme": 9}, "scheme"),
    ({"layout": -1}, "layout"),
    ({"precision": 5}, "precision"),
    ({"x_axis": 7}, "x axis"),
    ({"y_axis": 2}, "y axis"),
    ({"rho0": 1.1}, "rho0"),
    ({"g": (float("inf"), 0)}, "finite"),
    ({"tile_x": 64, "tile_y": 32, "scheme": 3}, "tile"),
    ({"tile_x": 64, "tile_y": 80}, "tile"),
    ({"tile_x": 64, "tile_y": 0}, "tile"),
    ({"flags": np.full((8, 16), 2, np.uint8)}, "flags"),
    ({"nx": 1, "x_axis": 2, "flags": np.zeros((8, 1), np.uint8)}, "nx >= 2"),
    ({"nx": 1 << 30, "ny": 1 << 30, "flags": np.zeros((8, 16), np.uint8)}, "2^40 nodes"),  # before flags are read
    ({"bounce": 2}, "bounce"),
    ({"bounce": 1, "scheme": 3}, "two-lattice pull"),
    ({"bounce": 1, "x_axis": 3}, "full-way"),
])
def test_create_rejects_invalid_arguments(over, needle):
    if not os.path.exists(lbm.LIB_PATH):
        pytest.skip("library not built")
    st, out, msg = _create(**over)
    assert st == lbm.EINVAL
    assert out.value is None
    assert needle in msg


def test_null_safety():
    if not os.path.exists(lbm.LIB_PATH):
        pytest.skip("library not built")
    lib = lbm.load_library()
    lib.lbm_destroy(None)
    assert lib.lbm_step(None, 1) == lbm.EINVAL
    assert lib.lbm_sync(None) == lbm.EINVAL
    assert lib.lbm_macros(None, None, None, 0) == lbm.EINVAL
    out = ctypes.c_void_p()
    assert lib.lbm_create(None, None, 0.8, None, None, ctypes.byref(out)) == lbm.EINVAL
    assert lib.lbm_bytes_per_update(0) == 72 and lib.lbm_bytes_per_update(1) == 36


def _create3(**over):
    flags = over.pop("flags", np.zeros((4, 5, 6), np.uint8))
    nz, ny, nx = flags.shape
    g = lbm.Grid3(over.get("nx", nx), over.get("ny", ny), over.get("nz", nz), over.get("scheme", 1),
                  over.get("layout", 0), over.get("precision", 0), over.get("tile_x", 0), over.get("tile_y", 0))
    bc = lbm.BC3(over.get("x_axis", 0), over.get("y_axis", 0), over.get("z_axis", 0), (ctypes.c_double * 3)(0, 0, 0),
                 (ctypes.c_double * 3)(*over.get("g", (0, 0, 0))), over.get("rho0", 1.0),
                 (ctypes.c_double * 3)(0, 0, 0))
    lib = lbm.load_library()
    out = ctypes.c_void_p()
    st = lib.lbm3_create(ctypes.byref(g), flags.ctypes.data_as(ctypes.c_void_p), over.get("tau", 0.8),
                         ctypes.byref(bc), None, ctypes.byref(out))
    return st, out, lib.lbm3_last_error(None).decode()


@pytest.mark.parametrize("over,needle", [
    ({"tau": 0.5}, "tau"),
    ({"nz": 0}, "nz"),
    ({"scheme": 0}, "scheme"),
    ({"layout": 1}, "layout"),
    ({"precision": 5}, "precision"),
    ({"x_axis": 3}, "x axis"),
    ({"z_axis": 2}, "z axis"),
    ({"rho0": 1.1}, "rho0"),
    ({"g": (0, float("nan"), 0)}, "finite"),
    ({"tile_x": 64, "tile_y": 8}, "256 threads"),
    ({"nx": 1 << 20, "ny": 1 << 20, "nz": 1 << 20}, "2^40 nodes"),
    ({"tile_x": 64, "tile_y": 0}, "tile"),
    ({"flags": np.full((3, 4, 5), 2, np.uint8)}, "flags"),
])
def test_create3_rejects_invalid_arguments(over, needle):
    """The D3Q19 entry point validates before touching the device."""
    if not os.path.exists(lbm.LIB_PATH):
        pytest.skip("library not built")
    st, out, msg = _create3(**over)
    assert st == lbm.EINVAL
    assert out.value is None
    assert needle in msg


@pytest.mark.parametrize("mode,nbytes,aligned", [(-1, 64, True), (4, 64, True), (3, 0, True), (3, 24, True),
                                                (0, 64, False), (3, 64, False)])
def test_bandwidth_probe_rejects_bad_arguments(mode, nbytes, aligned):
    """Argument checks happen before any launch (no GPU needed): unknown mode,
    a size that is not a positive multiple of 16, misaligned pointers."""
    if not os.path.exists(lbm.LIB_PATH):
        pytest.skip("library not built")
    lib = lbm.load_library()
    base = 0x10000 if aligned else 0x10004
    st = lib.lbm_bandwidth_probe(mode, ctypes.c_void_p(base), ctypes.c_void_p(base + 0x1000), nbytes, None)
    assert st == lbm.EINVAL


def test_diag_noalloc_rejects_null_arguments():
    """Checked before any device call: no context, or no output."""
    if not os.path.exists(lbm.LIB_PATH):
        pytest.skip("library not built")
    lib = lbm.load_library()
    assert lib.lbm_diag_noalloc(None, None, 0, ctypes.c_void_p(0x10000)) == lbm.EINVAL
