"""FP64 CPU oracle for the D3Q19 extension (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP library;
``d3q19_oracle.c`` is compiled here with the host C compiler.

Array conventions:
  * flags / types: uint8 (nz, ny, nx)
  * populations:   float64 (19, nz, ny, nx), velocities ordered by
                   (c_z, c_y, c_x) lexicographically (rest = 9, opposite = 18 - i)
  * pull state:    post-collision values that have not streamed yet
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "d3q19_oracle.c")
_LIB = os.path.join(_HERE, "liboracle3.so")
_lock = threading.Lock()
_lib = None

FLUID, SOLID, INLET, OUTLET = 0, 1, 2, 3
PERIODIC, CLOSED, INFLOW_OUTFLOW = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile d3q19_oracle.c into liboracle3.so (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-fno-fast-math",
               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("x_axis", ctypes.c_int32), ("y_axis", ctypes.c_int32), ("z_axis", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("tau", ctypes.c_double),
                ("u_in", ctypes.c_double * 3), ("g", ctypes.c_double * 3), ("u0", ctypes.c_double * 3)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.POINTER(_Params)
            u8 = ctypes.POINTER(ctypes.c_uint8)
            d = ctypes.POINTER(ctypes.c_double)
            for name, args in [("ora3_node_types", [P, u8, u8]), ("ora3_init_state", [P, u8, d]),
                               ("ora3_gather", [P, u8, d, d]), ("ora3_run", [P, u8, d, d, ctypes.c_int64]),
                               ("ora3_readout", [P, u8, d, d, d])]:
                fn = getattr(lib, name)
                fn.argtypes = args
                fn.restype = ctypes.c_int
            lib.ora3_equilibrium.argtypes = [ctypes.c_double] * 4 + [d]
            lib.ora3_equilibrium.restype = None
            lib.ora3_constants.argtypes = [ctypes.POINTER(ctypes.c_int)] * 3 + [d]
            lib.ora3_constants.restype = None
            _lib = lib
        return _lib


def _dptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8ptr(a):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def constants():
    """(cx, cy, cz, w) of the 19 velocities in the oracle's order."""
    c = [(ctypes.c_int * 19)() for _ in range(3)]
    w = np.zeros(19)
    _load().ora3_constants(c[0], c[1], c[2], _dptr(w))
    return np.array(c[0][:]), np.array(c[1][:]), np.array(c[2][:]), w


def equilibrium(rho, ux, uy, uz) -> np.ndarray:
    out = np.zeros(19)
    _load().ora3_equilibrium(float(rho), float(ux), float(uy), float(uz), _dptr(out))
    return out


@dataclass
class Oracle3:
    flags: np.ndarray
    tau: float
    x_axis: int = PERIODIC
    y_axis: int = PERIODIC
    z_axis: int = PERIODIC
    u_in: tuple = (0.0, 0.0, 0.0)
    g: tuple = (0.0, 0.0, 0.0)
    u0: tuple = (0.0, 0.0, 0.0)

    def __post_init__(self):
        self.flags = np.ascontiguousarray(self.flags, dtype=np.uint8)
        self.nz, self.ny, self.nx = self.flags.shape
        self.types = np.zeros_like(self.flags)
        self.t = 0
        n = self.flags.size
        self._f = np.zeros(n * 19)
        self._tmp = np.zeros(n * 19)
        _load().ora3_node_types(ctypes.byref(self._params()), _u8ptr(self.flags), _u8ptr(self.types))
        _load().ora3_init_state(ctypes.byref(self._params()), _u8ptr(self.types), _dptr(self._f))

    def _params(self):
        p = _Params()
        p.nx, p.ny, p.nz = self.nx, self.ny, self.nz
        p.x_axis, p.y_axis, p.z_axis = int(self.x_axis), int(self.y_axis), int(self.z_axis)
        p.tau = float(self.tau)
        for k in range(3):
            p.u_in[k], p.g[k], p.u0[k] = float(self.u_in[k]), float(self.g[k]), float(self.u0[k])
        return p

    @classmethod
    def from_scenario(cls, sc) -> "Oracle3":
        return cls(sc.flags, sc.tau, sc.x_axis, sc.y_axis, sc.z_axis, sc.u_in, sc.g, sc.u0)

    @property
    def state(self) -> np.ndarray:
        """Pull state (19, nz, ny, nx)."""
        return np.ascontiguousarray(self._f.reshape(-1, 19).T.reshape(19, self.nz, self.ny, self.nx))

    def set_state(self, f) -> None:
        """Replace the pull state (19, nz, ny, nx); inlet nodes are reset to
        feq(1, u_in) and solid nodes to 0."""
        f = np.asarray(f, np.float64).reshape(19, -1)
        self._f[...] = np.ascontiguousarray(f.T).ravel()
        fv = self._f.reshape(-1, 19)
        t = self.types.ravel()
        fv[t == INLET] = equilibrium(1.0, *self.u_in)
        fv[t == SOLID] = 0.0

    def run(self, steps: int) -> "Oracle3":
        _load().ora3_run(ctypes.byref(self._params()), _u8ptr(self.types), _dptr(self._f), _dptr(self._tmp),
                         int(steps))
        self.t += int(steps)
        return self

    def incoming(self) -> np.ndarray:
        """Incoming populations (19, nz, ny, nx) of the current state."""
        out = np.zeros_like(self._f)
        _load().ora3_gather(ctypes.byref(self._params()), _u8ptr(self.types), _dptr(self._f), _dptr(out))
        return np.ascontiguousarray(out.reshape(-1, 19).T.reshape(19, self.nz, self.ny, self.nx))

    def macros(self):
        """rho (nz, ny, nx) and u (3, nz, ny, nx)."""
        n = self.flags.size
        rho, u = np.zeros(n), np.zeros(3 * n)
        _load().ora3_readout(ctypes.byref(self._params()), _u8ptr(self.types), _dptr(self._f), _dptr(rho),
                             _dptr(u))
        shp = (self.nz, self.ny, self.nx)
        return rho.reshape(shp), u.reshape((3,) + shp)
