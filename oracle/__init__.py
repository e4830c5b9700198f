"""FP64 CPU oracle for the D2Q9I BGK lattice update (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library;
the C source ``lbm_oracle.c`` is compiled here with the host C compiler.

Definitions followed (paper Section 3.1, Eq. 1-2; Section 3.3 two-lattice
one-step pull): see the header of ``lbm_oracle.c``.

Array conventions of this wrapper:
  * flags / types: uint8 (ny, nx)
  * populations:   float64 (9, ny, nx), direction order of Fig. 2 (b)
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
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

FLUID, SOLID, INLET, OUTLET = 0, 1, 2, 3
PERIODIC, CLOSED, INFLOW_OUTFLOW, INFLOW_PRESSURE, NEUMANN_OUTFLOW, NEUMANN_PRESSURE = 0, 1, 2, 3, 4, 5


def build(force: bool = False) -> str:
    """Compile lbm_oracle.c into liboracle.so (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-fno-fast-math",
               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("x_axis", ctypes.c_int32), ("y_axis", ctypes.c_int32),
                ("tau", ctypes.c_double),
                ("u_in", ctypes.c_double * 2), ("g", ctypes.c_double * 2), ("u0", ctypes.c_double * 2),
                ("fullway", ctypes.c_int32), ("pad", ctypes.c_int32)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.POINTER(_Params)
            u8 = ctypes.POINTER(ctypes.c_uint8)
            d = ctypes.POINTER(ctypes.c_double)
            for name, args in {
                "ora_node_types": [P, u8, u8],
                "ora_init_state": [P, u8, d],
                "ora_gather": [P, u8, d, d],
                "ora_run": [P, u8, d, d, ctypes.c_int64],
                "ora_readout": [P, u8, d, d, d, d],
            }.items():
                fn = getattr(lib, name)
                fn.argtypes = args
                fn.restype = ctypes.c_int
            lib.ora_equilibrium.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, d]
            lib.ora_equilibrium.restype = None
            lib.ora_constants.argtypes = [ctypes.POINTER(ctypes.c_int)] * 3 + [d]
            lib.ora_constants.restype = None
            lib.ora_max_threads.restype = ctypes.c_int
            lib.ora_set_threads.argtypes = [ctypes.c_int]
            lib.ora_set_threads.restype = None
            _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8ptr(a: np.ndarray):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def constants():
    """(cx, cy, opp, w) exactly as the oracle uses them."""
    lib = _load()
    cx = (ctypes.c_int * 9)()
    cy = (ctypes.c_int * 9)()
    opp = (ctypes.c_int * 9)()
    w = np.zeros(9)
    lib.ora_constants(cx, cy, opp, _dptr(w))
    return np.array(cx[:]), np.array(cy[:]), np.array(opp[:]), w


def equilibrium(rho: float, vx: float, vy: float) -> np.ndarray:
    lib = _load()
    out = np.zeros(9)
    lib.ora_equilibrium(float(rho), float(vx), float(vy), _dptr(out))
    return out


def threads() -> int:
    return int(_load().ora_max_threads())


def set_threads(n: int) -> None:
    _load().ora_set_threads(int(n))


@dataclass
class Oracle:
    """Plain two-lattice pull simulation in FP64."""

    flags: np.ndarray
    tau: float
    x_axis: int = PERIODIC
    y_axis: int = PERIODIC
    u_in: tuple = (0.0, 0.0)
    g: tuple = (0.0, 0.0)
    u0: tuple = (0.0, 0.0)
    fullway: bool = False  # full-way bounce-back at solid nodes (halfway otherwise)

    def __post_init__(self):
        self.flags = np.ascontiguousarray(self.flags, dtype=np.uint8)
        self.ny, self.nx = self.flags.shape
        p = _Params()
        p.nx, p.ny = self.nx, self.ny
        p.x_axis, p.y_axis = int(self.x_axis), int(self.y_axis)
        p.tau = float(self.tau)
        p.u_in[0], p.u_in[1] = map(float, self.u_in)
        p.g[0], p.g[1] = map(float, self.g)
        p.u0[0], p.u0[1] = map(float, self.u0)
        p.fullway = int(bool(self.fullway))
        self._p = p
        self.types = np.zeros_like(self.flags)
        _load().ora_node_types(ctypes.byref(p), _u8ptr(self.flags), _u8ptr(self.types))
        # internal state, node-major [ny][nx][9]
        self._f = np.zeros((self.ny, self.nx, 9))
        self._tmp = np.zeros_like(self._f)
        _load().ora_init_state(ctypes.byref(p), _u8ptr(self.types), _dptr(self._f))
        self.t = 0

    @classmethod
    def from_scenario(cls, sc, fullway: bool = False) -> "Oracle":
        return cls(sc.flags, sc.tau, sc.x_axis, sc.y_axis, sc.u_in, sc.g, sc.u0, fullway)

    # -- state -------------------------------------------------------------
    @property
    def state(self) -> np.ndarray:
        """Pull state (post-collision, not yet streamed), shape (9, ny, nx)."""
        return np.ascontiguousarray(self._f.transpose(2, 0, 1))

    def set_state(self, f: np.ndarray) -> None:
        """Replace the pull state with f (9, ny, nx); inlet nodes are reset to
        feq(1, u_in) and solid nodes to 0, as the model keeps them fixed (with
        full-way bounce-back solid nodes hold state and keep the loaded values)."""
        f = np.asarray(f, dtype=np.float64)
        assert f.shape == (9, self.ny, self.nx)
        self._f[...] = f.transpose(1, 2, 0)
        ein = equilibrium(1.0, *self.u_in)
        self._f[self.types == INLET] = ein
        if not self.fullway:
            self._f[self.types == SOLID] = 0.0

    # -- dynamics ----------------------------------------------------------
    def run(self, steps: int) -> "Oracle":
        _load().ora_run(ctypes.byref(self._p), _u8ptr(self.types), _dptr(self._f), _dptr(self._tmp), int(steps))
        self.t += int(steps)
        return self

    def incoming(self) -> np.ndarray:
        """Pre-collision incoming populations at the current time, (9, ny, nx)."""
        fin = np.zeros_like(self._f)
        _load().ora_gather(ctypes.byref(self._p), _u8ptr(self.types), _dptr(self._f), _dptr(fin))
        return np.ascontiguousarray(fin.transpose(2, 0, 1))

    def macros(self):
        """(rho, ux, uy), each (ny, nx) float64."""
        rho = np.zeros((self.ny, self.nx))
        ux = np.zeros_like(rho)
        uy = np.zeros_like(rho)
        _load().ora_readout(ctypes.byref(self._p), _u8ptr(self.types), _dptr(self._f), _dptr(rho), _dptr(ux),
                            _dptr(uy))
        return rho, ux, uy
