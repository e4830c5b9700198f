"""Python binding of the C ABI in include/lbm.h (ctypes; argument marshalling only).

Every step of the lattice update runs in the gfx950 HIP kernels of
``liblbm.so``; this module only converts arguments, allocates output buffers
with PyTorch (device memory) and passes PyTorch's current HIP stream to the
library.  There is no fallback: if the library is missing the import of
:class:`Simulation` fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

# enum values of include/lbm.h
OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, EBUSY, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
SCHEMES = {"LPTL": 0, "NPTL": 1, "PUSH": 2, "NPOL": 3, "NSOL": 4, "AA": 5}
LAYOUTS = {"stream": 0, "bundle": 1, "collision": 2, "blocked": 3}
PRECISIONS = {"fp32": 0, "fp16s": 1, "fp16sr": 2, "fp16c": 3, "fp16csr": 4}
PERIODIC, CLOSED, INFLOW_OUTFLOW, INFLOW_PRESSURE, NEUMANN_OUTFLOW, NEUMANN_PRESSURE = 0, 1, 2, 3, 4, 5
STATUS_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE", -4: "LBM_EUNSTABLE",
                -5: "LBM_EBUSY", -6: "LBM_ENOTFOUND"}

EXPORTED = ["lbm_create", "lbm_step", "lbm_macros", "lbm_diag", "lbm_get_populations", "lbm_set_state",
            "lbm_get_info", "lbm_set_bundle", "lbm_sync", "lbm_last_error", "lbm_destroy", "lbm_bytes_per_update",
            "lbm_bandwidth_probe", "lbm_diag_noalloc", "lbm_server_create", "lbm_server_submit", "lbm_server_run_bundle",
            "lbm_server_poll", "lbm_server_fetch", "lbm_server_get_stats", "lbm_server_last_error",
            "lbm_server_destroy", "lbm3_create", "lbm3_step", "lbm3_macros", "lbm3_get_populations",
            "lbm3_set_state", "lbm3_diag", "lbm3_sync", "lbm3_last_error", "lbm3_destroy", "lbm3_bytes_per_update"]


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("scheme", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("precision", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("tile_y", ctypes.c_int32)]


class BC(ctypes.Structure):
    _fields_ = [("x_axis", ctypes.c_int32), ("y_axis", ctypes.c_int32), ("u_in", ctypes.c_double * 2),
                ("g", ctypes.c_double * 2), ("rho0", ctypes.c_double), ("u0", ctypes.c_double * 2),
                ("bounce", ctypes.c_int32)]


HALFWAY, FULLWAY = 0, 1


class Info(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("pitch", ctypes.c_int64),
                ("scheme", ctypes.c_int32), ("layout", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("block", ctypes.c_int32),
                ("bundle", ctypes.c_int32), ("device_bytes", ctypes.c_int64), ("fluid_nodes", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int32), ("running", ctypes.c_int32), ("finished_unfetched", ctypes.c_int32),
                ("pool_bytes", ctypes.c_int64), ("pool_used", ctypes.c_int64), ("bundles", ctypes.c_int64),
                ("node_updates", ctypes.c_int64)]


class Grid3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64), ("scheme", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("precision", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("tile_y", ctypes.c_int32)]


class BC3(ctypes.Structure):
    _fields_ = [("x_axis", ctypes.c_int32), ("y_axis", ctypes.c_int32), ("z_axis", ctypes.c_int32),
                ("u_in", ctypes.c_double * 3), ("g", ctypes.c_double * 3), ("rho0", ctypes.c_double),
                ("u0", ctypes.c_double * 3)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblbm.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run __graft_entry__.build() first")
    try:
        import torch  # noqa: F401  (HIP runtime first, shared by both)
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    sig = {
        "lbm_create": ([ctypes.POINTER(Grid), ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(BC), P,
                        ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
        "lbm_step": ([P, ctypes.c_int64], ctypes.c_int),
        "lbm_macros": ([P, P, P, ctypes.c_int], ctypes.c_int),
        "lbm_diag": ([P, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "lbm_get_populations": ([P, P, ctypes.c_int], ctypes.c_int),
        "lbm_set_state": ([P, P, ctypes.c_int], ctypes.c_int),
        "lbm_get_info": ([P, ctypes.POINTER(Info)], ctypes.c_int),
        "lbm_set_bundle": ([P, ctypes.c_int32], ctypes.c_int),
        "lbm_sync": ([P], ctypes.c_int),
        "lbm_last_error": ([P], ctypes.c_char_p),
        "lbm_destroy": ([P], None),
        "lbm_bytes_per_update": ([ctypes.c_int32], ctypes.c_int32),
        "lbm_bandwidth_probe": ([ctypes.c_int32, P, P, ctypes.c_int64, P], ctypes.c_int),
        "lbm_diag_noalloc": ([P, P, ctypes.c_int32, P], ctypes.c_int),
        "lbm_server_create": ([ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P,
                               ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
        "lbm_server_submit": ([P, ctypes.POINTER(Grid), P, ctypes.c_double, ctypes.POINTER(BC), ctypes.c_int64,
                               ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "lbm_server_run_bundle": ([P], ctypes.c_int),
        "lbm_server_poll": ([P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                             ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "lbm_server_fetch": ([P, ctypes.c_uint64, P, P], ctypes.c_int),
        "lbm_server_get_stats": ([P, ctypes.POINTER(ServerStats)], ctypes.c_int),
        "lbm_server_last_error": ([P], ctypes.c_char_p),
        "lbm_server_destroy": ([P], None),
        "lbm3_create": ([ctypes.POINTER(Grid3), ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(BC3), P,
                         ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
        "lbm3_step": ([P, ctypes.c_int64], ctypes.c_int),
        "lbm3_macros": ([P, P, P, ctypes.c_int], ctypes.c_int),
        "lbm3_get_populations": ([P, P, ctypes.c_int], ctypes.c_int),
        "lbm3_set_state": ([P, P, ctypes.c_int], ctypes.c_int),
        "lbm3_diag": ([P, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "lbm3_sync": ([P], ctypes.c_int),
        "lbm3_last_error": ([P], ctypes.c_char_p),
        "lbm3_destroy": ([P], None),
        "lbm3_bytes_per_update": ([ctypes.c_int32], ctypes.c_int32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible: the lattice update runs only on the GPU")
    return torch


@dataclass
class Config:
    scheme: str = "NPTL"
    layout: str = "stream"
    precision: str = "fp32"
    tile: tuple = (0, 0)


class Simulation:
    """One lattice Boltzmann simulation owned by the HIP library."""

    def __init__(self, flags, tau, x_axis=PERIODIC, y_axis=PERIODIC, u_in=(0.0, 0.0), g=(0.0, 0.0),
                 u0=(0.0, 0.0), scheme="NPTL", layout="stream", precision="fp32", tile=(0, 0), stream=None,
                 bundle=None, fullway=False):
        torch = _torch()
        self._lib = load_library()
        flags = np.ascontiguousarray(flags, dtype=np.uint8)
        self.ny, self.nx = flags.shape
        self.scheme, self.layout, self.precision = scheme, layout, precision
        grid = Grid(self.nx, self.ny, SCHEMES[scheme], LAYOUTS[layout], PRECISIONS[precision], int(tile[0]),
                    int(tile[1]))
        bc = BC(int(x_axis), int(y_axis), (ctypes.c_double * 2)(*u_in), (ctypes.c_double * 2)(*g), 1.0,
                (ctypes.c_double * 2)(*u0), FULLWAY if fullway else HALFWAY)
        if stream is None:
            # a stream of our own (default priority): never the legacy NULL stream
            stream = torch.cuda.Stream()
        self.stream = stream
        out = ctypes.c_void_p()
        st = self._lib.lbm_create(ctypes.byref(grid), flags.ctypes.data_as(ctypes.c_void_p), float(tau),
                                  ctypes.byref(bc), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(out))
        if st != OK:
            raise LbmError(st, self._lib.lbm_last_error(None).decode())
        self._ctx = out
        if bundle is not None:
            self._check(self._lib.lbm_set_bundle(self._ctx, int(bundle)))

    @classmethod
    def from_scenario(cls, sc, **kw):
        return cls(sc.flags, sc.tau, sc.x_axis, sc.y_axis, sc.u_in, sc.g, sc.u0, **kw)

    # ------------------------------------------------------------------ util
    def _check(self, st):
        if st != OK:
            raise LbmError(st, self._lib.lbm_last_error(self._ctx).decode())
        return st

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.lbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------ API
    def step(self, n: int = 1) -> "Simulation":
        self._check(self._lib.lbm_step(self._ctx, int(n)))
        return self

    def sync(self):
        self._check(self._lib.lbm_sync(self._ctx))

    def set_bundle(self, k: int):
        self._check(self._lib.lbm_set_bundle(self._ctx, int(k)))

    def info(self) -> dict:
        i = Info()
        self._check(self._lib.lbm_get_info(self._ctx, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in Info._fields_}

    def macros(self, device: bool = False):
        """(rho (ny, nx), u (2, ny, nx)) as float32 numpy arrays, or torch
        tensors on the device when device=True (enqueued on the stream)."""
        if device:
            torch = _torch()
            with torch.cuda.stream(self.stream):  # allocate in the order of our stream
                rho = torch.empty((self.ny, self.nx), dtype=torch.float32, device="cuda")
                u = torch.empty((2, self.ny, self.nx), dtype=torch.float32, device="cuda")
            self._check(self._lib.lbm_macros(self._ctx, ctypes.c_void_p(rho.data_ptr()),
                                             ctypes.c_void_p(u.data_ptr()), 1))
            return rho, u
        rho = np.empty((self.ny, self.nx), np.float32)
        u = np.empty((2, self.ny, self.nx), np.float32)
        self._check(self._lib.lbm_macros(self._ctx, rho.ctypes.data_as(ctypes.c_void_p),
                                         u.ctypes.data_as(ctypes.c_void_p), 0))
        return rho, u

    def populations(self) -> np.ndarray:
        """Shifted incoming populations (9, ny, nx) float32."""
        f = np.empty((9, self.ny, self.nx), np.float32)
        self._check(self._lib.lbm_get_populations(self._ctx, f.ctypes.data_as(ctypes.c_void_p), 0))
        return f

    def set_state(self, f_post_shifted) -> None:
        """Load shifted post-collision values (9, ny, nx)."""
        f = np.ascontiguousarray(f_post_shifted, dtype=np.float32)
        assert f.shape == (9, self.ny, self.nx)
        self._check(self._lib.lbm_set_state(self._ctx, f.ctypes.data_as(ctypes.c_void_p), 0))

    def diag(self):
        """(status, [mass, mom_x, mom_y, residual]) in FP64."""
        out = (ctypes.c_double * 4)()
        st = self._lib.lbm_diag(self._ctx, out)
        if st not in (OK, EUNSTABLE):
            self._check(st)
        return st, list(out)


class Simulation3:
    """One D3Q19 simulation owned by the HIP library (schemes NPTL and AA,
    layouts stream and collision).  Arrays are (nz, ny, nx) per component."""

    def __init__(self, flags, tau, x_axis=PERIODIC, y_axis=PERIODIC, z_axis=PERIODIC, u_in=(0.0, 0.0, 0.0),
                 g=(0.0, 0.0, 0.0), u0=(0.0, 0.0, 0.0), scheme="NPTL", layout="stream", precision="fp32",
                 tile=(0, 0), stream=None):
        torch = _torch()
        self._lib = load_library()
        flags = np.ascontiguousarray(flags, dtype=np.uint8)
        self.nz, self.ny, self.nx = flags.shape
        self.scheme, self.layout, self.precision = scheme, layout, precision
        grid = Grid3(self.nx, self.ny, self.nz, SCHEMES[scheme], LAYOUTS[layout], PRECISIONS[precision],
                     int(tile[0]), int(tile[1]))
        bc = BC3(int(x_axis), int(y_axis), int(z_axis), (ctypes.c_double * 3)(*u_in), (ctypes.c_double * 3)(*g),
                 1.0, (ctypes.c_double * 3)(*u0))
        self.stream = stream if stream is not None else torch.cuda.Stream()
        out = ctypes.c_void_p()
        st = self._lib.lbm3_create(ctypes.byref(grid), flags.ctypes.data_as(ctypes.c_void_p), float(tau),
                                   ctypes.byref(bc), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(out))
        if st != OK:
            raise LbmError(st, self._lib.lbm3_last_error(None).decode())
        self._ctx = out

    @classmethod
    def from_scenario(cls, sc, **kw):
        return cls(sc.flags, sc.tau, sc.x_axis, sc.y_axis, sc.z_axis, sc.u_in, sc.g, sc.u0, **kw)

    def _check(self, st):
        if st != OK:
            raise LbmError(st, self._lib.lbm3_last_error(self._ctx).decode())
        return st

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.lbm3_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def step(self, n: int = 1) -> "Simulation3":
        self._check(self._lib.lbm3_step(self._ctx, int(n)))
        return self

    def sync(self):
        self._check(self._lib.lbm3_sync(self._ctx))

    def macros(self, device: bool = False):
        """(rho (nz, ny, nx), u (3, nz, ny, nx)) float32 numpy arrays, or torch
        tensors on the device when device=True (enqueued on the stream)."""
        if device:
            torch = _torch()
            with torch.cuda.stream(self.stream):
                rho = torch.empty((self.nz, self.ny, self.nx), dtype=torch.float32, device="cuda")
                u = torch.empty((3, self.nz, self.ny, self.nx), dtype=torch.float32, device="cuda")
            self._check(self._lib.lbm3_macros(self._ctx, ctypes.c_void_p(rho.data_ptr()),
                                              ctypes.c_void_p(u.data_ptr()), 1))
            return rho, u
        rho = np.empty((self.nz, self.ny, self.nx), np.float32)
        u = np.empty((3, self.nz, self.ny, self.nx), np.float32)
        self._check(self._lib.lbm3_macros(self._ctx, rho.ctypes.data_as(ctypes.c_void_p),
                                          u.ctypes.data_as(ctypes.c_void_p), 0))
        return rho, u

    def populations(self) -> np.ndarray:
        """Shifted incoming populations (19, nz, ny, nx) float32."""
        f = np.empty((19, self.nz, self.ny, self.nx), np.float32)
        self._check(self._lib.lbm3_get_populations(self._ctx, f.ctypes.data_as(ctypes.c_void_p), 0))
        return f

    def diag(self):
        """(status, [mass, mom_x, mom_y, mom_z, residual]) in FP64."""
        out = (ctypes.c_double * 5)()
        st = self._lib.lbm3_diag(self._ctx, out)
        if st not in (OK, EUNSTABLE):
            self._check(st)
        return st, list(out)

    def set_state(self, f_post_shifted) -> None:
        """Load shifted post-collision values (19, nz, ny, nx)."""
        f = np.ascontiguousarray(f_post_shifted, dtype=np.float32)
        assert f.shape == (19, self.nz, self.ny, self.nx)
        self._check(self._lib.lbm3_set_state(self._ctx, f.ctypes.data_as(ctypes.c_void_p), 0))


def bytes_per_update(precision: str) -> int:
    return int(load_library().lbm_bytes_per_update(PRECISIONS[precision]))


def bandwidth_probe(mode: str, nbytes: int, reps: int = 5, stream=None):
    """Practical HBM bandwidth (GB/s, median of reps) of a plain copy / read /
    write kernel over nbytes (copy moves 2 * nbytes); "copy_nt" is the copy
    with non-temporal accesses and more bytes in flight."""
    torch = _torch()
    lib = load_library()
    m = {"copy": 0, "read": 1, "write": 2, "copy_nt": 3}[mode]
    nbytes = nbytes // 16 * 16
    stream = stream or torch.cuda.Stream()
    with torch.cuda.stream(stream):
        a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        a.zero_()
        b = torch.empty(nbytes if m in (0, 3) else 16, dtype=torch.uint8, device="cuda")
    src = ctypes.c_void_p(a.data_ptr())
    dst = ctypes.c_void_p(b.data_ptr()) if m != 2 else ctypes.c_void_p(a.data_ptr())
    if m == 2:
        src = ctypes.c_void_p(0)
    times = []
    for _ in range(reps + 1):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st = lib.lbm_bandwidth_probe(m, dst, src, nbytes, ctypes.c_void_p(stream.cuda_stream))
        e1.record(stream)
        e1.synchronize()
        if st != OK:
            raise LbmError(st, "bandwidth probe failed")
        times.append(e0.elapsed_time(e1))
    times = sorted(times[1:])
    moved = nbytes * (2 if m in (0, 3) else 1)
    return moved / (times[len(times) // 2] * 1e-3) / 1e9


class Server:
    """Continuous-batching engine: many independent simulations on one GPU."""

    def __init__(self, hbm_budget: int, max_slots: int = 512, bundle_steps: int = 50, layout: str = "stream",
                 precision: str = "fp32", stream=None):
        torch = _torch()
        self._lib = load_library()
        self.stream = stream or torch.cuda.Stream()
        out = ctypes.c_void_p()
        st = self._lib.lbm_server_create(int(hbm_budget), int(max_slots), int(bundle_steps), LAYOUTS[layout],
                                         PRECISIONS[precision], ctypes.c_void_p(self.stream.cuda_stream),
                                         ctypes.byref(out))
        if st != OK:
            raise LbmError(st, self._lib.lbm_server_last_error(None).decode())
        self._srv = out
        self._shape = {}
        self.layout, self.precision, self.bundle_steps = layout, precision, bundle_steps
        self._ids = (ctypes.c_uint64 * 4096)()
        self._sts = (ctypes.c_int32 * 4096)()

    def _check(self, st):
        if st != OK:
            raise LbmError(st, self._lib.lbm_server_last_error(self._srv).decode())
        return st

    def submit(self, flags, tau, x_axis=PERIODIC, y_axis=PERIODIC, u_in=(0.0, 0.0), g=(0.0, 0.0), u0=(0.0, 0.0),
               steps=100) -> int:
        flags = np.ascontiguousarray(flags, dtype=np.uint8)
        ny, nx = flags.shape
        grid = Grid(nx, ny, SCHEMES["NPTL"], 0, 0, 0, 0)
        bc = BC(int(x_axis), int(y_axis), (ctypes.c_double * 2)(*u_in), (ctypes.c_double * 2)(*g), 1.0,
                (ctypes.c_double * 2)(*u0))
        rid = ctypes.c_uint64()
        self._check(self._lib.lbm_server_submit(self._srv, ctypes.byref(grid), flags.ctypes.data_as(ctypes.c_void_p),
                                                float(tau), ctypes.byref(bc), int(steps), ctypes.byref(rid)))
        self._shape[rid.value] = (ny, nx)
        return rid.value

    def submit_scenario(self, sc, steps=None) -> int:
        return self.submit(sc.flags, sc.tau, sc.x_axis, sc.y_axis, sc.u_in, sc.g, sc.u0,
                           sc.steps if steps is None else steps)

    def run_bundle(self):
        self._check(self._lib.lbm_server_run_bundle(self._srv))

    def poll(self):
        """[(id, status)] of requests finished since the last poll (non-blocking)."""
        n = ctypes.c_int32()
        self._check(self._lib.lbm_server_poll(self._srv, self._ids, self._sts, 4096, ctypes.byref(n)))
        return [(int(self._ids[k]), int(self._sts[k])) for k in range(n.value)]

    def fetch(self, rid: int):
        """(status, rho (ny, nx), u (2, ny, nx)) of a finished request."""
        ny, nx = self._shape.pop(rid)
        rho = np.empty((ny, nx), np.float32)
        u = np.empty((2, ny, nx), np.float32)
        st = self._lib.lbm_server_fetch(self._srv, ctypes.c_uint64(rid), rho.ctypes.data_as(ctypes.c_void_p),
                                        u.ctypes.data_as(ctypes.c_void_p))
        if st not in (OK, EUNSTABLE):
            self._check(st)
        return st, rho, u

    def stats(self) -> dict:
        s = ServerStats()
        self._check(self._lib.lbm_server_get_stats(self._srv, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_srv", None):
            self._lib.lbm_server_destroy(self._srv)
            self._srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
