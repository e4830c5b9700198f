"""Shared test helpers: oracle comparison metrics and GPU availability."""
from __future__ import annotations

import numpy as np

import oracle

ALL_SCHEMES = ["LPTL", "NPTL", "PUSH", "NPOL", "NSOL", "AA"]
ALL_LAYOUTS = ["stream", "bundle", "collision"]
ALL_PRECISIONS = ["fp32", "fp16s", "fp16sr", "fp16c", "fp16csr"]


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def updated_mask(types):
    return (types == oracle.FLUID) | (types == oracle.OUTLET)


def velocity_error(u_gpu, ux, uy, mask):
    """max |u_gpu - u_ora|_2 over mask, divided by max |u_ora|_2 over mask."""
    d = np.hypot(u_gpu[0].astype(np.float64) - ux, u_gpu[1].astype(np.float64) - uy)[mask]
    return float(d.max() / np.hypot(ux, uy)[mask].max())


def weights():
    return oracle.constants()[3]


def fp16_round(a):
    return np.asarray(a, dtype=np.float16).astype(np.float32)


# FP16C values (sign, 4 exponent bits, 11 fraction bits, bias 15; subnormal
# spacing 2^-25; top code NaN), computed from the values the format holds,
# not from its bit encoding.
FP16C_MAX = 2.0 ** 0 * (1 + 2046 / 2048)  # largest finite value
FP16C_NAN_FROM = (FP16C_MAX + 2.0 ** 0 * (1 + 2047 / 2048)) / 2  # above this, RNE gives the NaN code


def fp16c_spacing(v):
    """Spacing of the FP16C values around |v| (|v| < 2)."""
    a = np.abs(np.asarray(v, np.float64))
    _, ex = np.frexp(a)  # a = m 2^ex, m in [0.5, 1)
    e = np.maximum(ex - 1, -14)  # binade exponent; subnormals share the lowest spacing
    return np.ldexp(1.0, e - 11)


def fp16c_neighbours(v):
    """(toward zero, away from zero) FP16C neighbours of finite |v| < 2, and
    the index of the first in units of its spacing."""
    v = np.asarray(v, np.float64)
    s = fp16c_spacing(v)
    k = np.floor(np.abs(v) / s)
    lo = np.copysign(k * s, v)
    hi = np.copysign((k + 1) * s, v)
    return lo, hi, k


def fp16c_rne(v):
    """FP16C round to nearest, ties to even (NaN beyond the finite range)."""
    v = np.asarray(v, np.float64)
    out = np.full(v.shape, np.nan)
    ok = np.isfinite(v) & (np.abs(v) <= FP16C_NAN_FROM)
    w = v[ok]
    lo, hi, k = fp16c_neighbours(w)
    d = np.abs(w) - np.abs(lo)
    half = fp16c_spacing(w) / 2
    up = (d > half) | ((d == half) & (k % 2 == 1))
    out[ok] = np.where(up, hi, lo)
    return out


_REPORT = {}


def report(key, value):
    """Record a measured value; with LBM_REPORT=<path> set, all recorded
    values of the session are (re)written to that JSON file."""
    import json
    import os
    _REPORT[key] = value
    path = os.environ.get("LBM_REPORT")
    if path:
        with open(path, "w") as f:
            json.dump(_REPORT, f, indent=1, sort_keys=True)
