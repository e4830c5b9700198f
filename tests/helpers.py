"""Shared test helpers: oracle comparison metrics and GPU availability."""
from __future__ import annotations

import numpy as np

import oracle

ALL_SCHEMES = ["LPTL", "NPTL", "PUSH", "NPOL", "NSOL", "AA"]
ALL_LAYOUTS = ["stream", "bundle", "collision"]
ALL_PRECISIONS = ["fp32", "fp16s", "fp16sr"]


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
