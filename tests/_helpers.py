"""Shared helpers of the GPU tests (parity metrics, device tensors, caching)."""
from __future__ import annotations

import functools
import sys

import numpy as np

import synth


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(B, ref):
    """max over (output set, channel) of ||B - ref||_inf / ||ref||_inf."""
    B = np.asarray(B, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    num = np.abs(B - ref).max(axis=1)
    den = np.abs(ref).max(axis=1)
    return float((num / den).max())


def elementwise(B, ref, floor=1e-3):
    """max relative error over entries with |ref| >= floor * ||ref||_inf."""
    B = np.asarray(B, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    mask = np.abs(ref) >= floor * scale
    return float((np.abs(B - ref)[mask] / np.abs(ref)[mask]).max())


def dev_tensor(a, dtype_name):
    import torch
    dt = {"f64": torch.float64, "f32": torch.float32}[dtype_name]
    return torch.tensor(np.asarray(a), dtype=dt, device="cuda:0").contiguous()


@functools.lru_cache(maxsize=None)
def oracle_scene(w: synth.Workload):
    from oracle.transport import Scene
    return Scene(w)


def light_dtype(w):
    return "f64" if w.storage == "f64" else "f32"
