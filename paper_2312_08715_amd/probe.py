"""Peak microbenchmarks (libb3d_probe.so, declared in include/b3d_probe.h):
measured FP32 FMA, HBM and LDS rates of the device, for the benchmark's
roofline lines.  Not part of the method; the library is separate from
libb3d.so."""

from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from . import B3DError, LIB_DIR, _ptr, _stream

PROBE_LIB_PATH = os.path.join(LIB_DIR, "libb3d_probe.so")
_plib = None


def load_probe_library(path: str = PROBE_LIB_PATH) -> ctypes.CDLL:
    global _plib
    if _plib is None:
        if not os.path.exists(path):
            raise B3DError(f"{path} is missing: build it with python -m paper_2312_08715_amd.build")
        L = ctypes.CDLL(path)
        P, I32 = ctypes.c_void_p, ctypes.c_int32
        L.b3d_probe_fma.argtypes = [P, I32, I32, P]
        L.b3d_probe_hbm.argtypes = [P, P, P, ctypes.c_int64, P]
        L.b3d_probe_lds.argtypes = [P, I32, I32, P]
        for f in (L.b3d_probe_fma, L.b3d_probe_hbm, L.b3d_probe_lds):
            f.restype = I32
        _plib = L
    return _plib


def _pcall(name: str, *args) -> None:
    rc = getattr(load_probe_library(), name)(*args)
    if rc != 0:
        raise B3DError(f"{name} failed (status {rc})")


def probe_fma(blocks: int = 4096, iters: int = 256) -> float:
    """Measured FP32 vector FMA rate in lane-FMAs/s (one FMA = 2 flops)."""
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    _pcall("b3d_probe_fma", _ptr(out), blocks, iters, _stream())  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    _pcall("b3d_probe_fma", _ptr(out), blocks, iters, _stream())
    e1.record(st)
    e1.synchronize()
    return blocks * 256.0 * iters * 128.0 / (e0.elapsed_time(e1) / 1e3)


def probe_hbm(n_floats: int = 1 << 28, reps: int = 5) -> float:
    """Measured HBM bandwidth in bytes/s: median of `reps` triads over three
    n_floats buffers (3 GiB at the default)."""
    a = torch.ones(n_floats, dtype=torch.float32, device="cuda")
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    st = torch.cuda.current_stream()
    _pcall("b3d_probe_hbm", _ptr(a), _ptr(b), _ptr(c), n_floats, _stream())  # warm-up
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        _pcall("b3d_probe_hbm", _ptr(a), _ptr(b), _ptr(c), n_floats, _stream())
        e1.record(st)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    return 12.0 * n_floats / float(np.median(ts))


def probe_lds(blocks: int = 4096, iters: int = 256) -> float:
    """Measured LDS read bandwidth in bytes/s over the whole chip."""
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    _pcall("b3d_probe_lds", _ptr(out), blocks, iters, _stream())  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    _pcall("b3d_probe_lds", _ptr(out), blocks, iters, _stream())
    e1.record(st)
    e1.synchronize()
    return blocks * 256.0 * iters * 32.0 * 16.0 / (e0.elapsed_time(e1) / 1e3)
