"""Measured hardware ceilings (include/hipsso_ceiling.h): the HBM bandwidth a streaming read and
a streaming copy of the library's own reach, and the FP64 vector FMA rate.  Marshalling only."""
from __future__ import annotations

import ctypes

import torch

from . import load_library

_vp = ctypes.c_void_p
EXPORTS = ("hipsso_ceiling_read", "hipsso_ceiling_copy", "hipsso_ceiling_fma")


def _lib():
    lib = load_library()
    if not getattr(lib, "_ceiling_declared", False):
        P = ctypes.POINTER
        lib.hipsso_ceiling_read.argtypes = [_vp, ctypes.c_int64, _vp, ctypes.c_int, _vp,
                                            P(ctypes.c_double)]
        lib.hipsso_ceiling_copy.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int, _vp,
                                            P(ctypes.c_double)]
        lib.hipsso_ceiling_fma.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp,
                                           P(ctypes.c_double)]
        for n in EXPORTS:
            getattr(lib, n).restype = ctypes.c_int
        lib._ceiling_declared = True
    return lib


def measure(mib: int = 2048, reps: int = 10, fma_workgroups: int = 8192,
            fma_iters: int = 4096) -> dict:
    """Read and copy bandwidth (GB/s, bytes moved / launch time) over a buffer of `mib` MiB and
    the FP64 FMA rate (TFLOP/s), on torch's current stream."""
    lib = _lib()
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    part = torch.zeros(max(8192, fma_workgroups), dtype=torch.float64, device="cuda")
    s = _vp(torch.cuda.current_stream().cuda_stream)
    us = ctypes.c_double()
    out = {}
    if lib.hipsso_ceiling_read(_vp(src.data_ptr()), n, _vp(part.data_ptr()), reps, s,
                               ctypes.byref(us)) != 0:
        raise RuntimeError("hipsso_ceiling_read failed")
    out["read_gbs"] = 8.0 * n / (us.value * 1e-6) / 1e9
    if lib.hipsso_ceiling_copy(_vp(src.data_ptr()), _vp(dst.data_ptr()), n, reps, s,
                               ctypes.byref(us)) != 0:
        raise RuntimeError("hipsso_ceiling_copy failed")
    out["copy_gbs"] = 16.0 * n / (us.value * 1e-6) / 1e9
    if lib.hipsso_ceiling_fma(_vp(part.data_ptr()), fma_workgroups, fma_iters, reps, s,
                              ctypes.byref(us)) != 0:
        raise RuntimeError("hipsso_ceiling_fma failed")
    out["fp64_fma_tflops"] = 16.0 * 256 * fma_workgroups * fma_iters / (us.value * 1e-6) / 1e12
    out["buffer_mib"] = mib
    del src, dst, part
    torch.cuda.empty_cache()
    return out
