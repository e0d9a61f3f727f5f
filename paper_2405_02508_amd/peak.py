"""Binding of ``libmer_peak.so`` (include/mer_peak.h): the reference kernels
the benchmark measures its rooflines with -- a plain streaming copy and
device-scope float atomic adds.  Argument marshalling only; raises if the
library has not been built."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmer_peak.so")
SYMBOLS = ("mer_peak_copy", "mer_peak_atomic_add")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP libraries first (__graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, i, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        L.mer_peak_copy.argtypes = [P, P, i64, P]
        L.mer_peak_atomic_add.argtypes = [P, i64, i64, i, P]
        for n in SYMBOLS:
            getattr(L, n).restype = i
        _lib = L
    return _lib


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def copy(src, dst):
    """dst <- src (float32 CUDA tensors of equal size, a multiple of 4)."""
    rc = lib().mer_peak_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), src.numel(), _stream())
    if rc != 0:
        raise RuntimeError(f"mer_peak_copy failed ({rc})")


def atomic_add(buf, footprint, lanes, per_lane):
    """lanes * per_lane float atomic adds of 1 into buf[:footprint]."""
    if footprint > buf.numel():
        raise RuntimeError("footprint exceeds the buffer")
    rc = lib().mer_peak_atomic_add(ctypes.c_void_p(buf.data_ptr()), int(footprint), int(lanes), int(per_lane),
                                   _stream())
    if rc != 0:
        raise RuntimeError(f"mer_peak_atomic_add failed ({rc})")
