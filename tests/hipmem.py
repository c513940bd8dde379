"""Device buffers for the tests of the context-free entry points, through the
HIP runtime that librbsog itself is linked against (loaded by its soname, so
the process holds one runtime).  Test infrastructure only."""
from __future__ import annotations

import ctypes

import numpy as np

from paper_2205_13824_amd import rbsog as R

_hip = None
H2D, D2H = 1, 2


def hip():
    global _hip
    if _hip is None:
        R.lib()  # librbsog first: its runtime is the one every call below uses
        h = ctypes.CDLL("libamdhip64.so.7")
        h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        h.hipFree.argtypes = [ctypes.c_void_p]
        h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        h.hipDeviceSynchronize.argtypes = []
        for f in (h.hipMalloc, h.hipFree, h.hipMemcpy, h.hipDeviceSynchronize):
            f.restype = ctypes.c_int
        _hip = h
    return _hip


class DeviceArray:
    """A device copy of a numpy array (or uninitialised storage of a shape and dtype)."""

    def __init__(self, host=None, shape=None, dtype=None):
        if host is not None:
            host = np.ascontiguousarray(host)
            shape, dtype = host.shape, host.dtype
        self.shape, self.dtype = tuple(shape), np.dtype(dtype)
        self.nbytes = int(np.prod(self.shape)) * self.dtype.itemsize
        p = ctypes.c_void_p()
        assert hip().hipMalloc(ctypes.byref(p), max(self.nbytes, 8)) == 0, "hipMalloc failed"
        self.ptr = p.value
        if host is not None:
            assert hip().hipMemcpy(self.ptr, host.ctypes.data, self.nbytes, H2D) == 0

    def fill_from(self, host):
        host = np.ascontiguousarray(host, dtype=self.dtype).reshape(self.shape)
        assert hip().hipMemcpy(self.ptr, host.ctypes.data, self.nbytes, H2D) == 0

    def numpy(self):
        out = np.empty(self.shape, dtype=self.dtype)
        assert hip().hipDeviceSynchronize() == 0
        assert hip().hipMemcpy(out.ctypes.data, self.ptr, self.nbytes, D2H) == 0
        return out

    def free(self):
        if self.ptr:
            hip().hipFree(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def synchronize():
    assert hip().hipDeviceSynchronize() == 0
