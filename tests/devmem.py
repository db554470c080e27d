"""Device buffers for GPU tests, through the HIP runtime the library itself uses (no torch):
ctypes opens libamdhip64.so.7 by its soname, which resolves to the copy already loaded in the
process as the library's dependency, so pointers and streams stay within one runtime."""
import ctypes

import numpy as np

from paper_1705_10045_amd import lbm

_HIP = None
_D2H = 2


def hip():
    global _HIP
    if _HIP is None:
        lbm.lib()   # load the library first: its runtime is the one to share
        h = ctypes.CDLL("libamdhip64.so.7")
        h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        h.hipFree.argtypes = [ctypes.c_void_p]
        h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        h.hipMemset.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t]
        h.hipDeviceSynchronize.argtypes = []
        _HIP = h
    return _HIP


class DeviceArray:
    """An FP64 device buffer of n values; `numpy()` copies it to the host (synchronous)."""

    def __init__(self, n, fill_byte=0xFF):
        self.n = int(n)
        self.ptr = ctypes.c_void_p()
        st = hip().hipMalloc(ctypes.byref(self.ptr), 8 * self.n)
        if st != 0:
            raise RuntimeError("hipMalloc failed (%d)" % st)
        # 0xFF bytes read back as NaN: anything the tested call leaves unwritten shows
        if hip().hipMemset(self.ptr, fill_byte, 8 * self.n) != 0:
            raise RuntimeError("hipMemset failed")

    def numpy(self):
        out = np.empty(self.n)
        if hip().hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), self.ptr, 8 * self.n, _D2H) != 0:
            raise RuntimeError("hipMemcpy failed")
        return out

    def free(self):
        if self.ptr:
            hip().hipFree(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
