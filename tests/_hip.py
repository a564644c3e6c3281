"""Device buffers for GPU tests through the HIP runtime that liblbm2p.so
itself is linked against (looked up by its soname once the library is
loaded), so that tests need no second GPU runtime in the process."""
import ctypes as C

import numpy as np

_hip = None


def hip():
    global _hip
    if _hip is None:
        from paper_1908_09235_amd import lbm
        lbm.lib()  # the library brings its HIP runtime in first
        L = C.CDLL("libamdhip64.so.7")
        L.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        L.hipFree.argtypes = [C.c_void_p]
        L.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        L.hipDeviceSynchronize.argtypes = []
        for f in (L.hipMalloc, L.hipFree, L.hipMemcpy, L.hipDeviceSynchronize):
            f.restype = C.c_int
        _hip = L
    return _hip


H2D, D2H = 1, 2


class DeviceArray:
    """n doubles of device memory, filled from a host array."""

    def __init__(self, host):
        self.host = np.ascontiguousarray(host, dtype=np.float64)
        self.ptr = C.c_void_p()
        assert hip().hipMalloc(C.byref(self.ptr), self.host.nbytes) == 0
        assert hip().hipMemcpy(self.ptr, self.host.ctypes.data_as(C.c_void_p),
                               self.host.nbytes, H2D) == 0

    def get(self):
        out = np.empty_like(self.host)
        assert hip().hipDeviceSynchronize() == 0
        assert hip().hipMemcpy(out.ctypes.data_as(C.c_void_p), self.ptr, out.nbytes, D2H) == 0
        return out

    def free(self):
        if self.ptr:
            hip().hipFree(self.ptr)
            self.ptr = C.c_void_p()
