"""Device memory and streams for the GPU tests, from the HIP runtime the
library itself links (libamdhip64.so.7 of /opt/rocm), through ctypes.

Test infrastructure: a caller's device allocation and stream handed to the
C-ABI.  torch on this image bundles its own ROCm runtime; a process can use
torch's device memory with the library only when torch's runtime starts first
(tests/test_gpu_runtime.py covers that in a child process), and torch's
stream handles belong to that other runtime, so the in-process tests take
memory and streams from here.
"""
import ctypes

import numpy as np

_hip = None


def hip():
    global _hip
    if _hip is None:
        from paper_2403_15773_amd import tslb
        tslb.load_library()  # the library's own runtime is then loaded; take the same one
        lib = ctypes.CDLL("libamdhip64.so.7")
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        lib.hipMalloc.argtypes = [ctypes.POINTER(vp), sz]
        lib.hipFree.argtypes = [vp]
        lib.hipMemcpy.argtypes = [vp, vp, sz, ctypes.c_int]
        lib.hipMemset.argtypes = [vp, ctypes.c_int, sz]
        lib.hipStreamCreate.argtypes = [ctypes.POINTER(vp)]
        lib.hipStreamDestroy.argtypes = [vp]
        lib.hipStreamSynchronize.argtypes = [vp]
        lib.hipDeviceSynchronize.argtypes = []
        for f in ("hipMalloc", "hipFree", "hipMemcpy", "hipMemset", "hipStreamCreate", "hipStreamDestroy",
                  "hipStreamSynchronize", "hipDeviceSynchronize"):
            getattr(lib, f).restype = ctypes.c_int
        _hip = lib
    return _hip


def _ok(rc, what):
    if rc != 0:
        raise RuntimeError("%s failed with hipError %d" % (what, rc))


H2D, D2H = 1, 2


class DeviceBuffer:
    """hipMalloc'ed bytes; .ptr is the device address."""

    def __init__(self, nbytes):
        self.nbytes = int(nbytes)
        p = ctypes.c_void_p()
        _ok(hip().hipMalloc(ctypes.byref(p), self.nbytes), "hipMalloc")
        self.ptr = p.value

    def upload(self, arr, offset=0):
        a = np.ascontiguousarray(arr)
        assert offset + a.nbytes <= self.nbytes
        _ok(hip().hipMemcpy(self.ptr + offset, a.ctypes.data, a.nbytes, H2D), "hipMemcpy H2D")

    def download(self, nbytes=None, offset=0, dtype=np.uint8):
        n = self.nbytes - offset if nbytes is None else int(nbytes)
        out = np.empty(n, np.uint8)
        _ok(hip().hipMemcpy(out.ctypes.data, self.ptr + offset, n, D2H), "hipMemcpy D2H")
        return out.view(dtype)

    def fill(self, byte, nbytes=None, offset=0):
        n = self.nbytes - offset if nbytes is None else int(nbytes)
        _ok(hip().hipMemset(self.ptr + offset, int(byte), n), "hipMemset")

    def free(self):
        if self.ptr:
            hip().hipFree(self.ptr)
            self.ptr = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.free()


class Stream:
    """A hipStream_t of the library's runtime; .handle is the pointer value."""

    def __init__(self):
        s = ctypes.c_void_p()
        _ok(hip().hipStreamCreate(ctypes.byref(s)), "hipStreamCreate")
        self.handle = s.value

    def synchronize(self):
        _ok(hip().hipStreamSynchronize(self.handle), "hipStreamSynchronize")

    def destroy(self):
        if self.handle:
            hip().hipStreamDestroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.destroy()


def device_synchronize():
    _ok(hip().hipDeviceSynchronize(), "hipDeviceSynchronize")
