"""ctypes access to the compiled twins of the genotype generator.

libpqrgen_host.so   OpenMP host twin (column-major int8 dosages)
libpqrgen_device.so HIP device twin (writes straight into device memory)
Both are built from datagen/csrc by the package build step.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_host = None
_dev = None


def host_lib():
    global _host
    if _host is None:
        path = os.path.join(_HERE, "libpqrgen_host.so")
        if not os.path.exists(path):
            return None
        lib = ctypes.CDLL(path)
        lib.pqrgen_genotype_i8_host.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32]
        lib.pqrgen_genotype_i8_host.restype = None
        lib.pqrgen_philox4x32.argtypes = [ctypes.c_void_p] * 3
        lib.pqrgen_philox4x32.restype = None
        _host = lib
    return _host


def device_lib():
    global _dev
    if _dev is None:
        path = os.path.join(_HERE, "libpqrgen_device.so")
        if not os.path.exists(path):
            raise RuntimeError(f"device generator not built: {path}")
        lib = ctypes.CDLL(path)
        lib.pqrgen_genotype_i8_device.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
        lib.pqrgen_genotype_i8_device.restype = ctypes.c_int
        _dev = lib
    return _dev


def genotype_host(n, p, thr, seed, tag, j0=0, out=None):
    """Column-major (Fortran-order) int8 dosages for columns j0 .. j0+p-1."""
    lib = host_lib()
    if lib is None:
        raise RuntimeError("host generator not built")
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    assert thr.shape[0] == p
    if out is None:
        out = np.empty((n, p), dtype=np.int8, order="F")
    assert out.flags.f_contiguous and out.shape == (n, p)
    lib.pqrgen_genotype_i8_host(out.ctypes.data, n, n, j0, p, thr.ctypes.data, seed, tag)
    return out


def genotype_device(out_ptr, n, ld, p, thr_dev_ptr, seed, tag, stream=0, j0=0):
    """Fill device memory (column-major, leading dimension ld bytes) with dosages."""
    rc = device_lib().pqrgen_genotype_i8_device(out_ptr, n, ld, j0, p, thr_dev_ptr, seed, tag,
                                               stream)
    if rc != 0:
        raise RuntimeError(f"pqrgen_genotype_i8_device failed ({rc})")
