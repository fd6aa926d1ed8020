"""ctypes wrapper of oracle/cmatvec.c (plain C OpenMP FP64 kernel product).

TEST INFRASTRUCTURE ONLY.  The shared object is built next to the source by
`build_oracle()` (called from the package build step) with gcc -O3 -fopenmp.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cmatvec.c")
_SO = os.path.join(_HERE, "libkaoracle.so")
_lib = None

KERNEL_IDS = {"gaussian": 0, "exponential": 1}


def build_oracle():
    cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _SO, "-lm"]
    subprocess.check_call(cmd)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build_oracle()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.ka_oracle_gamma_apply.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                              dp, ctypes.c_long, dp, ctypes.c_long, dp, ctypes.c_int,
                                              dp, dp, dp, ctypes.c_int]
        lib.ka_oracle_gamma_apply.restype = None
        lib.ka_oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def max_threads():
    return _load().ka_oracle_max_threads()


def gamma_apply(kind, sigma, ell, Xr, Xc, Y, rs=None, cs=None, nthreads=0):
    """Z = diag(rs) Gamma(Xr, Xc) diag(cs) Y in FP64 on the host cores."""
    lib = _load()
    Xr = np.ascontiguousarray(Xr, dtype=np.float64)
    Xc = np.ascontiguousarray(Xc, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    vec = Y.ndim == 1
    if vec:
        Y = Y[:, None]
    b = Y.shape[1]
    Z = np.empty((Xr.shape[0], b))
    rs = None if rs is None else np.ascontiguousarray(rs, dtype=np.float64)
    cs = None if cs is None else np.ascontiguousarray(cs, dtype=np.float64)
    lib.ka_oracle_gamma_apply(KERNEL_IDS[kind], float(sigma), float(ell), _ptr(Xr), Xr.shape[0],
                              _ptr(Xc), Xc.shape[0], _ptr(Y), b, _ptr(Z), _ptr(rs), _ptr(cs),
                              int(nthreads))
    return Z[:, 0] if vec else Z
