"""ctypes wrapper of the oracle's C direct-summation core (test infrastructure).

``build()`` compiles direct_core.c with gcc (OpenMP) into _direct_core.so next to
this file; the wrapper loads it lazily and builds it on first use if missing.
"""
import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct_core.c")
_LIB = os.path.join(_HERE, "_direct_core.so")
_lib = None


def build(force=True):
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_conv_add.argtypes = [P] * 9
        lib.oracle_conv_add.restype = None
        lib.oracle_corr.argtypes = [P] * 8
        lib.oracle_corr.restype = None
        _lib = lib
    return _lib


def _pad3(v, fill):
    v = [int(x) for x in np.asarray(v).ravel()]
    return np.array(v + [fill] * (3 - len(v)), dtype=np.int64)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def conv_add(t, tlo, K, zlo, out, olo=None):
    """out += (K * t) restricted to a window of the domain: out is the window
    starting at Omega point olo (default: the origin, out = the whole
    domain); FP64, in place."""
    lib = _load()
    t = np.ascontiguousarray(t, dtype=np.float64)
    K = np.ascontiguousarray(K, dtype=np.float64)
    assert out.dtype == np.float64 and out.flags.c_contiguous
    olo = np.zeros(out.ndim, dtype=np.int64) if olo is None else olo
    a = [_pad3(tlo, 0), _pad3(t.shape, 1), _pad3(zlo, 0), _pad3(K.shape, 1), _pad3(olo, 0), _pad3(out.shape, 1)]
    lib.oracle_conv_add(_p(t), _p(a[0]), _p(a[1]), _p(K), _p(a[2]), _p(a[3]), _p(out), _p(a[4]), _p(a[5]))


def corr(g, tlo, m, K, zlo):
    """c[x] = sum_z K[z] g[x + z] for x in the box at tlo of extent m."""
    lib = _load()
    g = np.ascontiguousarray(g, dtype=np.float64)
    K = np.ascontiguousarray(K, dtype=np.float64)
    c = np.zeros(tuple(int(v) for v in m))
    a = [_pad3(g.shape, 1), _pad3(zlo, 0), _pad3(K.shape, 1), _pad3(tlo, 0), _pad3(m, 1)]
    lib.oracle_corr(_p(g), _p(a[0]), _p(K), _p(a[1]), _p(a[2]), _p(c), _p(a[3]), _p(a[4]))
    return c
