"""Direct O(N^2) sums (the definition, eqn. HelmholtzMatrixVector) -- TEST INFRASTRUCTURE ONLY;
see oracle/__init__.py. The arithmetic is plain C + OpenMP in FP64 (oracle/direct.c); this module
builds it with gcc on first use and calls it through ctypes."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_LIB = os.path.join(_HERE, "_direct.so")
_lib = None


def build(force=False):
    """Compile oracle/direct.c with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        for name in ("oracle_direct_matvec", "oracle_direct_gradient"):
            f = getattr(lib, name)
            f.restype = None
            f.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                          ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def _prep(x, q, targets):
    x = np.ascontiguousarray(x, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.complex128)
    if targets is None:
        t = None
        nt = x.shape[0]
    else:
        t = np.ascontiguousarray(targets, dtype=np.int64)
        nt = t.shape[0]
    return x, q, t, nt


def matvec(x, q, kappa, targets=None):
    """sigma_i = sum_{j != i, R_ij > 0} e^{i kappa R_ij}/R_ij q_j for i in targets (all if None)."""
    lib = _load()
    x, q, t, nt = _prep(x, q, targets)
    out = np.empty(nt, dtype=np.complex128)
    lib.oracle_direct_matvec(x.shape[0], x.ctypes.data, q.ctypes.data, float(kappa), nt,
                             None if t is None else t.ctypes.data, out.ctypes.data)
    return out


def gradient(x, q, kappa, targets=None):
    """F_i = sum_{j != i, R_ij > 0} G'(R_ij) (x_i - x_j)/R_ij q_j, G'(R) = e^{i kappa R}(i kappa R - 1)/R^2.
    Returns complex [ntargets, 3]."""
    lib = _load()
    x, q, t, nt = _prep(x, q, targets)
    out = np.empty((nt, 3), dtype=np.complex128)
    lib.oracle_direct_gradient(x.shape[0], x.ctypes.data, q.ctypes.data, float(kappa), nt,
                               None if t is None else t.ctypes.data, out.ctypes.data)
    return out
