"""Plain FP64 CPU oracle for PDF / alpha_s interpolation (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does, and the
two share no code: this wraps ``oracle.c`` (plain C, FP64, libm) through ctypes.

Functions follow the paper's section 2.2 (PDF evaluation procedure), figure 1
(INTERPOLATE / EXTRAPOLATE) and section 2.3 (alpha_s evaluation procedure); see
the header of ``oracle.c`` for the readings taken where the paper is silent.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

REG_LOWX, REG_LOWQ, REG_HIGHQ, REG_INVALID = 1, 2, 4, 8


def build(force=False):
    """Compile oracle.c with gcc (FP64, no contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_xfxq2.argtypes = [ctypes.c_int32, P, ctypes.c_int32, P, P, P, ctypes.c_int32, P,
                                     P, P, ctypes.c_int64, P, P, ctypes.c_int32]
        lib.oracle_xfxq2.restype = ctypes.c_int
        lib.oracle_locate.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int64, P, P, P, P]
        lib.oracle_locate.restype = ctypes.c_int
        lib.oracle_alphas_q2.argtypes = [ctypes.c_int32, P, P, P, ctypes.c_int64, P]
        lib.oracle_alphas_q2.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Grid:
    """One member: K sub-grids in Q^2 order, each with x knots, Q^2 knots and
    values[ix][iq][column]; ``pids`` maps column -> PDG id."""

    def __init__(self, xknots, q2knots, values, pids):
        assert len(xknots) == len(q2knots) == len(values)
        self.K = len(xknots)
        self.pids = np.ascontiguousarray(pids, dtype=np.int32)
        self.shape = np.array([[len(xk), len(qk)] for xk, qk in zip(xknots, q2knots)], dtype=np.int32)
        self.knots = np.ascontiguousarray(np.concatenate(
            [np.concatenate([np.asarray(xk, np.float64), np.asarray(qk, np.float64)])
             for xk, qk in zip(xknots, q2knots)]))
        for k, v in enumerate(values):
            assert v.shape == (len(xknots[k]), len(q2knots[k]), len(self.pids)), v.shape
        self.values = np.ascontiguousarray(np.concatenate([np.asarray(v, np.float64).ravel() for v in values]))
        self.xknots = [np.asarray(x, np.float64) for x in xknots]
        self.q2knots = [np.asarray(q, np.float64) for q in q2knots]
        self.vals = [np.asarray(v, np.float64) for v in values]


def xfxq2(grid, pids, x, q2, n_threads=1, with_scale=False):
    """x*f at (x[i], q2[i]) for each requested pid; returns [n][len(pids)]
    (and the per-value error scale if ``with_scale``)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    q2 = np.ascontiguousarray(q2, dtype=np.float64)
    req = np.ascontiguousarray(pids, dtype=np.int32)
    n = x.shape[0]
    out = np.empty((n, len(req)), np.float64)
    scale = np.empty((n, len(req)), np.float64) if with_scale else None
    rc = lib.oracle_xfxq2(grid.K, _p(grid.shape), len(grid.pids), _p(grid.pids), _p(grid.knots),
                          _p(grid.values), len(req), _p(req), _p(x), _p(q2), n, _p(out),
                          _p(scale) if with_scale else None, int(n_threads))
    if rc != 0:
        raise ValueError("oracle_xfxq2 failed with code %d" % rc)
    return (out, scale) if with_scale else out


def locate(grid, x, q2):
    """(k, ix, iq, region) per query; region bits 1 low-x, 2 low-Q^2,
    4 high-Q^2, 8 invalid."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    q2 = np.ascontiguousarray(q2, dtype=np.float64)
    n = x.shape[0]
    k = np.empty(n, np.int32)
    ix = np.empty(n, np.int32)
    iq = np.empty(n, np.int32)
    reg = np.empty(n, np.int8)
    rc = lib.oracle_locate(grid.K, _p(grid.shape), _p(grid.knots), _p(x), _p(q2), n,
                           _p(k), _p(ix), _p(iq), _p(reg))
    if rc != 0:
        raise ValueError("oracle_locate failed with code %d" % rc)
    return k, ix, iq, reg


def alphas_q2(q2knots, alphas, q2):
    """alpha_s at each Q^2 (section 2.3)."""
    lib = _load()
    qk = np.ascontiguousarray(q2knots, dtype=np.float64)
    a = np.ascontiguousarray(alphas, dtype=np.float64)
    q2 = np.ascontiguousarray(q2, dtype=np.float64)
    out = np.empty(q2.shape[0], np.float64)
    rc = lib.oracle_alphas_q2(len(qk), _p(qk), _p(a), _p(q2), q2.shape[0], _p(out))
    if rc != 0:
        raise ValueError("oracle_alphas_q2 failed with code %d" % rc)
    return out
