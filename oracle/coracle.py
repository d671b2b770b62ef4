"""ctypes wrapper of the C++ oracle (oracle/liboracle.so, built from
oracle/c/sipg_oracle.cpp by oracle/c/build_oracle.py) — TEST INFRASTRUCTURE
ONLY: the same definitions as oracle/sipg.py and oracle/mg.py (uniform
meshes, GLL nodes, V(nu_pre, nu_post) with p halved to Q1 and Q1 coarsened
by 2, FP64 flexible CG), in plain C++ with OpenMP, for the timed CPU baseline
and as a second, independently written oracle checked against the first
(tests/test_oracle_cpp.py)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            from .c.build_oracle import build
            build()
        lib = ctypes.CDLL(LIB)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
        lib.oc_create.argtypes = [ip, ip, ip, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ip, ip, ip]
        lib.oc_create.restype = vp
        lib.oc_destroy.argtypes = [vp]
        lib.oc_ndof.argtypes = [vp]
        lib.oc_ndof.restype = ctypes.c_longlong
        lib.oc_nnz.argtypes = [vp]
        lib.oc_nnz.restype = ctypes.c_longlong
        lib.oc_csr.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_int), dp]
        lib.oc_apply.argtypes = [vp, dp, dp]
        lib.oc_smooth.argtypes = [vp, dp, dp, ip]
        lib.oc_vcycle.argtypes = [vp, dp, dp]
        lib.oc_solve.argtypes = [vp, dp, dp, ctypes.c_double, ip, dp]
        lib.oc_solve.restype = ip
        lib.oc_threads.restype = ip
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class CHierarchy:
    """SIPG hierarchy of the C++ oracle on the uniform n^dim mesh."""

    def __init__(self, dim, n, p, kappa=None, sigma0=2.0, omega_dg=0.7, omega_cg=2.0 / 3.0, nu_pre=2,
                 nu_post=2, coarsest_n=4):
        lib = _load()
        self._kap = None
        kp, kc = None, 1.0
        if kappa is not None and np.ndim(kappa) > 0:
            self._kap = np.ascontiguousarray(np.asarray(kappa, dtype=np.float64))
            kp = _dp(self._kap)
        elif kappa is not None:
            kc = float(kappa)
        self._h = lib.oc_create(dim, n, p, kp, kc, sigma0, omega_dg, omega_cg, nu_pre, nu_post, coarsest_n)
        if not self._h:
            raise ValueError("a cell block or the coarsest operator is not positive definite")
        self.ndof = int(lib.oc_ndof(self._h))

    def __del__(self):
        if getattr(self, "_h", None):
            _load().oc_destroy(self._h)
            self._h = None

    def csr(self):
        import scipy.sparse as sp
        lib = _load()
        nnz = int(lib.oc_nnz(self._h))
        ptr = np.empty(self.ndof + 1, dtype=np.int64)
        col = np.empty(nnz, dtype=np.int32)
        val = np.empty(nnz)
        lib.oc_csr(self._h, ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                   col.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(val))
        return sp.csr_matrix((val, col, ptr), shape=(self.ndof, self.ndof))

    def apply(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        y = np.empty_like(u)
        _load().oc_apply(self._h, _dp(u), _dp(y))
        return y

    def smooth(self, u, b, nsweeps):
        u = np.array(u, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        _load().oc_smooth(self._h, _dp(u), _dp(b), nsweeps)
        return u

    def vcycle(self, u, b):
        u = np.array(u, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        _load().oc_vcycle(self._h, _dp(u), _dp(b))
        return u

    def solve(self, b, rtol=1e-10, maxit=200):
        b = np.ascontiguousarray(b, dtype=np.float64)
        u = np.zeros_like(b)
        hist = np.zeros(maxit + 1)
        its = _load().oc_solve(self._h, _dp(u), _dp(b), rtol, maxit, _dp(hist))
        return u, list(hist[:its + 1])


def threads() -> int:
    return int(_load().oc_threads())
