"""ctypes wrapper of the plain C CSR conjugate-gradient solver (csr_cg.c).

TEST INFRASTRUCTURE ONLY (see the package docstring)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(_HERE, "liboracle_cg.so")
SRC = os.path.join(_HERE, "csr_cg.c")


def build():
    """Compile the C solver with gcc (-O2 -fopenmp)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", LIB, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        head = [ctypes.c_int64] + [vp] * 8
        lib.oracle_csr_cg.restype = ctypes.c_int64
        lib.oracle_csr_cg.argtypes = head + [ctypes.c_double, ctypes.c_int64, dp]
        lib.oracle_csr_cg_fixed.restype = ctypes.c_int64
        lib.oracle_csr_cg_fixed.argtypes = head + [ctypes.c_int64, dp]
        lib.oracle_csr_cg_timed.restype = ctypes.c_int64
        lib.oracle_csr_cg_timed.argtypes = head + [ctypes.c_int64, dp]
        lib.oracle_structured_csr.restype = None
        lib.oracle_structured_csr.argtypes = [ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int] + [vp] * 8
        _lib = lib
    return _lib


def _prep(K):
    K = K.tocsr()
    ip = np.ascontiguousarray(K.indptr, dtype=np.int64)
    ix = np.ascontiguousarray(K.indices, dtype=np.int32)
    a = np.ascontiguousarray(K.data, dtype=np.float64)
    return ip, ix, a


def _ptr(x):
    return x.ctypes.data_as(ctypes.c_void_p)


def solve(K, f, tol=1e-13, maxit=1_000_000):
    """Returns (u, iterations, relres)."""
    lib = _load()
    ip, ix, a = _prep(K)
    n = K.shape[0]
    f = np.ascontiguousarray(f, dtype=np.float64)
    u, r, p, q = (np.empty(n) for _ in range(4))
    rel = ctypes.c_double(0.0)
    it = lib.oracle_csr_cg(n, _ptr(ip), _ptr(ix), _ptr(a), _ptr(f), _ptr(u), _ptr(r), _ptr(p),
                           _ptr(q), float(tol), int(maxit), ctypes.byref(rel))
    return u, int(it), rel.value


def run_fixed(K, f, iters):
    """Run exactly ``iters`` CG iterations (timing helper); returns u."""
    lib = _load()
    ip, ix, a = _prep(K)
    n = K.shape[0]
    f = np.ascontiguousarray(f, dtype=np.float64)
    u, r, p, q = (np.empty(n) for _ in range(4))
    rel = ctypes.c_double(0.0)
    lib.oracle_csr_cg_fixed(n, _ptr(ip), _ptr(ix), _ptr(a), _ptr(f), _ptr(u), _ptr(r), _ptr(p),
                            _ptr(q), int(iters), ctypes.byref(rel))
    return u


def run_timed(K, f, iters):
    """Run exactly ``iters`` CG iterations and return the wall time of each
    iteration (seconds, host clock around every iteration)."""
    lib = _load()
    ip, ix, a = _prep(K)
    n = K.shape[0]
    f = np.ascontiguousarray(f, dtype=np.float64)
    u, r, p, q = (np.empty(n) for _ in range(4))
    t = np.zeros(int(iters))
    lib.oracle_csr_cg_timed(n, _ptr(ip), _ptr(ix), _ptr(a), _ptr(f), _ptr(u), _ptr(r), _ptr(p),
                            _ptr(q), int(iters), t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return t


def structured_csr(shape, slot_off, t_slot, t_vc, t_A, t_B, lam, mu):
    """Indices and values of the node-neighbour CSR (see fe.assemble_structured)."""
    lib = _load()
    dim = len(shape)
    N = int(np.prod(shape))
    nb = len(slot_off)
    shp = np.ascontiguousarray(list(shape) + [1] * (3 - dim), dtype=np.int64)
    indices = np.empty(N * dim * nb * dim, dtype=np.int32)
    data = np.empty(N * dim * nb * dim)
    lib.oracle_structured_csr(dim, _ptr(shp), nb, _ptr(np.ascontiguousarray(slot_off)), len(t_slot),
                              _ptr(np.ascontiguousarray(t_slot)), _ptr(np.ascontiguousarray(t_vc)),
                              _ptr(t_A), _ptr(t_B), _ptr(lam), _ptr(mu), _ptr(indices), _ptr(data))
    return indices, data
